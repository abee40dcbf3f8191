"""Local observables from the lattice Green's function (oracle; test only).

Paper: Sec. III.A.  The spin-sigma occupancy is -i G_loc(t, t + 0^+); on the
contour grid t + 0^+ is the backward point at the same physical time, so
n_i(t_a) = Re(-i G[(i,a), (i,b(a))]) = Im G[(i,a), (i,b(a))].  The kinetic
energy of site i is +i sum_{j NN of i} J(t) G(r_j, t; r_i, t), read at the same
pair of contour points.  Values are per spin; the paramagnetic total is twice.
"""
import numpy as np

from .contour import Contour


def occupancy(G_loc: np.ndarray, c: Contour) -> np.ndarray:
    """n[s, a] for a in [0, N_real) from per-source local blocks G_loc[s] (N_t x N_t)."""
    a = np.arange(c.n_real)
    return np.real(-1j * G_loc[:, a, c.partner(a)])


def kinetic_energy(G_nn: np.ndarray, nbr_of_src: np.ndarray, J_real: np.ndarray,
                   c: Contour) -> np.ndarray:
    """e_kin[s, a] from G_nn[s, d] = G(neighbour d of source s, source s) blocks."""
    a = np.arange(c.n_real)
    out = np.zeros((G_nn.shape[0], c.n_real), dtype=np.float64)
    for s in range(G_nn.shape[0]):
        acc = np.zeros(c.n_real, dtype=np.complex128)
        for d in range(4):
            if nbr_of_src[s, d] < 0:
                continue
            acc += np.asarray(J_real) * G_nn[s, d][a, c.partner(a)]
        out[s] = np.real(1j * acc)
    return out


def local_blocks_from_dense(G: np.ndarray, n_t: int, sites) -> np.ndarray:
    return np.stack([G[i * n_t:(i + 1) * n_t, i * n_t:(i + 1) * n_t] for i in sites])


def neighbour_blocks_from_dense(G: np.ndarray, n_t: int, nbr: np.ndarray, sites) -> np.ndarray:
    out = np.zeros((len(sites), 4, n_t, n_t), dtype=np.complex128)
    for s, j in enumerate(sites):
        for d in range(4):
            k = nbr[j, d]
            if k >= 0:
                out[s, d] = G[k * n_t:(k + 1) * n_t, j * n_t:(j + 1) * n_t]
    return out
