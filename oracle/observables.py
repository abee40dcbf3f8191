"""Local observables from the lattice Green's function (oracle; test only).

Paper: Sec. III.A.  The spin-sigma occupancy is -i G_loc(t, t + 0^+); on the
contour grid t + 0^+ is the backward point at the same physical time, so
n_i(t_a) = Re(-i G[(i,a), (i,b(a))]) = Im G[(i,a), (i,b(a))].  The kinetic
energy of site i is the expectation of its hopping terms, sum_j h_ij
<c_i^dag c_j>(t) = -i sum_j h_ij G(r_j, t; r_i, t^+), read at the same pair of
contour points.  The G solved here (eq. Glatt with +J, G = S + S D G) is the
propagator of hopping h_ij = +J (the U = 0 pin fixes this), the gauge image
c_i -> (-1)^(x+y) c_i of the Hamiltonian's -J c^dag c (eq. model); Sec. III.A
writes +i sum_j J G with the Hamiltonian's amplitude, so on this G the same
physical quantity is -i sum_j J G.  Values are per spin; the paramagnetic total
is twice.
"""
import numpy as np

from .contour import Contour


def occupancy(G_loc: np.ndarray, c: Contour) -> np.ndarray:
    """n[s, a] for a in [0, N_real) from per-source local blocks G_loc[s] (N_t x N_t)."""
    a = np.arange(c.n_real)
    return np.real(-1j * G_loc[:, a, c.partner(a)])


def kinetic_energy(G_nn: np.ndarray, nbr_of_src: np.ndarray, J_real: np.ndarray,
                   c: Contour) -> np.ndarray:
    """e_kin[s, a] = Re(-i J(t_a) sum_d G_nn[s, d][a, b(a)]) from the blocks
    G_nn[s, d] = G(neighbour d of source s, source s)."""
    a = np.arange(c.n_real)
    out = np.zeros((G_nn.shape[0], c.n_real), dtype=np.float64)
    for s in range(G_nn.shape[0]):
        acc = np.zeros(c.n_real, dtype=np.complex128)
        for d in range(4):
            if nbr_of_src[s, d] < 0:
                continue
            acc += np.asarray(J_real) * G_nn[s, d][a, c.partner(a)]
        out[s] = np.real(-1j * acc)
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


def double_occupancy(G_loc: np.ndarray, G_nn: np.ndarray, nbr_of_src: np.ndarray,
                     eps_src: np.ndarray, U_real: np.ndarray, J_real: np.ndarray,
                     c: Contour) -> np.ndarray:
    """D[s, a] = <n_up n_down>(t_a) of each source site from eq. docc:

        d/dt G_loc(t, t')|_{t' = t^+} = U(t) D(t) + eps n_sigma(t) + e_kin(t),

    the time derivative taken as App. B does, one-sided on the forward branch
    with t' = t^+ held at the backward point b(a) of the same time:
    (G[a, b(a)] - G[a-1, b(a)]) / dt for a >= 1, and the forward difference
    (G[1, b(0)] - G[0, b(0)]) / dt at a = 0.  The real part is used (the
    imaginary part is O(dt)).  Error O(dt), removed by extrapolation.
    """
    if c.n_real < 2:
        raise ValueError("the derivative needs at least two forward points")
    a = np.arange(c.n_real)
    b = c.partner(a)
    prev = np.where(a >= 1, a - 1, 1)
    n = occupancy(G_loc, c)
    ek = kinetic_energy(G_nn, nbr_of_src, J_real, c)
    U = np.asarray(U_real, dtype=np.float64)
    out = np.zeros((G_loc.shape[0], c.n_real), dtype=np.float64)
    for s in range(G_loc.shape[0]):
        diff = np.where(a >= 1, G_loc[s][a, b] - G_loc[s][prev, b],
                        G_loc[s][prev, b] - G_loc[s][a, b])
        dG = np.real(diff) / c.dt
        out[s] = (dG - eps_src[s] * n[s] - ek[s]) / U
    return out


def doubly_occupied_fraction(D: np.ndarray, n_sigma: np.ndarray) -> np.ndarray:
    """D~(t) = 2 sum_i D_i(t) / N with N = sum_i n_i(t) = 2 sum_i n_i,sigma(t)
    (Sec. V.B), over the sites given."""
    return 2.0 * D.sum(axis=0) / (2.0 * n_sigma.sum(axis=0))


def extrapolate_dt(dts, values) -> np.ndarray:
    """Value at dt -> 0 of the polynomial in dt through the given points (linear
    for two step sizes, quadratic for three), per entry (Sec. IV.D)."""
    h = np.asarray(dts, dtype=np.float64)
    vals = np.asarray(values, dtype=np.float64)
    if h.ndim != 1 or len(h) not in (2, 3) or vals.shape[0] != len(h):
        raise ValueError("two or three step sizes, one row of values each")
    if len(set(h.tolist())) != len(h):
        raise ValueError("step sizes must differ")
    out = np.zeros(vals.shape[1:], dtype=np.float64)
    for k in range(len(h)):
        wgt = 1.0
        for j in range(len(h)):
            if j != k:
                wgt *= (0.0 - h[j]) / (h[k] - h[j])
        out = out + wgt * vals[k]
    return out
