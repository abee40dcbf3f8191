"""Lattice geometry and the hopping operator (oracle; test infrastructure only).

Paper: Sec. IV.D, eq. Ginvblockstruct -- every row of the inverse lattice
Green's function holds at most four nearest-neighbour hopping blocks, and each
hopping block is diagonal in contour time (a contour delta function times the
tight-binding amplitude).  Discretised with the contour weights, the operator
is D[(i,a),(k,a)] = w_a J(z_a) for every nearest neighbour k of site i.

Site index i = x * Ly + y.  Neighbour slots are ordered (x-1, y), (x+1, y),
(x, y-1), (x, y+1); a missing neighbour (open edge) is -1.  Periodic lattices
need Lx, Ly >= 3 so that no bond is listed twice.

The hopping is uniform in space and given per forward time; the backward
branch uses the forward value at the same physical time and the imaginary
branch uses J(t_min) (a reading: the paper does not say).
"""
import numpy as np

from .contour import Contour, IMAGINARY


def neighbours(Lx: int, Ly: int, periodic: bool = False) -> np.ndarray:
    if periodic and (Lx < 3 or Ly < 3):
        raise ValueError("periodic lattices need Lx, Ly >= 3")
    nbr = -np.ones((Lx * Ly, 4), dtype=np.int64)
    for x in range(Lx):
        for y in range(Ly):
            i = x * Ly + y
            cand = [(x - 1, y), (x + 1, y), (x, y - 1), (x, y + 1)]
            for slot, (xx, yy) in enumerate(cand):
                if periodic:
                    xx %= Lx
                    yy %= Ly
                elif not (0 <= xx < Lx and 0 <= yy < Ly):
                    continue
                nbr[i, slot] = xx * Ly + yy
    return nbr


def hopping_on_contour(J_real: np.ndarray, c: Contour) -> np.ndarray:
    """J(z_a) for every contour point."""
    J_real = np.asarray(J_real, dtype=np.float64)
    if J_real.shape != (c.n_real,):
        raise ValueError("J must hold one value per forward time")
    out = np.zeros(c.n_t, dtype=np.float64)
    for a in range(c.n_t):
        out[a] = J_real[0] if c.branch[a] == IMAGINARY else J_real[c.tidx[a]]
    return out


def hopping_operator_dense(Lx: int, Ly: int, periodic: bool,
                           J_real: np.ndarray, c: Contour) -> np.ndarray:
    """Dense D of shape (N_r N_t, N_r N_t), index (i, a) -> i * N_t + a."""
    nbr = neighbours(Lx, Ly, periodic)
    Jc = hopping_on_contour(J_real, c)
    n_t = c.n_t
    N = Lx * Ly * n_t
    D = np.zeros((N, N), dtype=np.complex128)
    for i in range(Lx * Ly):
        for k in nbr[i]:
            if k < 0:
                continue
            for a in range(n_t):
                D[i * n_t + a, k * n_t + a] += c.w[a] * Jc[a]
    return D
