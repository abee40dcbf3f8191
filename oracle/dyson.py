"""Lattice Dyson equation, solved directly (oracle; test infrastructure only).

Paper: eq. Glatt gives G = [calG^-1 - J - Sigma]^-1.  At lowest order
(Sigma = 0) the diagonal block of the inverse is B_i = calG_i^-1
(eq. blockdiagdysonelement), so with S = blockdiag(calG_i) and the discretised
hopping operator D (see lattice.py) the lattice Green's function solves

    (I - S D) G = S,    i.e.  G = S + S D G.

The sign follows eq. Glatt literally (B - J, eq. Ginvblockstruct); on the
bipartite square lattice J -> -J is a gauge transformation, so densities,
kinetic energies and their gradients do not depend on it.  App. C shows that
the preconditioned Krylov iteration and the Dyson series sum_nu (S D)^nu S
both converge to this same solution, which is what the oracle computes
exactly:

* ``dyson_dense``            -- LU factorisation of the full (N_r N_t)^2 matrix
                                (LAPACK zgetrf/zgetrs through scipy).
* ``dyson_columns_blocktri`` -- the same solve for selected source columns by
                                exact block-tridiagonal (Thomas) elimination,
                                with one super-block per lattice row x (the
                                matrix couples row x only to rows x +- 1).
* ``neumann_partial_sums``   -- X_n = sum_{nu <= n} (S D)^nu S X restricted to
                                chosen columns, for the Dyson-series pins.
* ``dyson_columns_truncated`` -- the columns of each source solved on the
                                sites within a lattice distance of it only.
"""
import numpy as np
import scipy.linalg as sla

from .contour import Contour
from .lattice import neighbours, hopping_on_contour


def blockdiag(S_blocks: np.ndarray) -> np.ndarray:
    n_r, n_t, _ = S_blocks.shape
    out = np.zeros((n_r * n_t, n_r * n_t), dtype=np.complex128)
    for i in range(n_r):
        out[i * n_t:(i + 1) * n_t, i * n_t:(i + 1) * n_t] = S_blocks[i]
    return out


def dense_system_matrix(S_blocks: np.ndarray, D: np.ndarray) -> np.ndarray:
    """A = I - S D."""
    S = blockdiag(S_blocks)
    return np.eye(S.shape[0], dtype=np.complex128) - S @ D


def dyson_dense(S_blocks: np.ndarray, D: np.ndarray, cols=None) -> np.ndarray:
    """G = (I - S D)^-1 S by dense LU; all columns, or the listed global columns."""
    S = blockdiag(S_blocks)
    A = np.eye(S.shape[0], dtype=np.complex128) - S @ D
    lu = sla.lu_factor(A, check_finite=True)
    rhs = S if cols is None else S[:, np.asarray(cols)]
    return sla.lu_solve(lu, rhs)


def _site_coupling(S_i: np.ndarray, wJ: np.ndarray) -> np.ndarray:
    """Block (i, k) of S D for one bond: S_i diag(w J) (N_t x N_t)."""
    return S_i * wJ[None, :]


def dyson_columns_blocktri(S_blocks: np.ndarray, Lx: int, Ly: int,
                           J_real: np.ndarray, c: Contour, src_sites,
                           periodic_y: bool = False) -> np.ndarray:
    """Columns of G for the listed source sites, by block-tridiagonal elimination.

    Returns an array of shape (N_r, N_t, len(src_sites) * N_t): for each target
    site, row time a, and (source, column time).  Exact up to rounding; the
    lattice must be open in x (rows x and x +- 1 only), periodic in y allowed.
    """
    n_r, n_t, _ = S_blocks.shape
    if n_r != Lx * Ly:
        raise ValueError("S must hold one block per lattice site")
    nbr = neighbours(Lx, Ly, False)
    if periodic_y:
        if Ly < 3:
            raise ValueError("periodic_y needs Ly >= 3")
        for x in range(Lx):
            nbr[x * Ly + 0, 2] = x * Ly + Ly - 1
            nbr[x * Ly + Ly - 1, 3] = x * Ly + 0
    wJ = c.w * hopping_on_contour(J_real, c)
    src_sites = [int(s) for s in src_sites]
    n_rhs = len(src_sites) * n_t
    nb = Ly * n_t   # super-block size (one lattice row)

    def row_of(i):
        return i // Ly

    def super_blocks(x):
        """Diagonal, lower (x, x-1) and upper (x, x+1) super-blocks of I - S D."""
        diag = np.eye(nb, dtype=np.complex128)
        lower = np.zeros((nb, nb), dtype=np.complex128) if x > 0 else None
        upper = np.zeros((nb, nb), dtype=np.complex128) if x < Lx - 1 else None
        for y in range(Ly):
            i = x * Ly + y
            blk = _site_coupling(S_blocks[i], wJ)
            for k in nbr[i]:
                if k < 0:
                    continue
                yk = k % Ly
                rows = slice(y * n_t, (y + 1) * n_t)
                cols = slice(yk * n_t, (yk + 1) * n_t)
                if row_of(k) == x:
                    diag[rows, cols] -= blk
                elif row_of(k) == x - 1:
                    lower[rows, cols] -= blk
                else:
                    upper[rows, cols] -= blk
        return diag, lower, upper

    def rhs_row(x):
        r = np.zeros((nb, n_rhs), dtype=np.complex128)
        for s, j in enumerate(src_sites):
            if row_of(j) == x:
                y = j % Ly
                r[y * n_t:(y + 1) * n_t, s * n_t:(s + 1) * n_t] = S_blocks[j]
        return r

    # Forward elimination: Dp_x = A_x - L_x Dp_{x-1}^-1 U_{x-1}, Rp_x likewise.
    # The upper super-blocks are rebuilt during back substitution instead of
    # being kept, which halves the memory of large lattices.
    lus, rps = [], []
    prev_lu, prev_upper, prev_rp = None, None, None
    for x in range(Lx):
        diag, lower, upper = super_blocks(x)
        rp = rhs_row(x)
        if x > 0:
            diag = diag - lower @ sla.lu_solve(prev_lu, prev_upper)
            rp = rp - lower @ sla.lu_solve(prev_lu, prev_rp)
        del lower
        lu = sla.lu_factor(diag, overwrite_a=True)
        lus.append(lu)
        rps.append(rp)
        prev_lu, prev_upper, prev_rp = lu, upper, rp
    del prev_upper
    # Back substitution.
    out = np.zeros((Lx, nb, n_rhs), dtype=np.complex128)
    out[Lx - 1] = sla.lu_solve(lus[Lx - 1], rps[Lx - 1])
    for x in range(Lx - 2, -1, -1):
        upper = super_blocks(x)[2]
        out[x] = sla.lu_solve(lus[x], rps[x] - upper @ out[x + 1])
    return out.reshape(Lx * Ly, n_t, n_rhs)


def neumann_partial_sums(S_blocks: np.ndarray, D: np.ndarray, cols, n_terms: int):
    """[X_0, X_1, ..., X_n] with X_0 = S[:, cols] and X_{m+1} = X_0 + S D X_m."""
    S = blockdiag(S_blocks)
    SD = S @ D
    x0 = S[:, np.asarray(cols)]
    out = [x0]
    x = x0
    for _ in range(n_terms):
        x = x0 + SD @ x
        out.append(x)
    return out


def lattice_distance(i: int, j: int, Lx: int, Ly: int, periodic: bool = False) -> int:
    """Manhattan distance between sites i = x * Ly + y and j (minimum image if periodic)."""
    dx, dy = abs(i // Ly - j // Ly), abs(i % Ly - j % Ly)
    if periodic:
        dx, dy = min(dx, Lx - dx), min(dy, Ly - dy)
    return dx + dy


def dyson_columns_truncated(S_blocks: np.ndarray, D: np.ndarray, Lx: int, Ly: int,
                            periodic: bool, src_sites, radius: int) -> np.ndarray:
    """Columns of each source j solved on the sites within lattice distance
    `radius` of j only: the Dyson equation restricted to those sites (App. C:
    only blocks near the source matter), G zero elsewhere.  Shape
    (N_r, N_t, len(src_sites) * N_t)."""
    n_r, n_t, _ = S_blocks.shape
    S = blockdiag(S_blocks)
    out = np.zeros((n_r, n_t, len(src_sites) * n_t), dtype=np.complex128)
    for s, j in enumerate(src_sites):
        keep = [i for i in range(n_r) if lattice_distance(i, j, Lx, Ly, periodic) <= radius]
        idx = np.concatenate([np.arange(i * n_t, (i + 1) * n_t) for i in keep])
        A = np.eye(len(idx), dtype=np.complex128) - S[np.ix_(idx, idx)] @ D[np.ix_(idx, idx)]
        rhs = S[idx, j * n_t:(j + 1) * n_t]
        sol = np.linalg.solve(A, rhs)
        for k, i in enumerate(keep):
            out[i, :, s * n_t:(s + 1) * n_t] = sol[k * n_t:(k + 1) * n_t]
    return out
