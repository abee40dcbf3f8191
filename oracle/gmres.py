"""Preconditioned restarted GMRES for the lattice Dyson equation (oracle; test
infrastructure only).

Paper: App. C (the algorithm) and Sec. IV.D (eq. Ginvblockstruct: A = B - J;
the preconditioner P = B^-1, eq. definitionB; eq. blockedGMRESproblem: one
solve per unit vector e_j of a source site, all vectors of a bundle treated
alike).  At lowest order B^-1 = S = blockdiag(S_i), so the preconditioned
system of each column is

    P A u = P b   with   P A = I - S D,   P b = S e_j   (= X0, the first term
                                                        of the Dyson series),

and its solution is the column S e_j of G = (I - S D)^-1 S.

Steps, per column, in the appendix's order:
 1. u0 = P b; z0 = P b - P A u0; q_1 = z0 / |z0|_2; H = 0.
 2. For d = 1 .. m: w = P A q_d; for i = 1 .. d: h_id = <q_i|w>,
    w <- w - h_id q_i (modified Gram-Schmidt); h_{d+1,d} = |w|_2.
    Step 3 gives the residual of the current d: stop on convergence or
    breakdown (h_{d+1,d} = 0), else q_{d+1} = w / h_{d+1,d}.
 3. y = argmin | |z0|_2 e_1 - H_d y |_2, u = u0 + (q_1 .. q_d) y.
 After m steps without convergence the method restarts from u.

Reading (listed with the others in the design notes): the least-squares
problem of step 3 uses the (d+1) x d upper Hessenberg block of H.  The
appendix names the upper-left square, which would give the Galerkin (FOM)
iterate; only the rectangular block minimises the residual over the affine
Krylov space, which is the property the appendix defines the method by.
The stopping rule is the relative preconditioned residual
|z_d|_2 <= tol |P b|_2 per column, checked through step 3.
"""
import numpy as np


def gmres_column(M: np.ndarray, x0: np.ndarray, restart: int, tol: float,
                 max_iter: int, stop: bool = True):
    """GMRES(restart) for M u = x0 with u0 = x0 (App. C).

    M is the dense preconditioned operator P A; x0 = P b.  Returns
    (u, history, iterations): history[0] is |z0|_2, history[k] the residual
    2-norm after k Arnoldi steps (the value step 3 gives).  With stop=False the
    method runs exactly max_iter Arnoldi steps (unless it breaks down).
    """
    ref = np.linalg.norm(x0)
    u = x0.astype(np.complex128).copy()
    history = []
    n_it = 0
    while True:
        z = x0 - M @ u
        beta = np.linalg.norm(z)
        if not history:
            history.append(beta)
        if beta == 0.0 or (stop and beta <= tol * ref) or n_it >= max_iter:
            return u, history, n_it
        Q = [z / beta]
        H = np.zeros((restart + 1, restart), dtype=np.complex128)
        finished = False
        for d in range(restart):
            w = M @ Q[d]
            for i in range(d + 1):
                H[i, d] = np.vdot(Q[i], w)
                w = w - H[i, d] * Q[i]
            H[d + 1, d] = np.linalg.norm(w)
            n_it += 1
            rhs = np.zeros(d + 2, dtype=np.complex128)
            rhs[0] = beta
            Hd = H[:d + 2, :d + 1]
            y = np.linalg.lstsq(Hd, rhs, rcond=None)[0]
            res = np.linalg.norm(rhs - Hd @ y)
            history.append(res)
            breakdown = H[d + 1, d] == 0.0
            finished = breakdown or (stop and res <= tol * ref) or n_it >= max_iter
            if finished or d == restart - 1:
                u = u + np.stack(Q[:d + 1], axis=1) @ y
                break
            Q.append(w / H[d + 1, d])
        if finished:
            return u, history, n_it


def gmres_dense(S_blocks: np.ndarray, D: np.ndarray, cols, restart: int, tol: float,
                max_iter: int, stop: bool = True):
    """GMRES columns of G = (I - S D)^-1 S for the listed global columns.

    Returns (U, histories, iterations) with U of shape (N_r N_t, len(cols)).
    """
    from .dyson import blockdiag
    S = blockdiag(S_blocks)
    M = np.eye(S.shape[0], dtype=np.complex128) - S @ D
    cols = list(cols)
    U = np.zeros((S.shape[0], len(cols)), dtype=np.complex128)
    hists, iters = [], []
    for k, c in enumerate(cols):
        u, h, it = gmres_column(M, S[:, c], restart, tol, max_iter, stop)
        U[:, k] = u
        hists.append(h)
        iters.append(it)
    return U, hists, iters
