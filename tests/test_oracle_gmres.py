"""Pins for the oracle's preconditioned restarted GMRES (App. C).

* It converges to the direct solve G = (I - S D)^-1 S (also across restarts).
* Minimal residual: after d steps its residual equals, and its iterate is, the
  least-squares optimum over u0 + span(z0, M z0, ..., M^{d-1} z0) found by brute
  force from the explicit Krylov matrix (catches a dropped conjugate, a wrong
  Hessenberg index or the square-block (FOM) reading).
* The d-th Neumann partial sum lies in the same affine space (App. C: step d
  holds exactly d hopping processes), so GMRES's residual is never larger.
* Light cone: after d steps the iterate vanishes beyond lattice distance d.
* J = 0: the preconditioned start is already exact (zero steps).
* Finite termination of full GMRES on a small system, and convergence where
  the Dyson series itself diverges (spectral radius of S D above 1).
"""
import numpy as np
import pytest

import oracle as O
from paper_1309_5994_amd import workloads as W


def _system(wl):
    c = O.make_contour(wl.n_real, wl.n_imag, wl.dt, wl.beta, wl.t_min)
    eps = O.site_levels(wl.V, wl.U, wl.mu)
    S = np.stack([O.atomic_gf(e, wl.U, c) for e in eps])
    D = O.hopping_operator_dense(wl.Lx, wl.Ly, wl.periodic, wl.J, c)
    M = O.dense_system_matrix(S, D)
    return c, S, D, M


@pytest.mark.parametrize("restart", [3, 30])
def test_gmres_converges_to_direct_solve(restart):
    wl = W.custom(3, 3, 5, 4, J0=0.12, seed=5)
    c, S, D, M = _system(wl)
    n_t = c.n_t
    cols = [0, 4 * n_t + 3, 8 * n_t + n_t - 1, 2 * n_t + 7]
    G = O.dyson_dense(S, D, cols)
    U, hists, iters = O.gmres_dense(S, D, cols, restart, 1e-14, 200)
    assert np.abs(U - G).max() / np.abs(G).max() < 1e-12
    for h in hists:
        assert h[-1] <= 1e-14 * h[0] * 10 or h[-1] < 1e-13


def test_minimal_residual_against_explicit_krylov_space():
    wl = W.custom(3, 2, 4, 3, J0=0.15, seed=7)
    c, S, D, M = _system(wl)
    x0 = O.blockdiag(S)[:, 5]
    z0 = x0 - M @ x0
    for d in range(1, 5):
        u, hist, it = O.gmres_column(M, x0, 10, 1e-300, d, stop=False)
        assert it == d
        K = np.stack([np.linalg.matrix_power(M, k) @ z0 for k in range(d)], axis=1)
        y = np.linalg.lstsq(M @ K, z0, rcond=None)[0]
        best = np.linalg.norm(z0 - M @ K @ y)
        assert abs(hist[d] - best) <= 1e-9 * hist[0]
        assert abs(np.linalg.norm(x0 - M @ u) - best) <= 1e-9 * hist[0]
        assert np.abs(u - (x0 + K @ y)).max() <= 1e-8 * np.abs(x0).max()
        # monotone within a cycle
        assert all(hist[k + 1] <= hist[k] * (1 + 1e-12) for k in range(d))


def test_gmres_residual_never_above_neumann_partial_sum():
    wl = W.custom(3, 3, 4, 4, J0=0.1, seed=9)
    c, S, D, M = _system(wl)
    col = 4 * c.n_t + 2
    xs = O.neumann_partial_sums(S, D, [col], 6)
    x0 = xs[0][:, 0]
    for d in range(1, 6):
        u, hist, _ = O.gmres_column(M, x0, 10, 1e-300, d, stop=False)
        neumann_res = np.linalg.norm(x0 - M @ xs[d][:, 0])
        assert hist[d] <= neumann_res * (1 + 1e-10)
        assert np.linalg.norm(x0 - M @ u) <= neumann_res * (1 + 1e-10)


def test_gmres_light_cone():
    wl = W.custom(5, 5, 3, 3, J0=0.1, seed=2)
    c, S, D, M = _system(wl)
    n_t = c.n_t
    j = 12      # centre site (2, 2)
    x0 = O.blockdiag(S)[:, j * n_t + 1]
    for d in range(0, 4):
        u, _, _ = O.gmres_column(M, x0, 10, 1e-300, d, stop=False)
        for i in range(wl.Lx * wl.Ly):
            dist = abs(i // wl.Ly - 2) + abs(i % wl.Ly - 2)
            blk = u[i * n_t:(i + 1) * n_t]
            if dist > d:
                assert np.all(blk == 0)
            else:
                assert np.abs(blk).max() > 0


def test_zero_hopping_needs_no_step():
    wl = W.custom(2, 2, 4, 3, J0=0.0, seed=1)
    c, S, D, M = _system(wl)
    x0 = O.blockdiag(S)[:, 3]
    u, hist, it = O.gmres_column(M, x0, 5, 1e-12, 50)
    assert it == 0 and hist == [0.0]
    assert np.array_equal(u, x0)


def test_full_gmres_terminates_and_rescues_a_divergent_series():
    wl = W.custom(2, 2, 5, 4, J0=0.8, seed=3)
    c, S, D, M = _system(wl)
    n = M.shape[0]
    SD = O.blockdiag(S) @ D
    assert np.abs(np.linalg.eigvals(SD)).max() > 1.5      # Neumann diverges
    cols = [0, n // 2 + 1]
    G = O.dyson_dense(S, D, cols)
    U, hists, iters = O.gmres_dense(S, D, cols, n, 1e-13, n)
    assert max(iters) <= n
    assert np.abs(U - G).max() / np.abs(G).max() < 1e-10
    xs = O.neumann_partial_sums(S, D, cols, 40)
    assert np.abs(xs[-1] - G).max() > 1.0                  # the series does not
