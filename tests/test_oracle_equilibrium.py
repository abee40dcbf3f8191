"""Equilibrium diagnostics (Fig. 1 caption; Sec. V.B): with constant parameters
the densities stay constant in time and the total particle number is
conserved.  On the grid these hold only up to O(dt), so the bounds are loose
and the check is that the drift shrinks when dt is halved."""
import numpy as np

import oracle as O
from paper_1309_5994_amd import workloads as W


def _drift(dt, n_real, n_imag):
    wl = W.custom(3, 3, n_real, n_imag, J0=0.1, beta=4.0, dt=dt, curvature=0.05)
    c = O.make_contour(wl.n_real, wl.n_imag, wl.dt, wl.beta)
    eps = O.site_levels(wl.V, wl.U, wl.mu)
    S = np.stack([O.atomic_gf(e, wl.U, c) for e in eps])
    D = O.hopping_operator_dense(wl.Lx, wl.Ly, False, wl.J, c)
    G = O.dyson_dense(S, D)
    n = O.occupancy(O.local_blocks_from_dense(G, c.n_t, range(wl.n_r)), c)
    return np.abs(n - n[:, :1]).max(), np.abs(n.sum(0) - n[:, 0].sum()).max()


def test_equilibrium_drift_is_small_and_shrinks():
    d0, N0 = _drift(0.2, 6, 8)
    d1, N1 = _drift(0.1, 11, 16)
    assert d0 < 2e-2 and d1 < 1e-2
    assert d1 < 0.7 * d0
    assert N1 < 0.7 * N0
