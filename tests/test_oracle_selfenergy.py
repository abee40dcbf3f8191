"""Pins for the oracle's second-order self-energy (Sec. III, eq. defnSigma,
eq. defnSigmatilde, eq. Sigmamix).

* U = 0: the cumulant vanishes for every index quadruple, equal indices
  included (Wick's theorem; fixes the contour ordering, the fermionic signs
  and the equal-index rule against the one-particle G).
* The paper's printed evaluation of G^II_{up dn} for t1 > t2 > t1' > t2'
  (products and ratios of the tabulated zeta_nu) is reproduced.
* The dressed block S (S - Sigma~)^-1 S equals the contour-algebra inverse of
  calG^-1 - calG^-1 o Sigma~ o calG^-1 built with explicit weights.
* The contraction restricted to listed outputs equals the whole table's entries.
* J = 0 gives Sigma~ = 0; Sigma~ scales as J^2 at small J; the mixed
  self-consistency loop converges and its fixed point satisfies the
  self-consistency equation.
"""
import numpy as np
import pytest

import oracle as O
from oracle import selfenergy as SE


def _contour():
    return O.make_contour(5, 4, 0.15, 2.0, 0.0)


@pytest.mark.parametrize("s2", ["up", "dn"])
def test_cumulant_vanishes_without_interaction(s2):
    c = _contour()
    Gt = SE.cumulant(0.23, np.zeros(c.n_real), c, "up", s2)
    assert np.abs(Gt).max() < 1e-14
    U = np.ones(c.n_real)
    assert np.abs(SE.cumulant(0.23, U, c, "up", s2)).max() > 1e-2


def test_printed_two_particle_ordering():
    c = _contour()
    eps = -0.3
    U = 1.0 + 0.2 * np.sin(2 * c.real_times())
    zeta = np.exp(1j * SE.state_phases(eps, U, c))
    p0 = np.exp(O.boltzmann_weights(eps, U[0], c.beta))[0]
    quads = [(12, 9, 5, 2), (13, 12, 11, 0), (10, 4, 3, 1)]
    got = SE.two_particle_gf(eps, U, c, "up", "dn", idx=quads)
    for (a1, a2, b1, b2), g in zip(quads, got):
        ref = (-1j) ** 2 * p0 * zeta[0, a1] * zeta[2, a2] / (zeta[2, a1] * zeta[3, a2]) \
            * zeta[3, b1] * zeta[2, b2] / (zeta[2, b1] * zeta[0, b2])
        assert abs(g - ref) <= 1e-14 * abs(ref)


def test_dressed_block_is_the_contour_inverse():
    c = _contour()
    rng = np.random.default_rng(4)
    S = O.atomic_gf(0.1, np.ones(c.n_real), c)
    sig = 0.05 * (rng.standard_normal((c.n_t, c.n_t)) + 1j * rng.standard_normal((c.n_t, c.n_t)))
    W = np.diag(c.w)
    Wi = np.linalg.inv(W)
    cinv = lambda A: Wi @ np.linalg.inv(A) @ Wi          # inverse under (A o B) = A W B
    calG_inv = cinv(S)
    Sigma = calG_inv @ W @ sig @ W @ calG_inv            # calG^-1 o Sigma~ o calG^-1
    ref = cinv(calG_inv - Sigma)
    got = SE.dressed_blocks(S[None], sig[None])[0]
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def _sigma(J0):
    c = _contour()
    V = np.array([0.05, -0.1, 0.0, 0.12])
    U = np.ones(c.n_real)
    J = np.full(c.n_real, J0)
    S = np.stack([O.atomic_gf(v - 0.5, U, c) for v in V])
    G = O.dyson_dense(S, O.hopping_operator_dense(2, 2, False, J, c))
    n_t = c.n_t
    G_loc = np.stack([G[i * n_t:(i + 1) * n_t, i * n_t:(i + 1) * n_t] for i in range(4)])
    return SE.sigma_tilde(V, U, 0.0, J, c, 2, 2, False, G_loc)


def test_sigma_tilde_zero_hopping_and_j_squared_scaling():
    assert np.abs(_sigma(0.0)).max() == 0.0
    a, b = np.abs(_sigma(0.02)).max(), np.abs(_sigma(0.01)).max()
    assert 3.8 < a / b < 4.2


def test_sigma_tilde_entries_restrict_the_full_contraction():
    # the sampled form (for long contours) against the whole table, with a
    # time-dependent U and an arbitrary (non-lattice) G_loc
    c = _contour()
    rng = np.random.default_rng(4)
    V = np.array([0.05, -0.1, 0.0, 0.12])
    U = 1.0 + 0.2 * np.sin(np.arange(c.n_real))
    J = np.full(c.n_real, 0.08)
    G_loc = 0.3 * (rng.standard_normal((4, c.n_t, c.n_t)) + 1j * rng.standard_normal((4, c.n_t, c.n_t)))
    full = SE.sigma_tilde(V, U, 0.1, J, c, 2, 2, False, G_loc)
    entries = [(0, 0, 0), (1, 3, 11), (2, c.n_t - 1, 0), (3, 7, 7), (1, 12, 2)]
    got = SE.sigma_tilde_entries(V, U, 0.1, J, c, 2, 2, False, G_loc, entries)
    ref = np.array([full[i, a, b] for i, a, b in entries])
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(full).max()


def test_selfconsistent_loop_converges_to_a_fixed_point():
    c = _contour()
    V = np.array([0.05, -0.1, 0.0, 0.12])
    U = np.ones(c.n_real)
    J = np.full(c.n_real, 0.1)
    sig, G, hist = SE.selfconsistent(V, U, 0.0, J, c, 2, 2, delta_sc=1e-12, max_iter=60)
    assert hist[-1] <= 1e-12 and len(hist) < 60
    assert all(hist[k + 1] < hist[k] for k in range(2, len(hist) - 1))
    n_t = c.n_t
    G_loc = np.stack([G[i * n_t:(i + 1) * n_t, i * n_t:(i + 1) * n_t] for i in range(4)])
    again = SE.sigma_tilde(V, U, 0.0, J, c, 2, 2, False, G_loc)
    # after the last mixing step the gap to the fixed point is (1 - lam) times
    # the last measured increment
    assert np.abs(again - sig).max() <= hist[-1]
