"""Pins for the oracle's double occupancy (eq. docc with the one-sided time
derivative of App. B), the doubly occupied fraction (Sec. V.B) and the dt -> 0
extrapolation (Sec. IV.D).

In the atomic limit (J = 0) the double occupancy of every site stays the
Boltzmann weight of the doubly occupied state, p3 = e^{-beta (2 eps + U)} / Z,
at all times, also when U(t) is modulated (the atomic Hamiltonian commutes
with n_up n_down).  The formula applied to the exact atomic G reproduces it
with a discretisation error of second order for constant U (the first-order
term of the derivative is imaginary) and first order for modulated U (the
phase between t_{a-1} and t_a carries U at the half step), which quadratic
extrapolation from three step sizes removes.  Using U(0) instead of U(t), a
wrong derivative sign or a dropped eps n term each fail these checks.
"""
import numpy as np
import pytest

import oracle as O


def _atomic(dt, U_mod, T=2.0, beta=3.0):
    n_real = int(round(T / dt)) + 1
    c = O.make_contour(n_real, 6, dt, beta, 0.0)
    U = 1.0 + U_mod * np.sin(2.0 * c.real_times())
    eps = np.array([-0.5, -0.2, 0.1, 0.4])
    S = np.stack([O.atomic_gf(e, U, c) for e in eps])
    G_nn = np.zeros((len(eps), 4, c.n_t, c.n_t), dtype=complex)
    nbr = -np.ones((len(eps), 4), dtype=np.int64)
    D = O.double_occupancy(S, G_nn, nbr, eps, U, np.zeros(n_real), c)
    Z = 1.0 + 2.0 * np.exp(-beta * eps) + np.exp(-beta * (2.0 * eps + U[0]))
    p3 = np.exp(-beta * (2.0 * eps + U[0])) / Z
    n = O.occupancy(S, c)
    return c, D, p3, n


@pytest.mark.parametrize("U_mod,order", [(0.0, 2), (0.3, 1)])
def test_atomic_limit_double_occupancy_converges(U_mod, order):
    errs = []
    for dt in (0.1, 0.05, 0.025):
        c, D, p3, n = _atomic(dt, U_mod)
        idx = [int(round(t / dt)) for t in (0.0, 0.5, 1.0, 1.5, 2.0)]
        errs.append(D[:, idx] - p3[:, None])
    e = [np.abs(x).max() for x in errs]
    assert e[0] < 5e-3
    for k in range(2):
        assert abs(e[k] / e[k + 1] - 2.0 ** order) < 0.1 * 2.0 ** order
    ex = O.extrapolate_dt([0.1, 0.05, 0.025], errs)
    assert np.abs(ex).max() < 1e-2 * e[2]


def test_doubly_occupied_fraction_in_the_atomic_limit():
    c, D, p3, n = _atomic(0.025, 0.0)
    frac = O.doubly_occupied_fraction(D, n)
    assert np.abs(frac - p3.sum() / n[:, 0].sum()).max() < 1e-5
    assert np.allclose(n, n[:, :1])               # occupations are constant at J = 0


def test_extrapolation_is_exact_for_low_order_polynomials():
    rng = np.random.default_rng(3)
    a, b, c2 = rng.standard_normal((3, 5))
    h = [0.2, 0.1, 0.05]
    vals = [a + b * x + c2 * x * x for x in h]
    assert np.abs(O.extrapolate_dt(h, vals) - a).max() < 1e-13
    assert np.abs(O.extrapolate_dt(h[:2], [a + b * x for x in h[:2]]) - a).max() < 1e-13
    with pytest.raises(ValueError):
        O.extrapolate_dt([0.1, 0.1], vals[:2])
