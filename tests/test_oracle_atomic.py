"""Pins for the oracle's atomic-limit contour Green's function (Sec. III).

Each check is fixed by the physics or by an independent evaluation, never by
re-typing the closed form:
* brute-force 4x4 Fock-space trace with explicit operator matrices;
* contour normalisation G^>(t,t) - G^<(t,t) = -i (anticommutator);
* KMS boundary condition across the imaginary branch (S[end, c] = -S[0, c]);
* n_sigma = p2 + p3 read from Im G^<(t, t+0^+), constant in time, Re G^< = 0;
* closed-form derivatives against central finite differences.
"""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _contour(n_real=6, n_imag=5, dt=0.13, beta=2.5, t_min=0.0):
    return O.make_contour(n_real, n_imag, dt, beta, t_min)


def _U(c, amp=0.15):
    return 1.0 + amp * np.sin(2.0 * c.real_times() + 0.3)


@pytest.mark.parametrize("eps", [-0.7, -0.5, 0.0, 0.35, 1.9])
def test_closed_form_matches_fock_trace(eps):
    c = _contour()
    U = _U(c)
    S = O.atomic_gf(eps, U, c)
    F = O.atomic_gf_fock(eps, U, c)
    assert np.abs(S - F).max() <= 1e-14 * max(1.0, np.abs(F).max())


@pytest.mark.parametrize("eps,beta", [(-0.5, 10.0), (0.3, 5.0), (1.9, 10.0), (-0.2, 0.5)])
def test_probabilities_sum_to_one(eps, beta):
    logp = O.boltzmann_weights(eps, 1.0, beta)
    assert abs(np.exp(logp).sum() - 1.0) < 1e-15
    # Ratios fixed by the Boltzmann factors of the four number states.
    p = np.exp(logp)
    assert np.isclose(p[2] / p[0], np.exp(-beta * eps), rtol=1e-13)
    assert np.isclose(p[3] / p[1], np.exp(-beta * (eps + 1.0)), rtol=1e-13)


@pytest.mark.parametrize("eps", [-0.5, 0.2, 1.6])
def test_equal_time_normalisation(eps):
    c = _contour(n_real=7, n_imag=6, beta=10.0)
    S = O.atomic_gf(eps, _U(c), c)
    a = np.arange(c.n_real)
    b = c.partner(a)
    # S[b(a), a] is G^>(t,t), S[a, b(a)] is G^<(t,t); they differ by -i.
    assert np.abs(S[b, a] - S[a, b] - (-1j)).max() < 1e-14


@pytest.mark.parametrize("eps", [-0.5, 0.2, 1.6])
def test_kms_boundary_condition(eps):
    c = _contour(n_real=5, n_imag=8, beta=10.0)
    S = O.atomic_gf(eps, _U(c), c)
    last = c.n_t - 1
    cols = np.arange(1, last)
    assert np.abs(S[last, cols] + S[0, cols]).max() < 1e-14


@pytest.mark.parametrize("eps", [-0.5, 0.1, 1.0])
def test_density_constant_and_real(eps):
    c = _contour(n_real=9, n_imag=6, beta=4.0)
    U = _U(c)
    S = O.atomic_gf(eps, U, c)
    a = np.arange(c.n_real)
    g_less = S[a, c.partner(a)]
    p = np.exp(O.boltzmann_weights(eps, U[0], c.beta))
    assert np.abs(np.real(g_less)).max() < 1e-15          # Re G^<(t,t) = 0 at J = 0
    assert np.abs(np.imag(g_less) - (p[2] + p[3])).max() < 1e-14
    n = O.occupancy(S[None], c)
    assert np.abs(n - (p[2] + p[3])).max() < 1e-14


def test_half_filling_at_particle_hole_symmetric_level():
    c = _contour(beta=7.0)
    S = O.atomic_gf(-0.5, np.ones(c.n_real), c)        # eps = -U/2
    n = O.occupancy(S[None], c)
    assert np.abs(n - 0.5).max() < 1e-15


def test_atomic_gf_bounded_on_all_branches():
    c = _contour(n_real=4, n_imag=16, beta=10.0)
    for eps in (-0.5, 1.9, -1.5):
        S = O.atomic_gf(eps, np.ones(c.n_real), c)
        assert np.all(np.isfinite(S))
        assert np.abs(S).max() <= 1.0 + 1e-12


def test_derivatives_match_finite_differences():
    c = _contour(n_real=5, n_imag=4, beta=3.0)
    U = _U(c, amp=0.2)
    eps = 0.27
    dS_de, dS_dU = O.atomic_gf_derivatives(eps, U, c)
    h = 1e-6
    fd = (O.atomic_gf(eps + h, U, c) - O.atomic_gf(eps - h, U, c)) / (2 * h)
    assert np.abs(fd - dS_de).max() < 1e-8
    for k in range(c.n_real):
        Up, Um = U.copy(), U.copy()
        Up[k] += h
        Um[k] -= h
        fd = (O.atomic_gf(eps, Up, c) - O.atomic_gf(eps, Um, c)) / (2 * h)
        assert np.abs(fd - dS_dU[k]).max() < 1e-8, k
