"""U = 0 pin: the strong-coupling Dyson solve is exact for free fermions.

With U = 0 the atomic Green's function is the free single-site propagator, and
G = S + S D G is the exact free lattice propagator of h_ij = eps_i delta_ij
+ J_ij (the sign that eq. Glatt's [calG^-1 - J]^-1 implies), apart from the
contour discretisation.  The exact propagator is built here independently from
the one-body Hamiltonian: eigen-decomposition, Fermi function of h(t_min) and
exp(-i h z) along the contour.  The discretisation error must shrink linearly
as dt and dtau are halved together.  This is the only pin that fixes the contour
conventions (point placement, weights, the equal-index rule and the sign of J).
"""
import numpy as np
import pytest

import oracle as O


def free_lattice_gf(h, c):
    e, vec = np.linalg.eigh(h)
    n, n_t = h.shape[0], c.n_t
    z = c.z - c.t_min
    log_hole = -np.logaddexp(0.0, -c.beta * e)     # log(1 - f)
    log_part = -np.logaddexp(0.0, c.beta * e)      # log f
    G = np.zeros((n, n_t, n, n_t), dtype=complex)
    for a in range(n_t):
        for b in range(n_t):
            ph = -1j * e * (z[a] - z[b])
            g = -1j * np.exp(ph + log_hole) if a > b else 1j * np.exp(ph + log_part)
            G[:, a, :, b] = (vec * g[None, :]) @ vec.T
    return G.reshape(n * n_t, n * n_t)


def _run(dt, n_imag, T=1.0, beta=2.0, J=0.2, Lx=2, Ly=2, periodic=False,
         V=(0.1, -0.2, 0.3, 0.0), sign=+1.0, mutate=None):
    n_real = int(round(T / dt)) + 1
    c = O.make_contour(n_real, n_imag, dt, beta)
    V = np.asarray(V)
    U = np.zeros(n_real)
    S = np.stack([O.atomic_gf(v, U, c) for v in V])
    D = O.hopping_operator_dense(Lx, Ly, periodic, np.full(n_real, J), c)
    if mutate is not None:
        S, D = mutate(S, D, c)
    G = O.dyson_dense(S, D)
    nbr = O.neighbours(Lx, Ly, periodic)
    h = np.diag(V).astype(float)
    for i in range(Lx * Ly):
        for k in nbr[i]:
            if k >= 0:
                h[i, k] += sign * J
    Gx = free_lattice_gf(h, c)
    n_d = O.occupancy(O.local_blocks_from_dense(G, c.n_t, range(Lx * Ly)), c)
    n_x = O.occupancy(O.local_blocks_from_dense(Gx, c.n_t, range(Lx * Ly)), c)
    return np.abs(G - Gx).max(), np.abs(n_d - n_x).max()


GRIDS = [(0.1, 8), (0.05, 16), (0.025, 32)]


def test_free_fermion_first_order_convergence():
    errs = [_run(dt, m) for dt, m in GRIDS]
    for (eg0, en0), (eg1, en1) in zip(errs, errs[1:]):
        assert 1.8 < eg0 / eg1 < 2.3
        assert 1.8 < en0 / en1 < 2.3
    assert errs[-1][0] < 0.01


def _fails_to_converge(mutate=None, sign=+1.0):
    errs = [_run(dt, m, mutate=mutate, sign=sign) for dt, m in GRIDS]
    ratios = [errs[i][0] / errs[i + 1][0] for i in range(len(errs) - 1)]
    return min(ratios) < 1.5 or errs[-1][0] > 0.05


def test_planted_mistakes_break_the_pin():
    """A wrong sign, weight, branch rule or operand order must fail the U=0 pin."""
    # Sign of J opposite to the Dyson equation's.
    assert _fails_to_converge(sign=-1.0)

    # Imaginary-branch weight without the -i.
    def no_minus_i(S, D, c):
        scale = np.where(c.branch == 2, 1j, 1.0)      # -i dtau -> dtau
        n_t = c.n_t
        f = np.tile(scale, D.shape[0] // n_t)
        return S, D * f[None, :]
    assert _fails_to_converge(no_minus_i)

    # Transposed product D S instead of S D.
    def transposed(S, D, c):
        n_t = c.n_t
        St = np.stack([s.T for s in S])
        return St, D
    assert _fails_to_converge(transposed)

    # Equal contour index read as G^> instead of G^< (t' = t + 0^+).
    def diagonal_greater(S, D, c):
        S = S.copy()
        idx = np.arange(c.n_t)
        for s in S:
            s[idx, idx] -= 1j
        return S, D
    assert _fails_to_converge(diagonal_greater)


def test_free_fermion_periodic_lattice():
    errs = [_run(dt, m, Lx=3, Ly=3, periodic=True, V=np.linspace(-0.2, 0.2, 9), J=0.15)
            for dt, m in GRIDS[:2]]
    assert 1.8 < errs[0][0] / errs[1][0] < 2.3


def _ekin_errors(dt, n_imag, T=1.0, beta=2.0, J=0.2, Lx=2, Ly=2, V=(0.1, -0.2, 0.3, 0.0)):
    """Kinetic energy of each site (Sec. III.A) at U = 0 against the free value
    sum_j h_ij <c_i^dag c_j> = (h_hop f(h))_ii, constant in time for a
    time-independent h; returns (max error, the exact values)."""
    n_real = int(round(T / dt)) + 1
    c = O.make_contour(n_real, n_imag, dt, beta)
    V = np.asarray(V)
    S = np.stack([O.atomic_gf(v, np.zeros(n_real), c) for v in V])
    Jr = np.full(n_real, J)
    G = O.dyson_dense(S, O.hopping_operator_dense(Lx, Ly, False, Jr, c))
    nbr = O.neighbours(Lx, Ly, False)
    sites = list(range(Lx * Ly))
    ek = O.kinetic_energy(O.neighbour_blocks_from_dense(G, c.n_t, nbr, sites), nbr, Jr, c)
    hop = np.zeros((Lx * Ly, Lx * Ly))
    for i in sites:
        for k in nbr[i]:
            if k >= 0:
                hop[i, k] = J
    e, vec = np.linalg.eigh(np.diag(V) + hop)
    f = (vec * (1.0 / (1.0 + np.exp(beta * e)))[None, :]) @ vec.T
    exact = np.diag(hop @ f)
    return np.abs(ek - exact[:, None]).max(), exact


def test_free_fermion_kinetic_energy_sign_and_convergence():
    errs = [_ekin_errors(dt, m) for dt, m in GRIDS]
    exact = errs[0][1]
    assert np.all(exact < 0)                    # hopping lowers the energy
    for (e0, _), (e1, _) in zip(errs, errs[1:]):
        assert 1.7 < e0 / e1 < 2.4
    assert errs[-1][0] < 0.05 * np.abs(exact).min()
