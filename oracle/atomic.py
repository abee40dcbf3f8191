"""Atomic-limit (no-hopping) contour Green's function of one site (oracle).

Paper: Sec. III.  The on-site propagator is -i <T_C c(t) c^dagger(t')> under
the local Hamiltonian H_0^(l) = eps (n_up + n_dn) + U n_up n_dn, evaluated in
the particle-number basis {|0>, |dn>, |up>, |dn up>} with energies
E_0 = 0, E_1 = E_2 = eps, E_3 = 2 eps + U, by inserting the local time
evolution (eq. localtimeevolution) and the tabulated phases
zeta_nu(t) = exp(i int_0^t E_nu) (eq. cumulanttabulation).  The Boltzmann
weights are exp(-beta E_nu(0)) / Z (the equation defining Z), taken at the
point where the imaginary branch is attached (t_min here).  The level is
eps_i = V_i - U(0)/2 - mu (eq. onsitelevels); it keeps U at the initial time
even when U(t) is modulated.

Two independent evaluations:

* ``atomic_gf``      -- the closed form: for a later than b on the contour the
  propagator is G^> = -i [p0 e^{-i(th1_a - th1_b)} + p1 e^{-i(th2_a - th2_b)}],
  otherwise (including a == b, i.e. t' = t + 0^+) it is
  G^< = +i [p2 e^{-i(th1_a - th1_b)} + p3 e^{-i(th2_a - th2_b)}], where
  th1 = int eps and th2 = int (eps + U) along the contour.  Exponents are
  combined in log space before exponentiation so the imaginary branch never
  overflows.
* ``atomic_gf_fock`` -- brute force: 4x4 operator matrices, the density matrix
  and the evolution operators multiplied out for each contour ordering.  It is
  the pin for the closed form.

Readings (the paper is silent here): the phase integral of U(t) is a cumulative trapezoid on
the forward grid, backward points copy their forward partner, and imaginary
points use E(t_min) times the complex time elapsed since t_min.
"""
import numpy as np

from .contour import Contour, IMAGINARY


def _u_phase(U_real: np.ndarray, c: Contour) -> np.ndarray:
    """Phi_U(a) = int_{t_min}^{z_a} U(z) dz along the contour."""
    U_real = np.asarray(U_real, dtype=np.float64)
    if U_real.shape != (c.n_real,):
        raise ValueError("U must hold one value per forward time")
    fwd = np.zeros(c.n_real, dtype=np.float64)
    for k in range(1, c.n_real):
        fwd[k] = fwd[k - 1] + 0.5 * (U_real[k] + U_real[k - 1]) * c.dt
    phi = np.zeros(c.n_t, dtype=np.complex128)
    for a in range(c.n_t):
        if c.branch[a] == IMAGINARY:
            phi[a] = U_real[0] * (c.z[a] - c.t_min)
        else:
            phi[a] = fwd[c.tidx[a]]
    return phi


def level_phases(eps: float, U_real: np.ndarray, c: Contour):
    """theta1[a] = int eps dz and theta2[a] = int (eps + U) dz, from t_min to z_a."""
    th1 = eps * (c.z - c.t_min)
    th2 = th1 + _u_phase(U_real, c)
    return th1, th2


def boltzmann_weights(eps: float, U0: float, beta: float):
    """log p_nu for the four number states at the initial time (paper's Z)."""
    energies = np.array([0.0, eps, eps, 2.0 * eps + U0])
    logw = -beta * energies
    shift = logw.max()
    logZ = shift + np.log(np.sum(np.exp(logw - shift)))
    return logw - logZ


def atomic_gf(eps: float, U_real: np.ndarray, c: Contour) -> np.ndarray:
    """Closed-form atomic contour Green's function S[a, b] (N_t x N_t, complex128)."""
    U_real = np.asarray(U_real, dtype=np.float64)
    logp = boltzmann_weights(eps, U_real[0], c.beta)
    th1, th2 = level_phases(eps, U_real, c)
    n = c.n_t
    S = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            d1 = -1j * (th1[a] - th1[b])
            d2 = -1j * (th2[a] - th2[b])
            if a > b:
                S[a, b] = -1j * (np.exp(logp[0] + d1) + np.exp(logp[1] + d2))
            else:
                S[a, b] = 1j * (np.exp(logp[2] + d1) + np.exp(logp[3] + d2))
    return S


def _fock_operators():
    """Annihilator of the up spin in the basis {|0>, |dn>, |up>, |dn up>}.

    |dn up> = c_dn^dag c_up^dag |0>, so c_up |dn up> = -|dn>.
    """
    c = np.zeros((4, 4), dtype=np.complex128)
    c[0, 2] = 1.0     # c_up |up> = |0>
    c[1, 3] = -1.0    # c_up |dn up> = -|dn>
    return c


def atomic_gf_fock(eps: float, U_real: np.ndarray, c: Contour) -> np.ndarray:
    """Brute-force -i Tr[rho T_C c(z_a) c^dag(z_b)] with explicit 4x4 matrices."""
    U_real = np.asarray(U_real, dtype=np.float64)
    cu = _fock_operators()
    cd = cu.conj().T
    E0 = np.array([0.0, eps, eps, 2 * eps + U_real[0]])
    rho = np.diag(np.exp(-c.beta * E0))
    rho = rho / np.trace(rho)
    phiU = _u_phase(U_real, c)
    # Phase of each level accumulated along the contour: int E_nu(z) dz.
    occ = np.array([0.0, 1.0, 1.0, 2.0])
    dbl = np.array([0.0, 0.0, 0.0, 1.0])
    n = c.n_t
    evo = []   # U(z) = exp(-i Phi(z)), Heisenberg c(z) = U(z)^-1 c U(z)
    for a in range(n):
        phase = occ * eps * (c.z[a] - c.t_min) + dbl * phiU[a]
        evo.append((np.diag(np.exp(-1j * phase)), np.diag(np.exp(1j * phase))))
    S = np.zeros((n, n), dtype=np.complex128)
    for a in range(n):
        Ua, Ua_inv = evo[a]
        ca = Ua_inv @ cu @ Ua
        for b in range(n):
            Ub, Ub_inv = evo[b]
            cdb = Ub_inv @ cd @ Ub
            if a > b:
                S[a, b] = -1j * np.trace(rho @ ca @ cdb)
            else:
                S[a, b] = 1j * np.trace(rho @ cdb @ ca)
    return S
