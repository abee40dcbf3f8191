"""Dense gradients of a weighted density loss (oracle; test infrastructure only).

The paper has no gradients; this is the plain adjoint of its lowest-order
Dyson solve.  Loss: L = sum_l w_l n_l(t_end) with t_end the last forward time,
i.e. L = Im sum(Ebar * G) where Ebar holds w_l at ((l, e), (l, b(e))).

With G = (I - S D)^-1 S one has (I - S D)^-1 = I + G D, hence

    dG = (I + G D) dS (I + D G) + G dD G,

so  dL = Im sum(Lam * dS) + Im sum(K * dD)  with
    Lam = (I + G D)^T Ebar (I + D G)^T  and  K = G^T Ebar G^T.

dS is block diagonal: each site's closed-form atomic Green's function (Sec. III)
depends on its level eps_j = V_j - U(t_min)/2 - mu (eq. onsitelevels) and on
U(t) through the Boltzmann weights and the phase integral.  dD/dJ(z_c) has
w_c on every bond at contour point c; the gradient with respect to J at a
physical time sums the forward, backward and (at t_min) imaginary points that
carry it.
"""
import numpy as np

from .atomic import atomic_gf, boltzmann_weights, level_phases
from .contour import Contour, IMAGINARY
from .dyson import blockdiag, dyson_dense
from .lattice import neighbours, hopping_on_contour, hopping_operator_dense


def site_levels(V: np.ndarray, U_real: np.ndarray, mu: float) -> np.ndarray:
    """eps_i = V_i - U(t_min)/2 - mu (eq. onsitelevels)."""
    return np.asarray(V, dtype=np.float64) - 0.5 * float(U_real[0]) - mu


def _phase_u_jacobian(c: Contour) -> np.ndarray:
    """dPhi_U(a) / dU_k for the trapezoid phase of atomic.py, shape (N_t, N_real)."""
    jac = np.zeros((c.n_t, c.n_real), dtype=np.complex128)
    for a in range(c.n_t):
        if c.branch[a] == IMAGINARY:
            jac[a, 0] = c.z[a] - c.t_min
            continue
        m = c.tidx[a]
        for k in range(1, m + 1):
            jac[a, k] += 0.5 * c.dt
            jac[a, k - 1] += 0.5 * c.dt
    return jac


def atomic_gf_derivatives(eps: float, U_real: np.ndarray, c: Contour):
    """(dS/deps at fixed U, dS/dU_k at fixed eps for every k), closed form.

    S[a,b] is a sum of terms T_nu = (-/+ i) exp(log p_nu + d(a,b)): nu = 0, 1 for
    a > b and nu = 2, 3 otherwise, with d = -i (th_a - th_b) using th1 for
    nu in {0, 2} and th2 for nu in {1, 3}.
    d log p_nu / d eps = -beta (N_nu - <N>),  N = (0, 1, 1, 2);
    d log p_nu / d U0  = -beta (D_nu - <D>),  D = (0, 0, 0, 1);
    d th1 / d eps = d th2 / d eps = z - t_min;   d th2 / d U_k = dPhi_U / dU_k.
    """
    U_real = np.asarray(U_real, dtype=np.float64)
    logp = boltzmann_weights(eps, U_real[0], c.beta)
    p = np.exp(logp)
    Nn = np.array([0.0, 1.0, 1.0, 2.0])
    Dn = np.array([0.0, 0.0, 0.0, 1.0])
    dlogp_de = -c.beta * (Nn - np.dot(p, Nn))
    dlogp_dU0 = -c.beta * (Dn - np.dot(p, Dn))
    th1, th2 = level_phases(eps, U_real, c)
    jac = _phase_u_jacobian(c)
    dz = c.z - c.t_min
    n = c.n_t
    dS_de = np.zeros((n, n), dtype=np.complex128)
    dS_dU = np.zeros((c.n_real, n, n), dtype=np.complex128)
    for a in range(n):
        for b in range(n):
            d1 = -1j * (th1[a] - th1[b])
            d2 = -1j * (th2[a] - th2[b])
            dd_de = -1j * (dz[a] - dz[b])
            dd2_dU = -1j * (jac[a] - jac[b])          # vector over k
            if a > b:
                pref, nu1, nu2 = -1j, 0, 1
            else:
                pref, nu1, nu2 = 1j, 2, 3
            t1 = pref * np.exp(logp[nu1] + d1)
            t2 = pref * np.exp(logp[nu2] + d2)
            dS_de[a, b] = t1 * (dlogp_de[nu1] + dd_de) + t2 * (dlogp_de[nu2] + dd_de)
            dS_dU[:, a, b] = t2 * dd2_dU
            dS_dU[0, a, b] += t1 * dlogp_dU0[nu1] + t2 * dlogp_dU0[nu2]
    return dS_de, dS_dU


def loss_and_grad_dense(V, U_real, J_real, mu, Lx, Ly, periodic, c: Contour, w_loss):
    """L and (dL/dV [N_r], dL/dU [N_real], dL/dJ [N_real]) by dense linear algebra.

    dL/dU is the total derivative: it includes the dependence of every eps_i on
    U(t_min) through eq. onsitelevels.
    """
    V = np.asarray(V, dtype=np.float64)
    U_real = np.asarray(U_real, dtype=np.float64)
    J_real = np.asarray(J_real, dtype=np.float64)
    w_loss = np.asarray(w_loss, dtype=np.float64)
    n_r = Lx * Ly
    n_t = c.n_t
    eps = site_levels(V, U_real, mu)
    S_blocks = np.stack([atomic_gf(e, U_real, c) for e in eps])
    D = hopping_operator_dense(Lx, Ly, periodic, J_real, c)
    G = dyson_dense(S_blocks, D)
    e_idx = c.n_real - 1
    be = int(c.partner(e_idx))
    N = n_r * n_t
    Ebar = np.zeros((N, N), dtype=np.complex128)
    for l in range(n_r):
        Ebar[l * n_t + e_idx, l * n_t + be] = w_loss[l]
    L = float(np.imag(np.sum(Ebar * G)))
    I = np.eye(N, dtype=np.complex128)
    P = I + G @ D
    Q = I + D @ G
    Lam = P.T @ Ebar @ Q.T
    K = G.T @ Ebar @ G.T

    dV = np.zeros(n_r)
    dU = np.zeros(c.n_real)
    for j in range(n_r):
        blk = Lam[j * n_t:(j + 1) * n_t, j * n_t:(j + 1) * n_t]
        dS_de, dS_dU = atomic_gf_derivatives(eps[j], U_real, c)
        g_eps = float(np.imag(np.sum(blk * dS_de)))
        dV[j] = g_eps
        dU += np.imag(np.einsum("ab,kab->k", blk, dS_dU))
        dU[0] += -0.5 * g_eps          # eps_j = V_j - U(t_min)/2 - mu

    nbr = neighbours(Lx, Ly, periodic)
    dJc = np.zeros(n_t)
    for i in range(n_r):
        for k in nbr[i]:
            if k < 0:
                continue
            for a in range(n_t):
                dJc[a] += float(np.imag(K[i * n_t + a, k * n_t + a] * c.w[a]))
    dJ = np.zeros(c.n_real)
    for a in range(n_t):
        if c.branch[a] == IMAGINARY:
            dJ[0] += dJc[a]
        else:
            dJ[c.tidx[a]] += dJc[a]
    return L, dV, dU, dJ


def loss_dense(V, U_real, J_real, mu, Lx, Ly, periodic, c: Contour, w_loss) -> float:
    """L alone (for finite-difference pins)."""
    eps = site_levels(V, U_real, mu)
    S_blocks = np.stack([atomic_gf(e, U_real, c) for e in eps])
    D = hopping_operator_dense(Lx, Ly, periodic, J_real, c)
    G = dyson_dense(S_blocks, D)
    n_t = c.n_t
    e_idx = c.n_real - 1
    be = int(c.partner(e_idx))
    return float(sum(w_loss[l] * np.imag(G[l * n_t + e_idx, l * n_t + be])
                     for l in range(Lx * Ly)))


__all__ = ["site_levels", "atomic_gf_derivatives", "loss_and_grad_dense", "loss_dense",
           "blockdiag", "hopping_on_contour"]
