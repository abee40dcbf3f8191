"""Second-order strong-coupling self-energy and its self-consistency (oracle;
test infrastructure only).

Paper: Sec. III, eq. selfcons, eq. defnSigma, eq. defnSigmatilde,
eq. cumulanttabulation and eq. Sigmamix.

* The on-site two-particle propagator
      G^II_{s s~}(t1, t2; t1', t2') = (-i)^2 <T_C c_s(t1) c_s~(t2) c^dag_s~(t1') c^dag_s(t2')>
  of the atomic Hamiltonian eps (n_up + n_dn) + U(t) n_up n_dn is evaluated by
  brute force in the four-state Fock space |0>, |dn>, |up>, |up dn> = c^dag_up
  c^dag_dn |0> (the paper's number basis): Heisenberg operators
  O(z) = e^{i Theta(z)} O e^{-i Theta(z)} with the diagonal phases
  Theta_nu(z) = int E_nu dz along the contour (the tabulated zeta of
  eq. cumulanttabulation), contour ordering with the fermionic sign, and the
  trace with the initial Boltzmann weights.
* Its second-order cumulant  G~ = G^II + G(t1,t1') G(t2,t2') delta_{s s~}
  - G(t1,t2') G(t2,t1')  vanishes for U = 0 (Wick's theorem).
* Sigma~(t, t') = - sum_{s1} sum_{c, d} w_c w_d G~_{s s1}(t, z_d; z_c, t')
  J(z_c) K(z_c, z_d) J(z_d),  K = sum over the site's neighbours of their
  local Green's function (eq. defnSigmatilde, contour integrals as weighted
  sums; paramagnetic, so both spins of the neighbours carry the same G).
* Sigma = calG^-1 o Sigma~ o calG^-1 (eq. defnSigma) enters eq. Glatt through
  the block diagonal B = calG^-1 - Sigma.  With the contour product
  (A o B) = A W B, W = diag(w), whose unit is W^-1, its inverse block is
      B^-1 (contour) = S (S - Sigma~)^-1 S   (plain matrices),
  so the lattice solve is the lowest-order one with S replaced by that block.
* The loop (Sec. III): Sigma~ = 0; G_loc from the lattice solve; Sigma~_new;
  mix Sigma~ = lam Sigma~_new + (1 - lam) Sigma~_old (eq. Sigmamix; Sigma is
  linear in Sigma~ at fixed S); stop when
  |Delta|_F / N_bd + |Delta|_max <= delta_sc, N_bd = N_r N_t^2 entries.

Readings (listed with the others in the design notes): contour ordering at
equal contour indices places creation operators later than annihilation
operators (t' = t + 0^+, as for G at equal index), operators of one kind at
one index keep their written order; the convergence norm is taken on
Sigma~ (Sigma is a fixed linear image of it).
"""
import numpy as np

from .atomic import boltzmann_weights, level_phases, atomic_gf
from .dyson import dyson_dense
from .lattice import neighbours, hopping_on_contour, hopping_operator_dense
from .contour import Contour


def fock_annihilators():
    """c_up, c_dn as 4x4 matrices in the basis |0>, |dn>, |up>, |up dn>."""
    c_dn = np.zeros((4, 4))
    c_up = np.zeros((4, 4))
    c_dn[0, 1] = 1.0          # |dn> -> |0>
    c_dn[2, 3] = -1.0         # c_dn c^dag_up c^dag_dn |0> = -|up>
    c_up[0, 2] = 1.0          # |up> -> |0>
    c_up[1, 3] = 1.0          # c_up c^dag_up c^dag_dn |0> = |dn>
    return {"up": c_up, "dn": c_dn}


def state_phases(eps: float, U_real: np.ndarray, c: Contour) -> np.ndarray:
    """Theta_nu(z_a) for nu = 0..3 (energies 0, eps, eps, 2 eps + U(t)), shape (4, N_t)."""
    th1, th2 = level_phases(eps, U_real, c)
    return np.stack([np.zeros(c.n_t, dtype=complex), th1, th1, th1 + th2])


def two_particle_gf(eps: float, U_real: np.ndarray, c: Contour, s: str, s2: str,
                    idx=None) -> np.ndarray:
    """G^II_{s s2}(a1, a2; b1, b2) on the contour grid.

    Returns an array of shape (N_t,)*4 indexed [a1, a2, b1, b2], or the values
    at the listed index quadruples idx (array of shape (M, 4)).
    """
    U_real = np.asarray(U_real, dtype=np.float64)
    ops = fock_annihilators()
    Theta = state_phases(eps, U_real, c)                     # (4, N_t)
    p = np.exp(boltzmann_weights(eps, U_real[0], c.beta))    # initial weights
    # Heisenberg matrices per (operator kind, contour point): kinds
    # 0: c_s, 1: c_s2, 2: c^dag_s2, 3: c^dag_s
    mats = [ops[s], ops[s2], ops[s2].T, ops[s].T]
    H = np.zeros((4, c.n_t, 4, 4), dtype=complex)
    for k, O in enumerate(mats):
        for a in range(c.n_t):
            H[k, a] = np.exp(1j * Theta[:, a])[:, None] * O * np.exp(-1j * Theta[:, a])[None, :]
    if idx is None:
        grid = np.indices((c.n_t,) * 4).reshape(4, -1).T
    else:
        grid = np.asarray(idx, dtype=np.int64).reshape(-1, 4)
    M = grid.shape[0]
    # Contour order: later point leftmost; at equal index creators are later;
    # equal (index, kind class) keeps the written order (stable sort).
    is_creator = np.array([0, 0, 1, 1])
    key = grid * 2 + is_creator[None, :]
    order = np.argsort(-key, axis=1, kind="stable")          # (M, 4)
    # parity of each permutation
    perm = order.copy()
    sign = np.ones(M)
    for i in range(4):
        for j in range(i + 1, 4):
            sign *= np.where(perm[:, i] > perm[:, j], -1.0, 1.0)
    prod = np.broadcast_to(np.eye(4, dtype=complex), (M, 4, 4)).copy()
    for pos in range(4):
        kind = order[:, pos]
        point = grid[np.arange(M), kind]
        prod = prod @ H[kind, point]
    trace = np.einsum("n,mnn->m", p, prod)
    val = (-1j) ** 2 * sign * trace
    return val.reshape((c.n_t,) * 4) if idx is None else val


def cumulant(eps: float, U_real: np.ndarray, c: Contour, s: str, s2: str,
             S_site: np.ndarray = None) -> np.ndarray:
    """G~_{s s2}[a1, a2, b1, b2] = G^II + G(a1,b1) G(a2,b2) delta - G(a1,b2) G(a2,b1)."""
    G2 = two_particle_gf(eps, U_real, c, s, s2)
    S1 = atomic_gf(eps, U_real, c) if S_site is None else S_site
    out = G2 - np.einsum("ad,bc->abcd", S1, S1)               # - G(a1,b2) G(a2,b1)
    if s == s2:
        out = out + np.einsum("ac,bd->abcd", S1, S1)          # + G(a1,b1) G(a2,b2)
    return out


def sigma_tilde(V, U_real, mu, J_real, c: Contour, Lx: int, Ly: int, periodic: bool,
                G_loc: np.ndarray) -> np.ndarray:
    """Sigma~_i[t, t'] for every site from the local Green's functions G_loc[i]
    (eq. defnSigmatilde), shape (N_r, N_t, N_t)."""
    U_real = np.asarray(U_real, dtype=np.float64)
    eps = np.asarray(V, dtype=np.float64) - 0.5 * U_real[0] - mu
    nbr = neighbours(Lx, Ly, periodic)
    wJ = c.w * hopping_on_contour(J_real, c)                 # w_c J(z_c)
    out = np.zeros((Lx * Ly, c.n_t, c.n_t), dtype=complex)
    for i in range(Lx * Ly):
        K = np.zeros((c.n_t, c.n_t), dtype=complex)
        for k in nbr[i]:
            if k >= 0:
                K += G_loc[k]
        K = wJ[:, None] * K * wJ[None, :]                    # w_c J_c K(c, d) J_d w_d
        Gt = cumulant(eps[i], U_real, c, "up", "up") + cumulant(eps[i], U_real, c, "up", "dn")
        # Sigma~(a, b) = - sum_{c, d} G~(a, d; c, b) K(c, d)
        out[i] = -np.einsum("adcb,cd->ab", Gt, K)
    return out


def sigma_tilde_entries(V, U_real, mu, J_real, c: Contour, Lx: int, Ly: int, periodic: bool,
                        G_loc: np.ndarray, entries) -> np.ndarray:
    """Sigma~_i(a, b) of eq. defnSigmatilde at the listed (i, a, b) only: the
    same contraction as sigma_tilde, restricted to those outputs, for contour
    lengths where the whole N_t^4 table does not fit in memory."""
    U_real = np.asarray(U_real, dtype=np.float64)
    eps = np.asarray(V, dtype=np.float64) - 0.5 * U_real[0] - mu
    nbr = neighbours(Lx, Ly, periodic)
    wJ = c.w * hopping_on_contour(J_real, c)
    n = c.n_t
    cc, dd = (x.ravel() for x in np.meshgrid(np.arange(n), np.arange(n), indexing="ij"))
    out = []
    for i, a, b in entries:
        K = np.zeros((n, n), dtype=complex)
        for k in nbr[i]:
            if k >= 0:
                K += G_loc[k]
        K = wJ[:, None] * K * wJ[None, :]
        S1 = atomic_gf(eps[i], U_real, c)
        # G~(a, d; c, b) for all (c, d): operator points (a1, a2, b1, b2) = (a, d, c, b)
        idx = np.stack([np.full(n * n, a), dd, cc, np.full(n * n, b)], axis=1)
        Gt = np.zeros(n * n, dtype=complex)
        for s2 in ("up", "dn"):
            Gt += two_particle_gf(eps[i], U_real, c, "up", s2, idx)
            Gt -= S1[a, b] * S1[dd, cc]                        # - G(a1, b2) G(a2, b1)
            if s2 == "up":
                Gt += S1[a, cc] * S1[dd, b]                    # + G(a1, b1) G(a2, b2)
        out.append(-np.sum(Gt * K[cc, dd]))
    return np.array(out)


def dressed_blocks(S: np.ndarray, Sig_t: np.ndarray) -> np.ndarray:
    """B_i^-1 (contour inverse) = S_i (S_i - Sigma~_i)^-1 S_i per site."""
    return np.stack([S[i] @ np.linalg.solve(S[i] - Sig_t[i], S[i]) for i in range(S.shape[0])])


def selfconsistent(V, U_real, mu, J_real, c: Contour, Lx: int, Ly: int, periodic: bool = False,
                   lam: float = 0.7, delta_sc: float = 1e-10, max_iter: int = 50):
    """The self-consistency loop of Sec. III on a small lattice with the dense
    lattice solve.  Returns (Sigma~, G, history of the convergence norm)."""
    U_real = np.asarray(U_real, dtype=np.float64)
    eps = np.asarray(V, dtype=np.float64) - 0.5 * U_real[0] - mu
    S = np.stack([atomic_gf(e, U_real, c) for e in eps])
    D = hopping_operator_dense(Lx, Ly, periodic, J_real, c)
    n_r, n_t = S.shape[0], c.n_t
    sig = np.zeros_like(S)
    hist = []
    G = None
    for _ in range(max_iter):
        G = dyson_dense(dressed_blocks(S, sig), D)
        G_loc = np.stack([G[i * n_t:(i + 1) * n_t, i * n_t:(i + 1) * n_t] for i in range(n_r)])
        new = sigma_tilde(V, U_real, mu, J_real, c, Lx, Ly, periodic, G_loc)
        diff = new - sig
        hist.append(np.linalg.norm(diff) / (n_r * n_t * n_t) + np.abs(diff).max())
        sig = lam * new + (1.0 - lam) * sig
        if hist[-1] <= delta_sc:
            break
    G = dyson_dense(dressed_blocks(S, sig), D)
    return sig, G, hist
