"""Seeded synthetic workloads for the trapped-lattice Dyson solve.

Input generation only: this module holds none of the method's arithmetic (no
contour, no Green's function, no Dyson step).  It produces the model
parameters of the paper's Hamiltonian (eq. model, eq. onsitelevels) -- trap
potential V_i, interaction U(t) and hopping J(t) on the forward time grid,
inverse temperature, chemical potential and contour sizes -- for five named
workloads that stand in for the paper's Wannier-derived lattice-depth
modulation runs (Sec. V), whose inputs are not available.  Both the HIP
library and the CPU oracle are fed from here.

Geometry: site i = x * Ly + y, trap V_i = k |r_i|^2 with r_i measured from the
lattice centre ((Lx-1)/2, (Ly-1)/2), so C4v holds about the centre of the
lattice (a plaquette centre for even L).
"""
from dataclasses import dataclass, field

import numpy as np

LOSS_SEED = 1309
SAMPLE_SEED = 5994


@dataclass(frozen=True)
class Workload:
    name: str
    Lx: int
    Ly: int
    periodic: bool
    n_real: int
    n_imag: int
    dt: float
    beta: float
    mu: float
    t_min: float
    V: np.ndarray = field(repr=False)
    U: np.ndarray = field(repr=False)
    J: np.ndarray = field(repr=False)
    block_sites: int = 0
    note: str = ""

    @property
    def n_r(self) -> int:
        return self.Lx * self.Ly

    @property
    def n_t(self) -> int:
        return 2 * self.n_real + self.n_imag

    def forward_times(self) -> np.ndarray:
        return self.t_min + self.dt * np.arange(self.n_real)


def trap_potential(Lx: int, Ly: int, curvature: float) -> np.ndarray:
    x = np.arange(Lx)[:, None] - 0.5 * (Lx - 1)
    y = np.arange(Ly)[None, :] - 0.5 * (Ly - 1)
    return (curvature * (x * x + y * y)).reshape(-1).astype(np.float64)


def _make(name, L, U0, J0, beta, k, n_real, n_imag, dt=0.1, mu=0.0, block_sites=0,
          U_t=None, J_t=None, note=""):
    t = dt * np.arange(n_real)
    U = np.full(n_real, U0, dtype=np.float64) if U_t is None else U_t(t)
    J = np.full(n_real, J0, dtype=np.float64) if J_t is None else J_t(t)
    return Workload(name=name, Lx=L, Ly=L, periodic=False, n_real=n_real, n_imag=n_imag,
                    dt=dt, beta=beta, mu=mu, t_min=0.0, V=trap_potential(L, L, k),
                    U=np.asarray(U, dtype=np.float64), J=np.asarray(J, dtype=np.float64),
                    block_sites=block_sites or L * L, note=note)


def modulation(amplitude: float):
    """U(t) = 1 + A sin 2t and J(t) = 0.1 (1 - 2 A sin 2t): one lattice-depth knob."""
    return (lambda t: 1.0 + amplitude * np.sin(2.0 * t),
            lambda t: 0.1 * (1.0 - 2.0 * amplitude * np.sin(2.0 * t)))


def config(k: int, amplitude: float = 0.1) -> Workload:
    """The five named workloads (1-based)."""
    if k == 1:
        return _make("trap4x4_nt50", 4, 1.0, 0.05, 5.0, 0.02, 20, 10,
                     note="4x4 open, full 800x800 G, FP64")
    if k == 2:
        return _make("trap16x16_nt144", 16, 1.0, 0.08, 10.0, 0.01, 64, 16,
                     note="16x16 open, all G_ij, FP64 to 1e-12")
    if k == 3:
        return _make("trap24x24_nt176", 24, 1.0, 0.1, 10.0, 0.008, 80, 16, block_sites=64,
                     note="24x24 open, 64-site column blocks, FP64 vs mixed")
    if k == 4:
        return _make("trap12x12_nt112", 12, 1.0, 0.06, 8.0, 0.015, 48, 16,
                     note="12x12 open, density-loss gradients")
    if k == 5:
        U_t, J_t = modulation(amplitude)
        return _make("trap32x32_nt208_mod", 32, 1.0, 0.1, 10.0, 0.005, 96, 16,
                     block_sites=128, U_t=U_t, J_t=J_t,
                     note="32x32 open, lattice-depth modulation, 128-site blocks")
    raise ValueError("workloads are numbered 1..5")


def custom(Lx, Ly, n_real, n_imag, *, U0=1.0, J0=0.05, beta=5.0, curvature=0.02, dt=0.1,
           mu=0.0, periodic=False, t_min=0.0, seed=None, name="custom") -> Workload:
    """Small test lattices; with a seed, V gets a reproducible random offset."""
    V = trap_potential(Lx, Ly, curvature)
    if seed is not None:
        V = V + 0.05 * np.random.default_rng(seed).standard_normal(Lx * Ly)
    t = t_min + dt * np.arange(n_real)
    return Workload(name=name, Lx=Lx, Ly=Ly, periodic=periodic, n_real=n_real,
                    n_imag=n_imag, dt=dt, beta=beta, mu=mu, t_min=t_min, V=V,
                    U=np.full(n_real, U0), J=np.full(n_real, J0) + 0.0 * t,
                    block_sites=Lx * Ly)


def loss_weights(n_r: int) -> np.ndarray:
    """w_i ~ U(0, 1) for the density loss sum_i w_i n_i(t_end)."""
    return np.random.default_rng(LOSS_SEED).random(n_r)


def sample_sources(wl: Workload, n_random: int = 8) -> list:
    """Seeded source sites for column-sampled checks: random sites plus the
    centre, a corner, an edge midpoint and the site whose trap energy is
    closest to U(t_min)/2 + mu (the ring where the on-site level is near zero)."""
    rng = np.random.default_rng(SAMPLE_SEED)
    picks = [int(s) for s in rng.choice(wl.n_r, size=min(n_random, wl.n_r), replace=False)]
    cx, cy = wl.Lx // 2, wl.Ly // 2
    picks += [cx * wl.Ly + cy, 0, (wl.Lx // 2) * wl.Ly + 0,
              int(np.argmin(np.abs(wl.V - (0.5 * wl.U[0] + wl.mu))))]
    out = []
    for s in picks:
        if s not in out:
            out.append(s)
    return out
