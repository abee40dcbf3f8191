"""Discretised Kadanoff-Baym-Keldysh contour (oracle; test infrastructure only).

Paper: Sec. IV.A ("Representation of the Green's functions and self-energies")
and the caption of Fig. 1.  The contour starts at the first real time t_min,
runs forward to t_max, back to t_min, and then down the imaginary axis to
t_min - i beta, where the thermal initial state lives.  N_t = 2 N_real + N_imag.

The paper does not fix where the points sit or which quadrature is used; this
module takes the following reading:

* forward  a in [0, N_real):          z_a = t_min + a dt,              w_a = +dt
* backward a in [N_real, 2 N_real):   z_a = t_min + (2N_real-1-a) dt,   w_a = -dt
* imaginary a = 2 N_real + m:         z_a = t_min - i (m+1) dtau,       w_a = -i dtau
  with dtau = beta / N_imag.

Contour order is index order; the same-time partner of a forward point a is
the backward point 2 N_real - 1 - a.  Contour integrals are Riemann sums with
the weights w_a (rectangle rule), so results converge as O(dt).
"""
from dataclasses import dataclass

import numpy as np

FORWARD, BACKWARD, IMAGINARY = 0, 1, 2


@dataclass(frozen=True)
class Contour:
    n_real: int
    n_imag: int
    dt: float
    beta: float
    t_min: float
    z: np.ndarray       # complex contour coordinate of each point
    w: np.ndarray       # complex quadrature weight of each point
    branch: np.ndarray  # FORWARD / BACKWARD / IMAGINARY
    tidx: np.ndarray    # forward-grid index of the point's physical time (0 on the imaginary branch)

    @property
    def n_t(self) -> int:
        return 2 * self.n_real + self.n_imag

    @property
    def dtau(self) -> float:
        return self.beta / self.n_imag

    def partner(self, a):
        """Backward point at the same physical time as forward point a (t + 0^+)."""
        return 2 * self.n_real - 1 - np.asarray(a)

    def real_times(self) -> np.ndarray:
        return self.t_min + self.dt * np.arange(self.n_real)


def make_contour(n_real: int, n_imag: int, dt: float, beta: float,
                 t_min: float = 0.0) -> Contour:
    if n_real < 1 or n_imag < 1:
        raise ValueError("need n_real >= 1 and n_imag >= 1")
    n_t = 2 * n_real + n_imag
    dtau = beta / n_imag
    z = np.zeros(n_t, dtype=np.complex128)
    w = np.zeros(n_t, dtype=np.complex128)
    branch = np.zeros(n_t, dtype=np.int64)
    tidx = np.zeros(n_t, dtype=np.int64)
    for a in range(n_t):
        if a < n_real:
            tidx[a] = a
            z[a] = t_min + a * dt
            w[a] = dt
            branch[a] = FORWARD
        elif a < 2 * n_real:
            tidx[a] = 2 * n_real - 1 - a
            z[a] = t_min + tidx[a] * dt
            w[a] = -dt
            branch[a] = BACKWARD
        else:
            m = a - 2 * n_real
            tidx[a] = 0
            z[a] = t_min - 1j * (m + 1) * dtau
            w[a] = -1j * dtau
            branch[a] = IMAGINARY
    return Contour(n_real, n_imag, float(dt), float(beta), float(t_min),
                   z, w, branch, tidx)
