"""Motion of a density-matched particle under the radiation force (the paper's outlook: coupling
the force to standard integration algorithms).

The inviscid wave model gives the time-averaged force F(x) on a particle at
rest; the fluid's viscosity enters only through a drag.  In the overdamped
(Stokes) regime the particle's position obeys
    gamma dx/dt = F_x(x),   gamma = 6 pi eta R,
and a particle with Psi > 0 (c_p > c_0) drifts to the pressure node
(kh = pi/2), one with Psi < 0 to the antinode (kh = 0).  Near the stable
point the approach is exponential with rate -F'(x*) / gamma.

The force along x comes from any callable F(kh) (the trained surrogate
through `surrogate_force`, or a closed form); positions are phases kh = k h
measured from the antinode, and F(kh) is extended from [0, pi/2] to all kh
by the standing wave's symmetry: F(-kh) = -F(kh) and F(pi - kh) = -F(kh).
"""
from __future__ import annotations

import math

import numpy as np


def fold(kh):
    """Map kh to [0, pi/2] and the sign of F there, from the symmetries of F(kh) (period pi)."""
    kh = np.asarray(kh, dtype=np.float64)
    r = np.mod(kh, math.pi)                  # period pi in kh
    sign = np.where(r > math.pi / 2, -1.0, 1.0)
    r = np.where(r > math.pi / 2, math.pi - r, r)
    return r, sign


def extended(F_half):
    """F(kh) on all kh from a callable valid on [0, pi/2]."""
    def F(kh):
        r, s = fold(kh)
        return s * np.asarray(F_half(r), dtype=np.float64)
    return F


def integrate(F, kh0, gamma_over_k: float, t_end: float, dt: float):
    """RK4 for dkh/dt = k F(kh) / gamma (overdamped); returns times and phases (one trajectory
    per starting phase in kh0)."""
    kh = np.atleast_1d(np.asarray(kh0, dtype=np.float64)).copy()
    n = int(math.ceil(t_end / dt))
    out = np.empty((n + 1, kh.size))
    out[0] = kh
    rate = 1.0 / gamma_over_k

    def f(x):
        return rate * F(x)

    for i in range(n):
        k1 = f(kh)
        k2 = f(kh + 0.5 * dt * k1)
        k3 = f(kh + 0.5 * dt * k2)
        k4 = f(kh + dt * k3)
        kh = kh + dt * (k1 + 2 * k2 + 2 * k3 + k4) / 6.0
        out[i + 1] = kh
    return np.arange(n + 1) * dt, out


def surrogate_force(mlp, kR: float, ratio: float, R_cells: float, F0: float = 1.0):
    """F(kh) on [0, pi/2] from a trained surrogate network (F/F0 times F0)."""
    from . import surrogate as S

    def F_half(kh):
        kh = np.atleast_1d(kh)
        x = S.normalize(np.full(kh.shape, kR), kh, np.full(kh.shape, ratio),
                        np.full(kh.shape, R_cells))
        return F0 * mlp.predict(x).astype(np.float64).reshape(kh.shape)
    return F_half
