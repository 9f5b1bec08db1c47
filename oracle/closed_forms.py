"""Small-object closed forms for the time-averaged acoustic radiation force.

TEST INFRASTRUCTURE ONLY (part of the oracle package).

Sources in the paper (Castro-Avila et al., arXiv 2404.02346):
  * Gor'kov potential for a sphere in a standing wave, eq. Gorkov_potential_3D,
    with f1 of eq. a_3D and f2 of eq. A_3D;
  * force on a sphere, eq. ARF_Gorkov_3D, and on a cylinder per unit length,
    eq. ARF_Gorkov_2D (the latter with the 2D potential and f1, f2 of
    eqs. a_2D, A_2D);
  * the density-matched rewrite with the contrast factor
    Psi = 1/c0^2 - 1/c_p^2, eqs. expected_arf_3D, expected_arf_2D,
    speeds_factor.

Sign.  The printed force formulas carry a leading minus, but the paper's own
potential gives F = -dU/dx with the opposite sign, so that an object with
Psi > 0 is pushed toward the pressure node.  Here h is the distance of the
object's centre from a pressure antinode (p_in = Pa sin(wt) cos(k h)) and
the force is F_x = -dU/dh; ``gorkov_potential_*`` keeps the paper's U so
the tests check this reading by differentiating it.
"""
from __future__ import annotations

import numpy as np


def contrast_psi(c0: float, cp: float) -> float:
    """Contrast factor Psi(c0, c_p) = 1/c0^2 - 1/c_p^2 (eq. speeds_factor)."""
    return 1.0 / c0 ** 2 - 1.0 / cp ** 2


def f1_f2_3d(rho0, c0, rhop, cp):
    """Monopole and dipole factors of eqs. a_3D and A_3D."""
    f1 = 1.0 - (rho0 * c0 ** 2) / (rhop * cp ** 2)
    f2 = 2.0 * (rhop - rho0) / (2.0 * rhop + rho0)
    return f1, f2


def f1_f2_2d(rho0, c0, rhop, cp):
    """Monopole and dipole factors of eqs. a_2D and A_2D (kappa = 1/(rho c^2))."""
    f1 = 1.0 - (rho0 * c0 ** 2) / (rhop * cp ** 2)
    f2 = (rho0 - rhop) / (rho0 + rhop)
    return f1, f2


def gorkov_potential_3d(h, R, Pa, k, rho0, c0, rhop, cp):
    """Gor'kov potential for a standing wave, eq. Gorkov_potential_3D (as printed)."""
    f1, f2 = f1_f2_3d(rho0, c0, rhop, cp)
    V = 4.0 / 3.0 * np.pi * R ** 3
    return V * Pa ** 2 / (4 * rho0 * c0 ** 2) * (f1 * np.cos(k * h) ** 2
                                                 + 1.5 * f2 * np.sin(k * h) ** 2)


def wei_potential_2d(h, R, Pa, k, rho0, c0, rhop, cp):
    """Two-dimensional potential per unit length (the U printed before eq. ARF_Gorkov_2D)."""
    f1, f2 = f1_f2_2d(rho0, c0, rhop, cp)
    A = np.pi * R ** 2
    return A * Pa ** 2 / (4 * rho0 * c0 ** 2) * (f1 * np.cos(k * h) ** 2
                                                 + f2 * np.sin(k * h) ** 2)


def phi_3d(rho_t, kappa_t):
    """Acoustic contrast of eq. ARF_Gorkov_3D: (5 rho~ - 2)/(2 rho~ + 1) - kappa~."""
    return (5 * rho_t - 2) / (2 * rho_t + 1) - kappa_t


def phi_2d(rho_t, kappa_t):
    """Acoustic contrast of eq. ARF_Gorkov_2D: (3 - rho~)/(1 + rho~) - kappa~."""
    return (3 - rho_t) / (1 + rho_t) - kappa_t


def gorkov_force_3d(h, R, Pa, k, rho0, c0, rhop, cp):
    """Axial force on a sphere at distance h from an antinode (eq. ARF_Gorkov_3D, sign of -dU/dh)."""
    kappa_t = (rho0 * c0 ** 2) / (rhop * cp ** 2)
    return (np.pi * R ** 3 * Pa ** 2 * k / (3 * rho0 * c0 ** 2)
            * phi_3d(rhop / rho0, kappa_t) * np.sin(2 * k * h))


def wei_force_2d(h, R, Pa, k, rho0, c0, rhop, cp):
    """Axial force per length on a cylinder (eq. ARF_Gorkov_2D, sign of -dU/dh)."""
    kappa_t = (rho0 * c0 ** 2) / (rhop * cp ** 2)
    return (np.pi * R ** 2 * Pa ** 2 * k / (4 * rho0 * c0 ** 2)
            * phi_2d(rhop / rho0, kappa_t) * np.sin(2 * k * h))


def matched_force_3d(h, R, Pa, k, rho0, c0, cp):
    """Density-matched sphere, eq. expected_arf_3D with the -dU/dh sign."""
    return np.pi * R ** 3 * Pa ** 2 * k / (3 * rho0) * contrast_psi(c0, cp) * np.sin(2 * k * h)


def matched_force_2d(h, R, Pa, k, rho0, c0, cp):
    """Density-matched cylinder, eq. expected_arf_2D with the -dU/dh sign."""
    return np.pi * R ** 2 * Pa ** 2 * k / (4 * rho0) * contrast_psi(c0, cp) * np.sin(2 * k * h)


def gorkov_scale_3d(R, Pa, k, rho0, c0):
    """F0 = pi R^3 Pa^2 k / (3 rho0 c0^2): with it F/F0 -> f1 sin 2kh as kR -> 0."""
    return np.pi * R ** 3 * Pa ** 2 * k / (3 * rho0 * c0 ** 2)
