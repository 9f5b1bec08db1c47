"""Seeded synthetic inputs shared by the GPU library's callers and the oracle.

This module holds none of the method's arithmetic: it only lays out
parameter sets, surface point sets and seeded random draws.  Quantities that
need the method itself (the antinode position and wavenumber of the driven
standing wave) are passed in by the caller, from the oracle's calibration in
the tests and from the GPU library's calibration in the benchmark.

A problem is a plain dict with the keys of the C descriptor:
  dim, nx, ny, nz, xbc ("driven" | "periodic"), c0, rho0, center (3,),
  radius, cp, d, rho_a, omega, wall_phi, surf_xyz (N,3), surf_normal (N,3),
  surf_area (N,), avg_start, and for convenience n_steps, lam, kh.

Workloads (lattice units, rho0 = 1, source amplitude rho_a = 1, Phi = 0.99,
d = 4; the paper's set-up in Sec. "Results and discussion"):
  * cylinder_2d: 128 x 64 D2Q5, lambda = 128, c0 = 0.5, R = 8, c_p = 1.2 c0,
    64 surface points, object lambda/8 from the central antinode, 20 periods,
    average over the last 5;
  * sphere_3d: 256 x 128 x 128 D3Q7, lambda = 256, c0 = 0.5, R = 12,
    c_p = 1.1 c0, 2048 Fibonacci points, 30 periods, average over the last
    10, 16 positions kh_j = j (pi/2)/15;
  * batch: seeded boxes with edge in {64, 96, 128, 192} (cubic, lambda =
    edge), R ~ U[4, 16], c_p/c0 ~ U[0.8, 1.5], kh ~ U[0, pi/2], c0 = 1/3.
The integration surface sits two cells outside the object's radius.
"""
from __future__ import annotations

import math

import numpy as np

SURFACE_OFFSET = 2.0   # integration radius R_s = R + 2 (in the fluid)
KERNEL_REACH = 1.5     # the 3-point kernel touches nodes within 1.5 cells


def circle_surface(center, Rs: float, N: int):
    """N equal segments of a circle: centres at angles 2 pi (k + 1/2)/N."""
    th = 2.0 * np.pi * (np.arange(N) + 0.5) / N
    nrm = np.stack([np.cos(th), np.sin(th), np.zeros(N)], axis=1)
    xyz = np.asarray(center, dtype=np.float64)[None, :3] + Rs * nrm
    xyz[:, 2] = 0.0
    area = np.full(N, 2.0 * np.pi * Rs / N)
    return xyz, nrm, area


def fibonacci_surface(center, Rs: float, N: int):
    """N Fibonacci points on a sphere, polar axis along x, equal areas."""
    k = np.arange(N, dtype=np.float64)
    u = 1.0 - (2.0 * k + 1.0) / N
    phi = k * np.pi * (3.0 - np.sqrt(5.0))
    s = np.sqrt(np.maximum(0.0, 1.0 - u * u))
    nrm = np.stack([u, s * np.cos(phi), s * np.sin(phi)], axis=1)
    xyz = np.asarray(center, dtype=np.float64)[None, :3] + Rs * nrm
    area = np.full(N, 4.0 * np.pi * Rs * Rs / N)
    return xyz, nrm, area


def _problem(dim, nx, ny, nz, c0, cp, R, center, lam, n_periods, avg_periods, n_surf,
             rho_a=1.0, wall_phi=0.99, d=4.0, kh=None):
    period = lam / c0
    assert abs(period - round(period)) < 1e-9, "the drive period must be a whole number of steps"
    period = int(round(period))
    Rs = R + SURFACE_OFFSET
    if dim == 2:
        xyz, nrm, area = circle_surface(center, Rs, n_surf)
    else:
        xyz, nrm, area = fibonacci_surface(center, Rs, n_surf)
    return {
        "dim": dim, "nx": nx, "ny": ny, "nz": nz if dim == 3 else 1, "xbc": "driven",
        "c0": c0, "rho0": 1.0, "center": tuple(float(v) for v in center), "radius": float(R),
        "cp": float(cp), "d": d, "rho_a": rho_a, "omega": 2.0 * np.pi * c0 / lam,
        "wall_phi": wall_phi, "surf_xyz": xyz, "surf_normal": nrm, "surf_area": area,
        "avg_start": (n_periods - avg_periods) * period, "n_steps": n_periods * period,
        "lam": float(lam), "period": period, "kh": kh,
    }


def cylinder_2d(x_mid: float, k: float, n_periods: int = 20, avg_periods: int = 5,
                cp_ratio: float = 1.2, R: float = 8.0, kh: float = math.pi / 4):
    """The 2D cylinder workload (object at lambda/8 from the central antinode)."""
    nx, ny, lam, c0 = 128, 64, 128.0, 0.5
    center = (x_mid + kh / k, ny / 2.0, 0.0)
    return _problem(2, nx, ny, 1, c0, cp_ratio * c0, R, center, lam, n_periods, avg_periods,
                    64, kh=kh)


def sphere_3d_positions(n: int = 16):
    """kh_j = j (pi/2)/(n-1), j = 0 .. n-1."""
    return [j * (math.pi / 2.0) / (n - 1) for j in range(n)]


def sphere_3d(x_mid: float, k: float, kh: float, n_periods: int = 30, avg_periods: int = 10,
              shape=(256, 128, 128), lam: float = 256.0, R: float = 12.0, cp_ratio: float = 1.1,
              n_surf: int = 2048, c0: float = 0.5):
    """The 3D sphere workload at phase kh (shape and lam overridable for small cases)."""
    nx, ny, nz = shape
    center = (x_mid + kh / k, ny / 2.0, nz / 2.0)
    return _problem(3, nx, ny, nz, c0, cp_ratio * c0, R, center, lam, n_periods, avg_periods,
                    n_surf, kh=kh)


BATCH_EDGES = (64, 96, 128, 192)
BATCH_C0 = 1.0 / 3.0


def geometry_ok(p: dict) -> bool:
    """True when every surface stencil stays off the x sheets and inside y, z."""
    xyz = np.asarray(p["surf_xyz"])
    lo = np.ceil(xyz[:, 0] - KERNEL_REACH).min()
    hi = np.floor(xyz[:, 0] + KERNEL_REACH).max()
    if lo < 2 or hi > p["nx"] - 3:
        return False
    rs = p["radius"] + SURFACE_OFFSET + KERNEL_REACH
    if 2 * rs >= p["ny"] or (p["dim"] == 3 and 2 * rs >= p["nz"]):
        return False
    return True


def batch(seed: int, n: int, x_mid_by_edge: dict, k_by_edge: dict, n_periods: int = 30,
          avg_periods: int = 10, n_surf: int = 2048, kr_max: float | None = None,
          edges=BATCH_EDGES, return_draws: bool = False):
    """Seeded uneven batch of 3D boxes (numpy PCG64 stream ``seed``).

    Each draw takes (edge, R, c_p/c0, kh) in that order; a draw whose
    surface stencil would touch an x sheet, or (when ``kr_max`` is given)
    whose k R exceeds it, is redrawn from the same stream.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out, draws, rejected = [], [], 0
    while len(out) < n:
        edge = int(rng.choice(np.asarray(edges)))
        R = float(rng.uniform(4.0, 16.0))
        ratio = float(rng.uniform(0.8, 1.5))
        kh = float(rng.uniform(0.0, math.pi / 2.0))
        lam = float(edge)
        if kr_max is not None and 2.0 * math.pi * R / lam > kr_max:
            rejected += 1
            continue
        k = k_by_edge[edge]
        center = (x_mid_by_edge[edge] + kh / k, edge / 2.0, edge / 2.0)
        p = _problem(3, edge, edge, edge, BATCH_C0, ratio * BATCH_C0, R, center, lam,
                     n_periods, avg_periods, n_surf, kh=kh)
        p["cp_ratio"] = ratio
        if not geometry_ok(p):
            rejected += 1
            continue
        out.append(p)
        draws.append((edge, R, ratio, kh))
    if return_draws:
        return out, {"draws": draws, "rejected": rejected}
    return out


CHANNEL_WIDTH = 64     # the paper's L_y = L_z = 64 (Sec. Results and discussion)


def channel_draws(seed: int, n: int, kr_range=(0.05, 2.0 * math.pi * 4.0 / 192.0),
                  lam_step: int = 8):
    """Seeded draws (lambda, R, c_p/c0, kh) for boxes lambda x 64 x 64 at small k R.

    Each draw takes k R ~ U[kr_range), R ~ U[4, 16], c_p/c0 ~ U[0.8, 1.5], kh ~ U[0, pi/2]
    in that order (numpy PCG64 stream ``seed``); lambda = 2 pi R / k R is rounded to a
    multiple of lam_step (so that draws share calibrations), and a draw whose k R = 2 pi R /
    lambda then leaves kr_range is redrawn.  Objects of R <= 16 with their integration
    surface fit across 64 cells and away from the x sheets for every kh at these lengths.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out, rejected = [], 0
    while len(out) < n:
        kr = float(rng.uniform(*kr_range))
        R = float(rng.uniform(4.0, 16.0))
        ratio = float(rng.uniform(0.8, 1.5))
        kh = float(rng.uniform(0.0, math.pi / 2.0))
        lam = int(lam_step * round(2.0 * math.pi * R / kr / lam_step))
        kr_eff = 2.0 * math.pi * R / lam
        if not kr_range[0] <= kr_eff < kr_range[1]:
            rejected += 1
            continue
        out.append((lam, R, ratio, kh))
    return out, rejected


def channel_problem(draw, x_mid: float, k: float, n_periods: int = 30, avg_periods: int = 10,
                    n_surf: int = 2048, width: int = CHANNEL_WIDTH):
    """The box lambda x width x width of one channel draw (c0 = 1/3, lambda = the length)."""
    lam, R, ratio, kh = draw
    center = (x_mid + kh / k, width / 2.0, width / 2.0)
    p = _problem(3, int(lam), width, width, BATCH_C0, ratio * BATCH_C0, R, center, float(lam),
                 n_periods, avg_periods, n_surf, kh=kh)
    p["cp_ratio"] = ratio
    return p


def random_state(seed: int, ncell: int, Q: int, scale: float = 0.1) -> np.ndarray:
    """Seeded random populations (cells x Q), uniform in [-scale, scale)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=(ncell, Q))


def random_c_field(seed: int, shape, c0: float, spread: float) -> np.ndarray:
    """Seeded per-cell sound speeds uniform in [c0 - spread, c0 + spread)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(c0 - spread, c0 + spread, size=int(np.prod(shape)))
