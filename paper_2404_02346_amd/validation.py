"""Validation cases of the wave model beyond the radiation force (Sec. "Lattice-
Boltzmann for acoustics"): an oscillating point source and a plane interface
between two media.

Point source (eq. waves_with_pointSource and the Green's-function solution
after it).  One node of a periodic cube is imposed, like the source sheet,
with rho1 = rho_a sin(w t) and its own momentum.  Far from it the field is
the outgoing spherical wave of the inhomogeneous wave equation,
rho1 = A sin(w t - k r + phi) / r: the complex amplitude P(r) at the drive
frequency has |P| r constant and phase -k r, with k the lattice wavenumber
along the ray (1 - cos w = c^2 sum_a (1 - cos k_a) for the wave vector k n).
The printed prefactor of the solution is not dimensionally consistent, and a
node-sized source has no continuum strength, so A and phi are fitted, not
predicted.  The record ends before the first image from the periodic copies
arrives and starts one period after the direct wave has passed the
outermost fitted node.

Plane interface.  The paper models the interface as a smooth change of the
sound speed along x (eq. c_plane_int),
    c(x) = ((c_p - c_0)/2) tanh((x - x_i)/w) + (c_p + c_0)/2,
with c_0 = 0.5 and c_p = 0.25, and checks that pressure and normal velocity
are continuous across it, p_I + p_R = p_T and u_I + u_R = u_T, to 1%.

Here the wave comes from the driven source sheet (x = 1) of a long box one
cell wide (D2Q5, ny = 1).  After the incident wave has reached the
interface and before any second reflection (from the source sheet or the far
wall) is back, rho1(x, t) is recorded for one drive period; its complex
amplitude P(x) = (2/T) sum_t c(x)^2 rho1(x, t) exp(-i w t) is fitted by least
squares to a e^{-i k1 (x - x_i)} + b e^{i k1 (x - x_i)} on the incident side
and to t e^{-i k2 (x - x_i)} (+ a small backward part) on the far side, with
the lattice wavenumbers of the exact dispersion cos w = 1 - c^2 (1 - cos k).
R = b / a and T = t / a are the pressure reflection and transmission
coefficients; for density-matched media a sharp interface gives
R = (c_p - c_0)/(c_p + c_0) and T = 2 c_p / (c_p + c_0), so that
|1 + R| = |T| (pressure) and |1 - R| = |T| c_0 / c_p (normal velocity); any
interface conserves the energy flux: |R|^2 + (c_0 / c_p) |T|^2 = 1.  A
smooth interface (width w) reflects less than a sharp one.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbwave


def point_source_problem(n: int = 64, lam: float = 12.0, c0: float = 0.5, rho_a: float = 1.0,
                         dim: int = 3):
    """A periodic cube (square in 2D) of n cells per side with the source node at its centre."""
    s = n // 2
    p = {"dim": dim, "nx": n, "ny": n, "xbc": "periodic", "c0": c0, "rho0": 1.0,
         "center": (0.0, 0.0, 0.0), "radius": 0.0, "cp": c0, "rho_a": rho_a,
         "omega": 2.0 * math.pi * c0 / lam, "wall_phi": 0.99, "avg_start": 0, "lam": lam,
         "src_cell": (s, s, s if dim == 3 else 0)}
    if dim == 3:
        p["nz"] = n
    return p


def ray_cells(p: dict, direction, r_max: float):
    """Nodes s + m d (m = 1, 2, ...) along a lattice direction d within r_max: distances, cell indices."""
    d = np.asarray(list(direction) + [0] * (3 - len(direction)), dtype=np.int64)
    s = np.asarray(p["src_cell"], dtype=np.int64)
    nx, ny = p["nx"], p["ny"]
    step = float(np.linalg.norm(d))
    m = np.arange(1, int(r_max / step) + 1)
    xyz = s[None, :] + m[:, None] * d[None, :]
    return m * step, (xyz[:, 2] * ny + xyz[:, 1]) * nx + xyz[:, 0]


def ray_wavenumber(omega: float, c: float, direction) -> float:
    """|k| of the lattice plane wave of frequency omega whose wave vector points along direction."""
    d = np.asarray(direction, dtype=np.float64)
    u = d / np.linalg.norm(d)
    lo, hi = 0.0, math.pi
    for _ in range(200):  # 1 - cos w = c^2 sum_a (1 - cos(k u_a)) is increasing in k on [0, pi]
        mid = 0.5 * (lo + hi)
        if c * c * float(np.sum(1.0 - np.cos(mid * u))) < 1.0 - math.cos(omega):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def point_source_window(p: dict, r_fit: float):
    """(t0, n): one drive period that starts a period after the direct wave has passed r_fit and
    ends before the first image (distance n - r from the nearest periodic copy) reaches r_fit."""
    c0, n = p["c0"], p["nx"]
    period = int(round(2 * math.pi / p["omega"]))
    t_end = int((n - r_fit) / c0) - 4
    t0 = t_end - period
    assert t0 >= r_fit / c0 + period, "the box is too small for this r_fit"
    return t0, period


def spherical_amplitude(p: dict, rho_tr: np.ndarray, t0: int):
    """Complex amplitude P = (2/T) sum_t rho1(t) exp(-i w t) over one period, per column."""
    n = rho_tr.shape[0]
    t = t0 + np.arange(n)
    return (2.0 / n) * (rho_tr * np.exp(-1j * p["omega"] * t)[:, None]).sum(axis=0)


def rho_probe_gpu(p: dict, cells, t0: int, n: int, storage: str = "f64") -> np.ndarray:
    """rho1 of steps t0 .. t0+n-1 at the given cells, summed by the GPU library
    (lb_wave_probe_rho) after each step."""
    import torch
    cells = torch.as_tensor(np.asarray(cells, dtype=np.int64), device="cuda")
    h = lbwave.LBWave([p], storage=storage)
    out = torch.empty((n, cells.numel()), dtype=torch.float64, device="cuda")
    h.step(t0)
    for j in range(n):
        h.step(1)
        h.probe_rho(cells, out[j])
    res = out.cpu().numpy()
    h.close()
    return res


def point_source(storage: str = "f32", r_fit: float | None = None, directions=((1, 0, 0),),
                 **kw):
    """Run the point source on the GPU library; per direction: r, |P| r and phase + k r."""
    p = point_source_problem(**kw)
    r_fit = p["nx"] / 4 if r_fit is None else r_fit
    t0, n = point_source_window(p, r_fit)
    rays = [ray_cells(p, d, r_fit) for d in directions]
    cells = np.concatenate([c for _, c in rays])
    P = spherical_amplitude(p, rho_probe_gpu(p, cells, t0, n, storage), t0)
    out, j = [], 0
    for d, (r, c) in zip(directions, rays):
        Pd = P[j: j + c.size]
        j += c.size
        k = ray_wavenumber(p["omega"], p["c0"], d)
        out.append({"direction": tuple(d), "r": r, "amp_r": np.abs(Pd) * r,
                    "phase_kr": np.unwrap(np.angle(Pd)) + k * r, "k": k})
    return out


def interface_problem(nx: int = 2048, c0: float = 0.5, cp: float = 0.25, lam: float = 64.0,
                      w: float = 0.5, x_i: float | None = None):
    """The driven one-cell-wide box with a tanh interface at x_i (default nx/2)."""
    x_i = nx / 2.0 if x_i is None else x_i
    x = np.arange(nx, dtype=np.float64)
    c = (cp - c0) / 2.0 * np.tanh((x - x_i) / w) + (cp + c0) / 2.0
    return {"dim": 2, "nx": nx, "ny": 1, "nz": 1, "xbc": "driven", "c0": c0, "rho0": 1.0,
            "center": (x_i, 0.5, 0.0), "radius": 1.0, "cp": c0, "d": 4.0, "rho_a": 1.0,
            "omega": 2.0 * math.pi * c0 / lam, "wall_phi": 0.99, "c_field": c,
            "avg_start": 0, "x_i": x_i, "cp_medium": cp, "lam": lam}


def lattice_k(omega: float, c: float) -> float:
    """Wavenumber of the exact lattice dispersion cos(omega) = 1 - c^2 (1 - cos k)."""
    return math.acos(1.0 - (1.0 - math.cos(omega)) / (c * c))


def window(p: dict):
    """(t0, n): one drive period after the incident wave has passed the interface and before any
    second reflection reaches the fitted regions (see fit_regions)."""
    period = int(round(2 * math.pi / p["omega"]))
    c0, cp, x_i, nx = p["c0"], p["cp_medium"], p["x_i"], p["nx"]
    t_hit = (x_i - 1) / c0                          # incident front at the interface
    t_src = t_hit + (x_i - 1) / c0                  # reflected front back at the source
    t0 = int(t_hit + 0.7 * (x_i - 1) / c0)          # reflected front 70% of the way back
    assert t0 + period < t_src, "the box is too short for the window"
    assert t0 + period < t_hit + (nx - 1 - x_i) / cp, "the transmitted front reached the wall"
    return t0, period


def fit_regions(p: dict, t_end: int):
    """Incident side: from just before the reflected front to 20 cells before the interface;
    far side: 20 cells after the interface to just before the transmitted front."""
    c0, cp, x_i = p["c0"], p["cp_medium"], p["x_i"]
    t_hit = (x_i - 1) / c0
    back = x_i - (t_end - p["lam"] / c0 - t_hit) * c0   # reflected front one period earlier
    ahead = x_i + (t_end - p["lam"] / c0 - t_hit) * cp - 2 * p["lam"] * cp / c0
    return (int(math.ceil(back)) + 8, int(x_i) - 20), (int(x_i) + 20, int(ahead) - 8)


def coefficients(p: dict, rho_xt: np.ndarray, t0: int):
    """R, T and the residual backward part on the far side from rho1(t0 + j, x), j < period."""
    n = rho_xt.shape[0]
    om = p["omega"]
    t = t0 + np.arange(n)
    pxt = rho_xt * (p["c_field"] ** 2)[None, :]
    P = (2.0 / n) * (pxt * np.exp(-1j * om * t)[:, None]).sum(axis=0)
    k1, k2 = lattice_k(om, p["c0"]), lattice_k(om, p["cp_medium"])
    (a1, b1), (a2, b2) = fit_regions(p, t0 + n)
    x_i = p["x_i"]
    x = np.arange(a1, b1) - x_i
    A = np.stack([np.exp(-1j * k1 * x), np.exp(1j * k1 * x)], axis=1)
    (a, b), *_ = np.linalg.lstsq(A, P[a1:b1], rcond=None)
    x = np.arange(a2, b2) - x_i
    A = np.stack([np.exp(-1j * k2 * x), np.exp(1j * k2 * x)], axis=1)
    (tt, back), *_ = np.linalg.lstsq(A, P[a2:b2], rcond=None)
    R, T = b / a, tt / a
    c0, cp = p["c0"], p["cp_medium"]
    return {"R": complex(R), "T": complex(T), "backward": float(abs(back / a)),
            "R_sharp": (cp - c0) / (cp + c0), "T_sharp": 2 * cp / (cp + c0),
            "energy": float(abs(R) ** 2 + (c0 / cp) * abs(T) ** 2),
            # |p_I + p_R| = |p_T| and |u_I + u_R| = |u_T| (u = p / (rho0 c) of each wave), as
            # relative errors; magnitudes need no reference position inside the smooth interface
            "pressure_continuity": float(abs(abs(1 + R) - abs(T)) / abs(T)),
            "velocity_continuity": float(abs(abs(1 - R) - abs(T) * c0 / cp) / (abs(T) * c0 / cp)),
            "regions": ((a1, b1), (a2, b2))}


def rho_window_gpu(p: dict, t0: int, n: int, storage: str = "f64"):
    """rho1(t, x), t = t0 .. t0+n-1, of the one-row box: the sum of the populations of step t
    at every cell, summed by the GPU library (lb_wave_probe_rho)."""
    return rho_probe_gpu(p, np.arange(p["nx"] * p["ny"] * p.get("nz", 1)), t0, n, storage)


def plane_interface(storage: str = "f64", **kw):
    """Run the plane-interface case on the GPU library and return its coefficients."""
    p = interface_problem(**kw)
    t0, n = window(p)
    return coefficients(p, rho_window_gpu(p, t0, n, storage), t0)
