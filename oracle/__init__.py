"""FP64 CPU oracle of the wave lattice Boltzmann acoustic-radiation-force method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the GPU library ``paper_2404_02346_amd``; the two meet only through the
seeded input generators in ``workloads``.

The heavy lifting is plain C (``lb_oracle.c``, FP64, array-of-structures);
this module marshals arguments with ctypes and adds the cavity calibration
fit.  Every function cites the passage of the paper it follows (Castro-Avila
et al., arXiv 2404.02346).

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against algebraic facts, closed forms or brute force, except the absolute
value of the time-averaged force of a discrete set-up, which has no closed
form ("parity unpinned" beyond the physics bands and invariants listed in
the design notes).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import closed_forms  # noqa: F401  (re-exported)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborc.so")

XBC = {"driven": 0, "periodic": 1}

_dp = C.POINTER(C.c_double)
_i64p = C.POINTER(C.c_int64)


class _Desc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("xbc", C.c_int32),
        ("c0", C.c_double), ("rho0", C.c_double),
        ("c_field", _dp),
        ("center", C.c_double * 3),
        ("radius", C.c_double), ("cp", C.c_double), ("d", C.c_double),
        ("rho_a", C.c_double), ("omega", C.c_double), ("wall_phi", C.c_double),
        ("n_surf", C.c_int32),
        ("surf_xyz", _dp), ("surf_normal", _dp), ("surf_area", _dp),
        ("avg_start", C.c_int64),
        ("src_kind", C.c_int32), ("src_cell", C.c_int32 * 3),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        lib = C.CDLL(LIB_PATH)
        lib.orc_lattice.argtypes = [C.c_int, _dp, _dp, C.POINTER(C.c_int)]
        lib.orc_feq.argtypes = [C.c_int, C.c_double, C.c_double, _dp, _dp]
        lib.orc_collide_cell.argtypes = [C.c_int, C.c_double, _dp, _dp]
        lib.orc_roma.argtypes = [C.c_double]
        lib.orc_roma.restype = C.c_double
        lib.orc_sound_speed.argtypes = [C.POINTER(_Desc), C.c_double, C.c_double, C.c_double]
        lib.orc_sound_speed.restype = C.c_double
        lib.orc_stream.argtypes = [C.POINTER(_Desc), _dp, _dp]
        lib.orc_interp.argtypes = [C.POINTER(_Desc), _dp, _dp, _dp, _dp, _dp]
        lib.orc_interp.restype = C.c_int
        lib.orc_surface_integral.argtypes = [C.POINTER(_Desc), _dp, _dp, _dp]
        lib.orc_run.argtypes = [C.POINTER(_Desc), C.c_int64, _dp, _dp, _dp, _dp, _i64p, _dp,
                                C.c_int64, C.c_int64, _i64p, C.c_int64, _dp]
        lib.orc_run.restype = C.c_int
        lib.orc_run_segment.argtypes = [C.POINTER(_Desc), C.c_int64, C.c_int64, _dp, _dp, _dp,
                                        _i64p]
        lib.orc_run_segment.restype = C.c_int
        _lib = lib
    return _lib


def _ptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(_dp)


def _f64(a, shape=None):
    if a is None:
        return None
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    if shape is not None:
        a = a.reshape(shape)
    return a


class _Bound:
    """Keeps the numpy arrays a ctypes descriptor points into alive."""

    def __init__(self, p: dict):
        dim = int(p["dim"])
        self.c_field = _f64(p.get("c_field"))
        surf = p.get("surf_xyz")
        self.n_surf = 0 if surf is None else int(np.asarray(surf).size // 3)
        self.surf_xyz = _f64(surf, (-1,)) if self.n_surf else None
        self.surf_normal = _f64(p.get("surf_normal"), (-1,)) if self.n_surf else None
        self.surf_area = _f64(p.get("surf_area"), (-1,)) if self.n_surf else None
        d = _Desc()
        d.dim = dim
        d.nx, d.ny = int(p["nx"]), int(p["ny"])
        d.nz = int(p.get("nz", 1)) if dim == 3 else 1
        d.xbc = XBC[p.get("xbc", "driven")]
        d.c0 = float(p["c0"])
        d.rho0 = float(p.get("rho0", 1.0))
        d.c_field = _ptr(self.c_field)
        cen = list(p.get("center", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
        for a in range(3):
            d.center[a] = float(cen[a])
        d.radius = float(p.get("radius", 0.0))
        d.cp = float(p.get("cp", p["c0"]))
        d.d = float(p.get("d", 4.0))
        d.rho_a = float(p.get("rho_a", 1.0))
        d.omega = float(p.get("omega", 0.0))
        d.wall_phi = float(p.get("wall_phi", 0.99))
        d.n_surf = self.n_surf
        d.surf_xyz = _ptr(self.surf_xyz)
        d.surf_normal = _ptr(self.surf_normal)
        d.surf_area = _ptr(self.surf_area)
        d.avg_start = int(p.get("avg_start", 0))
        sc = p.get("src_cell")  # a point source at this node (periodic x)
        d.src_kind = 0 if sc is None else 1
        for a in range(3):
            d.src_cell[a] = 0 if sc is None else int((list(sc) + [0, 0, 0])[a])
        self.desc = d
        self.Q = 2 * dim + 1
        self.ncell = d.nx * d.ny * d.nz
        self.shape = (d.nz, d.ny, d.nx) if dim == 3 else (d.ny, d.nx)


# ---------------------------------------------------------------------------
# Lattice algebra (Sec. "Lattice-Boltzmann for acoustics")
# ---------------------------------------------------------------------------

def lattice(dim: int):
    """Weights, c_s^2 and velocity vectors of D2Q5 / D3Q7 (eq. velocity_properties)."""
    lib = _load()
    Q = 2 * dim + 1
    w = np.zeros(7)
    cs2 = C.c_double()
    vel = (C.c_int * 21)()
    lib.orc_lattice(dim, _ptr(w), C.byref(cs2), vel)
    v = np.array(vel[:], dtype=np.int64).reshape(7, 3)[:Q]
    return w[:Q].copy(), cs2.value, v


def feq(dim: int, c2: float, rho: float, J) -> np.ndarray:
    """Equilibrium populations of eq. feq_waves at one cell."""
    lib = _load()
    Jv = _f64(list(J) + [0.0] * (3 - len(J)))
    out = np.zeros(7)
    lib.orc_feq(dim, float(c2), float(rho), _ptr(Jv), _ptr(out))
    return out[: 2 * dim + 1].copy()


def collide_cell(dim: int, c2: float, f) -> np.ndarray:
    """BGK collision with tau = 1/2 at one cell (eq. LBM-Collision)."""
    lib = _load()
    fin = _f64(f)
    out = np.zeros(2 * dim + 1)
    lib.orc_collide_cell(dim, float(c2), _ptr(fin), _ptr(out))
    return out


def roma(r) -> np.ndarray:
    """The 3-point interpolation kernel printed after eq. InterpolatedFields."""
    lib = _load()
    r = np.asarray(r, dtype=np.float64)
    return np.vectorize(lambda v: lib.orc_roma(float(v)), otypes=[np.float64])(r)


def sound_speed(p: dict, x, y, z=0.0) -> np.ndarray:
    """c(r) of the object, eq. sound_speed_object (c_p inside, c0 outside)."""
    lib = _load()
    b = _Bound(p)
    f = lambda a, bb, cc: lib.orc_sound_speed(C.byref(b.desc), float(a), float(bb), float(cc))
    return np.vectorize(f, otypes=[np.float64])(x, y, z)


def stream(p: dict, fin: np.ndarray) -> np.ndarray:
    """Advection of eq. LBM-Advection on a whole AoS state (cells x Q)."""
    lib = _load()
    b = _Bound(p)
    fin = _f64(fin)
    assert fin.size == b.ncell * b.Q
    out = np.empty_like(fin)
    lib.orc_stream(C.byref(b.desc), _ptr(fin), _ptr(out))
    return out


def interp(p: dict, rho: np.ndarray, J: np.ndarray, P) -> tuple[float, np.ndarray]:
    """Kernel interpolation of eq. InterpolatedFields at one point P."""
    lib = _load()
    b = _Bound(p)
    rho = _f64(rho, (-1,))
    J = _f64(J, (-1,))
    assert rho.size == b.ncell and J.size == 3 * b.ncell
    Pv = _f64(list(P) + [0.0] * (3 - len(P)))
    rI = C.c_double()
    JI = np.zeros(3)
    st = lib.orc_interp(C.byref(b.desc), _ptr(rho), _ptr(J), _ptr(Pv), C.byref(rI), _ptr(JI))
    if st != 0:
        raise ValueError(f"interpolation stencil leaves the lattice (status {st})")
    return rI.value, JI


def surface_integral(p: dict, rhoI, JI) -> np.ndarray:
    """Instantaneous surface integral of eq. arf_integral_LBM from interpolated fields."""
    lib = _load()
    b = _Bound(p)
    rhoI = _f64(rhoI, (-1,))
    JI = _f64(JI, (-1,))
    assert rhoI.size == b.n_surf and JI.size == 3 * b.n_surf
    F = np.zeros(3)
    lib.orc_surface_integral(C.byref(b.desc), _ptr(rhoI), _ptr(JI), _ptr(F))
    return F


# ---------------------------------------------------------------------------
# The full run
# ---------------------------------------------------------------------------

def run(p: dict, n_steps: int, fnew_init=None, want_fields: bool = False,
        want_trace: bool = False, line: tuple[int, int] | None = None,
        probes=None) -> dict:
    """Run the method for ``n_steps`` steps (see ``orc_run`` in lb_oracle.c).

    Returns a dict with ``F_avg`` (3,), ``n_acc``, and on request ``fnew``
    (the post-collision state of the last step, shape cells x Q, cell index
    (z*ny + y)*nx + x), ``F_trace`` (n_steps, 3) and ``rho_line``
    (line_n, nx) for steps line_t0 .. line_t0+line_n-1; with ``probes`` (cell
    indices) also ``rho_probe`` (line_n, len(probes)) for the same steps.
    """
    lib = _load()
    b = _Bound(p)
    init = None
    if fnew_init is not None:
        init = _f64(fnew_init, (-1,))
        assert init.size == b.ncell * b.Q
    fout = np.empty(b.ncell * b.Q) if want_fields else None
    trace = np.empty(int(n_steps) * 3) if want_trace else None
    Favg = np.zeros(3)
    nacc = C.c_int64()
    rl = None
    lt0, ln = 0, 0
    if line is not None:
        lt0, ln = int(line[0]), int(line[1])
        rl = np.zeros(ln * b.desc.nx)
    pr = rp = None
    if probes is not None:
        assert line is not None, "probes are recorded over the line window"
        pr = np.ascontiguousarray(np.asarray(probes, dtype=np.int64).reshape(-1))
        rp = np.zeros(ln * pr.size)
    st = lib.orc_run(C.byref(b.desc), int(n_steps), _ptr(init), _ptr(fout), _ptr(trace),
                     _ptr(Favg), C.byref(nacc), _ptr(rl), lt0, ln,
                     None if pr is None else pr.ctypes.data_as(_i64p), 0 if pr is None else pr.size,
                     _ptr(rp))
    if st != 0:
        raise ValueError(f"oracle run failed with status {st}")
    out = {"F_avg": Favg, "n_acc": nacc.value}
    if want_fields:
        out["fnew"] = fout.reshape(b.ncell, b.Q)
    if want_trace:
        out["F_trace"] = trace.reshape(int(n_steps), 3)
    if line is not None:
        out["rho_line"] = rl.reshape(ln, b.desc.nx)
    if pr is not None:
        out["rho_probe"] = rp.reshape(ln, pr.size)
    return out


def run_segments(p: dict, n_steps: int, n_segments: int, progress=None) -> dict:
    """``run(p, n_steps)`` in n_segments consecutive pieces (orc_run_segment), carrying the
    state and the FP64 force sums across them: the same time average, bit for bit, with a
    progress callback progress(steps_done) after each piece.  Returns F_avg and n_acc."""
    lib = _load()
    b = _Bound(p)
    cur = np.zeros(b.ncell * b.Q)
    nxt = np.empty_like(cur)
    acc = np.zeros(3)
    nacc = C.c_int64(0)
    bounds = np.linspace(0, int(n_steps), int(n_segments) + 1).round().astype(np.int64)
    for t0, t1 in zip(bounds[:-1], bounds[1:]):
        st = lib.orc_run_segment(C.byref(b.desc), int(t0), int(t1 - t0), _ptr(cur), _ptr(nxt),
                                 _ptr(acc), C.byref(nacc))
        if st != 0:
            raise ValueError(f"oracle segment failed with status {st}")
        cur, nxt = nxt, cur
        if progress is not None:
            progress(int(t1))
    n = nacc.value
    return {"F_avg": acc / n if n > 0 else np.zeros(3), "n_acc": n}


# ---------------------------------------------------------------------------
# Empty-cavity calibration of the driven standing wave
# ---------------------------------------------------------------------------

def lattice_wavenumber(omega: float, c: float) -> float:
    """Wavenumber of a plane wave of frequency omega on the homogeneous lattice.

    From the exact dispersion cos(omega) = 1 - c^2 (1 - cos k) of the
    tau = 1/2 scheme along a lattice axis (pinned in the tests by a free
    standing-wave run).
    """
    return float(np.arccos(1.0 - (1.0 - np.cos(omega)) / (c * c)))


def cavity_calibration(nx: int, c0: float, omega: float, rho_a: float = 1.0,
                       wall_phi: float = 0.99, n_periods: int = 30, n_fit: int = 5) -> dict:
    """Standing-wave amplitude and antinodes of the empty driven box.

    Follows the set-up of Sec. "Results and discussion" (absorbing wall at
    x = 0, source sheet at x = 1, damped reflector at x = Lx-1) without an
    object.  The wave depends on x only, so a box one cell wide in y gives
    the same field as any cross-section.  After ``n_periods`` drive periods
    the complex amplitude P(x) of rho1 at the drive frequency is taken over
    the last ``n_fit`` periods, |P(x)|^2 is fitted by a + b cos 2kx +
    c sin 2kx with k the lattice wavenumber, and

      A   = sqrt(a + sqrt(b^2 + c^2))  (density amplitude at an antinode),
      x_a = antinodes x where 2k x = atan2(c, b) mod 2 pi,
      Pa  = c0^2 A (pressure amplitude, eq. eq_state).
    """
    period = 2.0 * np.pi / omega
    n_total = int(round(n_periods * period))
    m = int(round(n_fit * period))
    p = {"dim": 2, "nx": nx, "ny": 1, "c0": c0, "cp": c0, "radius": 0.0,
         "center": (0.0, 0.0, 0.0), "rho_a": rho_a, "omega": omega, "wall_phi": wall_phi}
    r = run(p, n_total, line=(n_total - m, m))
    t = np.arange(n_total - m, n_total, dtype=np.float64)
    rl = r["rho_line"]
    P = (2.0 / m) * (rl * np.exp(-1j * omega * t)[:, None]).sum(axis=0)
    k = lattice_wavenumber(omega, c0)
    xs = np.arange(2, nx - 2, dtype=np.float64)
    M = np.stack([np.ones_like(xs), np.cos(2 * k * xs), np.sin(2 * k * xs)], axis=1)
    coef, *_ = np.linalg.lstsq(M, np.abs(P[2:nx - 2]) ** 2, rcond=None)
    a, bb, cc = coef
    A = float(np.sqrt(a + np.hypot(bb, cc)))
    x0 = float(np.arctan2(cc, bb) / (2 * k))
    spacing = np.pi / k
    first = x0 - np.floor((x0 + spacing) / spacing) * spacing  # smallest antinode >= -spacing
    antinodes = [first + j * spacing for j in range(int((nx + 2 * spacing) / spacing) + 1)]
    antinodes = [v for v in antinodes if -spacing < v < nx]
    centre = (nx - 1) / 2.0
    below = [v for v in antinodes if v <= centre]
    mid = max(below) if below else min(antinodes)
    return {"A": A, "Pa": c0 * c0 * A, "k": k, "antinodes": antinodes, "x_mid": mid,
            "P": P, "fit": (a, bb, cc)}
