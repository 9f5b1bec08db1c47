"""ctypes binding of the C ABI in include/lb_wave.h (argument marshalling only).

PyTorch provides the device workspace (a uint8 tensor) and the stream; every
step of the computation runs in the HIP kernels of ``liblbwave.so``.  There is
no fallback: if the library is missing, loading raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbwave.so")

STORAGE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
XBC = {"driven": 0, "periodic": 1}
STATUS = {0: "LB_OK", -1: "LB_EINVAL", -2: "LB_ENOMEM", -3: "LB_EUNSTABLE", -4: "LB_EGEOMETRY",
          -5: "LB_EDEVICE", -6: "LB_ENAN", -7: "LB_EEMPTY"}

_dp = C.POINTER(C.c_double)


class LBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Desc(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("storage", C.c_int32), ("xbc", C.c_int32),
        ("c0", C.c_double), ("rho0", C.c_double),
        ("c_field", _dp),
        ("obj_center", C.c_double * 3),
        ("obj_radius", C.c_double), ("obj_cp", C.c_double), ("obj_d", C.c_double),
        ("rho_a", C.c_double), ("omega", C.c_double), ("wall_phi", C.c_double),
        ("n_surf", C.c_int32),
        ("surf_xyz", _dp), ("surf_normal", _dp), ("surf_area", _dp),
        ("avg_start", C.c_int64), ("max_steps", C.c_int64), ("trace_steps", C.c_int64),
        ("src_kind", C.c_int32), ("src_cell", C.c_int32 * 3),
    ]


class StateView(C.Structure):
    _fields_ = [("offset_bytes", C.c_size_t), ("plane_bytes", C.c_size_t),
                ("pitch", C.c_int32), ("elem_bytes", C.c_int32), ("scale", C.c_double)]


_lib = None


def lib():
    """Load liblbwave.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.lb_last_error.restype = C.c_char_p
        L.lb_wave_check.argtypes = [C.POINTER(Desc), C.c_int32]
        L.lb_wave_workspace_bytes.argtypes = [C.POINTER(Desc), C.c_int32]
        L.lb_wave_workspace_bytes.restype = C.c_size_t
        L.lb_wave_create.argtypes = [C.POINTER(Desc), C.c_int32, vp, C.c_size_t, vp,
                                     C.POINTER(vp)]
        L.lb_wave_step_n.argtypes = [vp, C.c_int64]
        L.lb_surface_force.argtypes = [vp, _dp, C.POINTER(C.c_int64)]
        L.lb_wave_destroy.argtypes = [vp]
        L.lb_wave_steps_done.argtypes = [vp, C.POINTER(C.c_int64)]
        L.lb_wave_reset.argtypes = [vp]
        L.lb_wave_get_state.argtypes = [vp, C.c_int32, _dp]
        L.lb_wave_set_state.argtypes = [vp, C.c_int32, _dp]
        L.lb_wave_force_trace.argtypes = [vp, C.c_int32, _dp, C.c_int64]
        L.lb_wave_state_view.argtypes = [vp, C.c_int32, C.POINTER(StateView)]
        L.lb_wave_probe_rho.argtypes = [vp, C.c_int32, vp, C.c_int32, vp]
        L.lb_wave_set_variant.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
        L.lb_wave_get_variant.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                          C.POINTER(C.c_int32)]
        L.lb_wave_set_tile.argtypes = [vp, C.c_int32]
        L.lb_wave_set_graph.argtypes = [vp, C.c_int32]
        L.lb_wave_set_steps_per_launch.argtypes = [vp, C.c_int32]
        L.lb_wave_get_steps_per_launch.argtypes = [vp, C.POINTER(C.c_int32)]
        L.lb_wave_get_tile.argtypes = [vp, C.POINTER(C.c_int32)]
        L.lb_wave_autotune.argtypes = [vp, C.c_int32, _dp]
        L.lb_stream_copy.argtypes = [vp, vp, C.c_size_t, vp]
        L.lb_cavity_workspace_bytes.argtypes = [C.c_int32]
        L.lb_cavity_workspace_bytes.restype = C.c_size_t
        L.lb_cavity_calibrate.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double,
                                          C.c_double, C.c_int32, C.c_int32, vp, C.c_size_t, vp,
                                          _dp, _dp]
        _lib = L
    return _lib


def _check(code: int):
    if code != 0:
        raise LBError(code, lib().lb_last_error().decode())


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_dp)


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def make_descs(problems, storage: str = "f32", freeze_at_n_steps: bool = False,
               trace_steps: int = 0):
    """Build the C descriptors for a list of problem dicts.

    Returns (array of Desc, list of numpy arrays the descriptors point into).
    """
    keep = []
    arr = (Desc * len(problems))()
    for d, p in zip(arr, problems):
        dim = int(p["dim"])
        d.dim, d.nx, d.ny = dim, int(p["nx"]), int(p["ny"])
        d.nz = int(p.get("nz", 1)) if dim == 3 else 1
        d.storage = STORAGE[storage]
        d.xbc = XBC[p.get("xbc", "driven")]
        d.c0, d.rho0 = float(p["c0"]), float(p.get("rho0", 1.0))
        cf = p.get("c_field")
        if cf is not None:
            cf = np.ascontiguousarray(np.asarray(cf, dtype=np.float64).reshape(-1))
            keep.append(cf)
        d.c_field = _ptr(cf)
        cen = list(p.get("center", (0.0, 0.0, 0.0))) + [0.0, 0.0, 0.0]
        for a in range(3):
            d.obj_center[a] = float(cen[a])
        d.obj_radius = float(p.get("radius", 0.0))
        d.obj_cp = float(p.get("cp", p["c0"]))
        d.obj_d = float(p.get("d", 4.0))
        d.rho_a = float(p.get("rho_a", 1.0))
        d.omega = float(p.get("omega", 0.0))
        d.wall_phi = float(p.get("wall_phi", 0.99))
        xyz = p.get("surf_xyz")
        n = 0 if xyz is None else int(np.asarray(xyz).size // 3)
        d.n_surf = n
        if n:
            xyz = np.ascontiguousarray(np.asarray(xyz, dtype=np.float64).reshape(-1))
            nrm = np.ascontiguousarray(np.asarray(p["surf_normal"], dtype=np.float64).reshape(-1))
            area = np.ascontiguousarray(np.asarray(p["surf_area"], dtype=np.float64).reshape(-1))
            keep += [xyz, nrm, area]
            d.surf_xyz, d.surf_normal, d.surf_area = _ptr(xyz), _ptr(nrm), _ptr(area)
        d.avg_start = int(p.get("avg_start", 0))
        ms = p.get("max_steps")
        if ms is None and freeze_at_n_steps:
            ms = p.get("n_steps", 0)
        d.max_steps = int(ms or 0)
        d.trace_steps = int(p.get("trace_steps", trace_steps))
        sc = p.get("src_cell")  # a point source at this node (periodic x)
        d.src_kind = 0 if sc is None else 1
        for a in range(3):
            d.src_cell[a] = 0 if sc is None else int((list(sc) + [0, 0, 0])[a])
    return arr, keep


def check(problems, storage: str = "f32") -> int:
    """Host-only validation (lb_wave_check); returns the status code."""
    arr, _ = make_descs(problems, storage)
    return lib().lb_wave_check(arr, len(problems))


def workspace_bytes(problems, storage: str = "f32", trace_steps: int = 0) -> int:
    arr, _ = make_descs(problems, storage, trace_steps=trace_steps)
    return lib().lb_wave_workspace_bytes(arr, len(problems))


class LBWave:
    """One handle over one or more problem instances (lb_wave_create)."""

    def __init__(self, problems, storage: str = "f32", stream=None, trace_steps: int = 0,
                 freeze_at_n_steps: bool = False, device: str = "cuda"):
        import torch
        self.problems = list(problems)
        self.storage = storage
        self.n = len(self.problems)
        L = lib()
        descs, keep = make_descs(self.problems, storage, freeze_at_n_steps, trace_steps)
        nbytes = L.lb_wave_workspace_bytes(descs, self.n)
        if nbytes == 0:
            _check(L.lb_wave_check(descs, self.n) or -1)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self.ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.nbytes = nbytes
        self._h = C.c_void_p()
        _check(L.lb_wave_create(descs, self.n, C.c_void_p(self.ws.data_ptr()), nbytes,
                                _stream_handle(self.stream), C.byref(self._h)))
        self._trace = [int(p.get("trace_steps", trace_steps)) for p in self.problems]
        self.Q = [2 * int(p["dim"]) + 1 for p in self.problems]
        self.ncell = [int(p["nx"]) * int(p["ny"]) * (int(p.get("nz", 1)) if int(p["dim"]) == 3
                                                     else 1) for p in self.problems]

    # -- core ABI --
    def step(self, n: int):
        _check(lib().lb_wave_step_n(self._h, int(n)))

    def force(self, allow_empty: bool = False):
        F = np.zeros(3 * self.n)
        nacc = np.zeros(self.n, dtype=np.int64)
        code = lib().lb_surface_force(self._h, _ptr(F), nacc.ctypes.data_as(C.POINTER(C.c_int64)))
        if code != 0 and not (allow_empty and code == -7):
            _check(code)
        return F.reshape(self.n, 3), nacc

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            lib().lb_wave_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- inspection and control --
    @property
    def t(self) -> int:
        v = C.c_int64()
        _check(lib().lb_wave_steps_done(self._h, C.byref(v)))
        return v.value

    def reset(self):
        _check(lib().lb_wave_reset(self._h))

    def get_state(self, inst: int = 0) -> np.ndarray:
        out = np.empty(self.ncell[inst] * self.Q[inst])
        _check(lib().lb_wave_get_state(self._h, int(inst), _ptr(out)))
        return out.reshape(self.ncell[inst], self.Q[inst])

    def set_state(self, inst: int, fnew) -> None:
        a = np.ascontiguousarray(np.asarray(fnew, dtype=np.float64).reshape(-1))
        assert a.size == self.ncell[inst] * self.Q[inst]
        _check(lib().lb_wave_set_state(self._h, int(inst), _ptr(a)))

    def trace(self, inst: int = 0, n: int | None = None) -> np.ndarray:
        n = self._trace[inst] if n is None else int(n)
        out = np.zeros(3 * n)
        _check(lib().lb_wave_force_trace(self._h, int(inst), _ptr(out), n))
        return out.reshape(n, 3)

    def probe_rho(self, cells_dev, out_dev, inst: int = 0):
        """rho1 at the cells (int64 device tensor) into out_dev (float64 device tensor),
        stream-ordered after the steps enqueued so far (lb_wave_probe_rho)."""
        assert cells_dev.dtype.itemsize == 8 and out_dev.numel() >= cells_dev.numel()
        _check(lib().lb_wave_probe_rho(self._h, int(inst), C.c_void_p(cells_dev.data_ptr()),
                                       int(cells_dev.numel()), C.c_void_p(out_dev.data_ptr())))

    def state_view(self, inst: int = 0) -> StateView:
        v = StateView()
        _check(lib().lb_wave_state_view(self._h, int(inst), C.byref(v)))
        return v

    def set_tile(self, cells_per_lane: int):
        _check(lib().lb_wave_set_tile(self._h, int(cells_per_lane)))

    def set_variant(self, cells_per_lane: int, x_mode: int = 0, nontemporal: int = 0):
        _check(lib().lb_wave_set_variant(self._h, int(cells_per_lane), int(x_mode),
                                         int(nontemporal)))

    def variant(self):
        a, b, c = C.c_int32(), C.c_int32(), C.c_int32()
        _check(lib().lb_wave_get_variant(self._h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def set_graph(self, chunk: int):
        _check(lib().lb_wave_set_graph(self._h, int(chunk)))

    def set_steps_per_launch(self, k: int):
        """1: one lattice step per launch; 2: the fused two-step kernel (3D, driven sheets)."""
        _check(lib().lb_wave_set_steps_per_launch(self._h, int(k)))

    def steps_per_launch(self) -> int:
        v = C.c_int32()
        _check(lib().lb_wave_get_steps_per_launch(self._h, C.byref(v)))
        return v.value

    def tile(self) -> int:
        v = C.c_int32()
        _check(lib().lb_wave_get_tile(self._h, C.byref(v)))
        return v.value

    def autotune(self, n_trial: int = 8) -> float:
        ms = C.c_double()
        _check(lib().lb_wave_autotune(self._h, int(n_trial), C.byref(ms)))
        return ms.value


def stream_copy(src, dst, nbytes: int, stream=None):
    """Plain device copy (lb_stream_copy): the bandwidth reference of the roofline."""
    _check(lib().lb_stream_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()),
                                int(nbytes), _stream_handle(stream)))


def cavity_calibrate(nx: int, c0: float, omega: float, rho_a: float = 1.0,
                     wall_phi: float = 0.99, n_periods: int = 30, n_fit: int = 5, stream=None):
    """Empty-cavity standing-wave calibration on the GPU (lb_cavity_calibrate)."""
    import torch
    L = lib()
    nb = L.lb_cavity_workspace_bytes(int(nx))
    if nb == 0:
        raise LBError(-1, f"nx = {nx} outside the supported range")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out = np.zeros(6)
    P = np.zeros(2 * nx)
    _check(L.lb_cavity_calibrate(int(nx), float(c0), float(omega), float(rho_a),
                                 float(wall_phi), int(n_periods), int(n_fit),
                                 C.c_void_p(ws.data_ptr()), nb, _stream_handle(stream),
                                 _ptr(out), _ptr(P)))
    return {"A": out[0], "x_mid": out[1], "k": out[2], "Pa": c0 * c0 * out[0],
            "fit": tuple(out[3:6]), "P": P[0::2] + 1j * P[1::2]}
