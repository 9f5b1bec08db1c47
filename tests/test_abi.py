"""Host-side tests of the C ABI (no GPU): exports, descriptor checks, sizes."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in ("lb_wave.h", "lb_mlp.h")]


@pytest.fixture(scope="module")
def P():
    import paper_2404_02346_amd as P
    if not os.path.exists(P.lbwave.LIB_PATH):
        from paper_2404_02346_amd import build
        build.build()
    P.lib()
    return P


def declared_functions():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(lb_\w+)\s*\(", src))
    return sorted(names - {"lb_wave_desc"})


def test_header_declares_the_core_calls():
    names = declared_functions()
    for core in ("lb_wave_create", "lb_wave_step_n", "lb_surface_force", "lb_wave_destroy",
                 "lb_wave_workspace_bytes", "lb_wave_check", "lb_cavity_calibrate",
                 "lb_mlp_create", "lb_mlp_forward", "lb_mlp_train_step", "lb_mlp_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol(P):
    names = declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", P.lbwave.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [n for n in names if n not in exported]
    assert not missing, f"not exported with C linkage: {missing}"
    lib = P.lib()
    for n in names:
        assert hasattr(lib, n)


def test_binding_refuses_to_run_without_library(monkeypatch, P):
    import paper_2404_02346_amd.lbwave as lw
    monkeypatch.setattr(lw, "_lib", None)
    monkeypatch.setattr(lw, "LIB_PATH", "/nonexistent/liblbwave.so")
    with pytest.raises(RuntimeError):
        lw.lib()


def _cyl(**kw):
    p = workloads.cylinder_2d(62.63, 2 * np.pi / 128)
    p.update(kw)
    return p


def _sph(**kw):
    p = workloads.sphere_3d(30.6, 2 * np.pi / 64, 0.7, shape=(64, 32, 32), lam=64.0, R=3.0,
                            n_surf=256)
    p.update(kw)
    return p


def test_check_accepts_the_workloads(P):
    assert P.check([_cyl()], "f64") == 0
    assert P.check([_sph()], "f32") == 0
    for s in ("f16", "bf16"):
        assert P.check([_sph()], s) == 0


def test_check_rejects_unstable_sound_speed(P):
    # tau = 1/2 is stable only for c <= 1/sqrt(dim)
    assert P.check([_cyl(cp=0.71)], "f64") == -3
    assert P.check([_cyl(cp=0.70)], "f64") == 0
    assert P.check([_sph(cp=0.58)]) == -3
    assert P.check([_sph(cp=0.577)]) == 0
    assert P.check([_sph(c0=0.6, cp=0.5)]) == -3
    cf = np.full(64 * 32 * 32, 0.5)
    cf[1234] = 0.6
    assert P.check([_sph(c_field=cf)]) == -3
    cf[1234] = 0.55
    assert P.check([_sph(c_field=cf)]) == 0


def test_check_rejects_stencils_on_the_sheets(P):
    # nodes round(P)-1 .. round(P)+1 must avoid x = 0, 1 and nx-1 (driven sheets)
    p = _cyl()
    xyz = np.array(p["surf_xyz"])

    def at_min(v):
        s = xyz.copy()
        s[:, 0] += v - xyz[:, 0].min()
        return _cyl(surf_xyz=s)

    def at_max(v):
        s = xyz.copy()
        s[:, 0] += v - xyz[:, 0].max()
        return _cyl(surf_xyz=s)

    assert P.check([at_min(2.4)]) == -4         # base 2 -> node 1 (source sheet)
    assert P.check([at_min(2.5 + 1e-9)]) == 0   # base 3 -> nodes 2..4
    assert P.check([at_max(125.5 - 1e-9)]) == 0  # base 125 -> nodes 124..126
    assert P.check([at_max(125.5 + 1e-9)]) == -4  # base 126 -> node 127 (reflector)


@pytest.mark.parametrize("field,value", [
    ("dim", 4), ("nz", 3), ("wall_phi", 1.0), ("wall_phi", -0.1), ("rho0", 0.0), ("c0", -0.5),
    ("nx", 2), ("avg_start", -1), ("trace_steps", -5), ("omega", float("nan")), ("obj_d", 0.0),
    ("storage", 7), ("xbc", 3), ("n_surf", -1), ("ny", 0),
])
def test_check_rejects_bad_parameters(P, field, value):
    arr, keep = P.make_descs([_cyl()], "f64")
    assert P.lib().lb_wave_check(arr, 1) == 0
    setattr(arr[0], field, value)
    assert P.lib().lb_wave_check(arr, 1) == -1
    assert P.lib().lb_wave_workspace_bytes(arr, 1) == 0


def test_check_point_source_rules(P):
    # a point source needs periodic x and a node inside the lattice
    from paper_2404_02346_amd import validation as V
    p = V.point_source_problem(n=16, lam=8.0)
    assert P.check([p]) == 0
    assert P.check([V.point_source_problem(n=16, dim=2)]) == 0
    arr, keep = P.make_descs([p], "f32")
    assert arr[0].src_kind == 1 and tuple(arr[0].src_cell) == (8, 8, 8)
    for field, value in [("xbc", 0), ("src_kind", 2), ("src_kind", -1)]:
        arr, keep = P.make_descs([p], "f32")
        setattr(arr[0], field, value)
        assert P.lib().lb_wave_check(arr, 1) == -1, (field, value)
    for cell in [(16, 0, 0), (0, -1, 0), (0, 0, 16)]:
        arr, keep = P.make_descs([p], "f32")
        for a in range(3):
            arr[0].src_cell[a] = cell[a]
        assert P.lib().lb_wave_check(arr, 1) == -1, cell
    arr, keep = P.make_descs([V.point_source_problem(n=16, dim=2)], "f32")
    arr[0].src_cell[2] = 1  # z must be 0 in 2D
    assert P.lib().lb_wave_check(arr, 1) == -1
    # descriptors without the fields set keep the sheet
    arr, keep = P.make_descs([_cyl()], "f64")
    assert arr[0].src_kind == 0


def test_check_rejects_launches_beyond_32_bit_grids(P):
    # 64 x 8192 x 8192 cells = 2^26 wave tasks of 64 threads: one thread more than a 1D grid holds
    p = {"dim": 3, "nx": 64, "ny": 8192, "nz": 8192, "xbc": "periodic", "c0": 0.5, "radius": 0.0,
         "center": (0, 0, 0), "rho_a": 1.0, "omega": 0.1}
    assert P.check([p], "f16") == -1
    p["nz"] = 8191                                   # 2^26 - 8192 tasks: within the limit
    assert P.check([p], "f16") == 0


def test_check_rejects_mixed_handles(P):
    arr, _ = P.make_descs([_sph(), _sph()], "f32")
    arr[1].storage = 2
    assert P.lib().lb_wave_check(arr, 2) == -1
    assert P.check([_cyl(), _sph()]) == -1
    arr, _ = P.make_descs([_sph()], "f32")
    arr[0].surf_xyz = None
    assert P.lib().lb_wave_check(arr, 1) == -1


def test_workspace_bytes(P):
    p = _sph()
    b = P.workspace_bytes([p], "f32")
    pitch = 64
    assert b >= 2 * 7 * pitch * 32 * 32 * 4
    assert P.workspace_bytes([p], "f64") > b > P.workspace_bytes([p], "f16")
    assert P.workspace_bytes([p], "f32", trace_steps=1000) >= b + 1000 * 24
    assert P.workspace_bytes([p, p], "f32") >= 2 * 2 * 7 * pitch * 32 * 32 * 4
    assert P.workspace_bytes([_sph(cp=0.9)], "f32") == 0
    assert b % 256 == 0


def test_cavity_workspace_bounds(P):
    lib = P.lib()
    assert lib.lb_cavity_workspace_bytes(8) == 0
    assert lib.lb_cavity_workspace_bytes(2049) == 0
    assert lib.lb_cavity_workspace_bytes(128) >= 2 * 128 * 8


def test_create_rejects_bad_workspace_without_device_work(P):
    # argument errors are reported before any device call
    lib = P.lib()
    arr, _ = P.make_descs([_sph()], "f32")
    h = ctypes.c_void_p()
    assert lib.lb_wave_create(arr, 1, None, 0, None, ctypes.byref(h)) == -2
    assert lib.lb_wave_create(arr, 1, ctypes.c_void_p(256), 10, None, ctypes.byref(h)) == -2
    assert lib.lb_wave_create(arr, 1, ctypes.c_void_p(257), 1 << 40, None, ctypes.byref(h)) == -2
    assert lib.lb_wave_destroy(None) == 0
    assert lib.lb_wave_step_n(None, 1) == -1


def test_mlp_sizes_and_argument_errors(P):
    # the surrogate network's host-side checks: sizes and errors before any device call
    from oracle import mlp_oracle as M
    lib = P.lib()
    lib.lb_mlp_workspace_bytes.restype = ctypes.c_size_t
    assert lib.lb_mlp_num_params() == M.num_params()
    assert lib.lb_mlp_workspace_bytes(0) == 0
    assert lib.lb_mlp_workspace_bytes((1 << 24) + 1) == 0
    small, big = lib.lb_mlp_workspace_bytes(256), lib.lb_mlp_workspace_bytes(4096)
    assert 0 < small < big and small % 256 == 0
    h = ctypes.c_void_p()
    assert lib.lb_mlp_create(0, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h)) == -1
    assert lib.lb_mlp_create(256, None, 1 << 40, None, ctypes.byref(h)) == -2
    assert lib.lb_mlp_create(256, ctypes.c_void_p(256), 10, None, ctypes.byref(h)) == -2
    assert lib.lb_mlp_forward(None, None, 1, None) == -1
    assert lib.lb_mlp_forward_layered(None, None, 1, None) == -1
    assert lib.lb_mlp_destroy(None) == 0
    lib.lb_mlp_activation.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_void_p, ctypes.c_void_p]
    assert lib.lb_mlp_activation(None, -1, 0, None, None) == -1
    assert lib.lb_mlp_activation(None, 5, 0, None, None) == -1
    assert lib.lb_mlp_activation(None, 0, 1, None, None) == 0  # nothing to do, no device call
    assert lib.lb_mlp_activation(ctypes.c_void_p(256), (1 << 31) + 1, 0, ctypes.c_void_p(256),
                                 None) == -1              # beyond the 32-bit grid
