"""The calibration entry point that allocates nothing (lb_cavity_calibrate_noalloc), through the
C ABI, against lb_cavity_calibrate on the same arguments: every output bit for bit, on two
calls in a row, the second on a smaller box (the scratch array keeps the first call's sums,
which the second call must fully overwrite for its own nx)."""
import ctypes as C
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_02346_amd as P
    L = P.lib()
    dp = C.POINTER(C.c_double)
    L.lb_cavity_workspace_bytes.argtypes = [C.c_int32]
    L.lb_cavity_workspace_bytes.restype = C.c_size_t
    L.lb_cavity_calibrate.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double, C.c_double,
                                      C.c_int32, C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                                      dp, dp]
    L.lb_cavity_calibrate_noalloc.argtypes = [C.c_int32, C.c_double, C.c_double, C.c_double,
                                              C.c_double, C.c_int32, C.c_int32, C.c_void_p, dp,
                                              dp]
    return L


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _both(L, nx, c0, n_periods=30, n_fit=5):
    import torch
    omega = 2 * math.pi * c0 / nx
    stream = torch.cuda.current_stream()
    nb = L.lb_cavity_workspace_bytes(nx)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    out_a, P_a = np.zeros(6), np.zeros(2 * nx)
    out_b, P_b = np.zeros(6), np.zeros(2 * nx)
    st = L.lb_cavity_calibrate(nx, c0, omega, 1.0, 0.99, n_periods, n_fit,
                               C.c_void_p(ws.data_ptr()), nb, C.c_void_p(stream.cuda_stream),
                               _ptr(out_a), _ptr(P_a))
    assert st == 0
    st = L.lb_cavity_calibrate_noalloc(nx, c0, omega, 1.0, 0.99, n_periods, n_fit,
                                       C.c_void_p(stream.cuda_stream), _ptr(out_b), _ptr(P_b))
    assert st == 0
    return out_a, P_a, out_b, P_b


def test_noalloc_matches_workspace_calibration(lib):
    for nx, c0 in ((256, 0.5), (96, 1.0 / 3.0)):  # the second call on a smaller box
        out_a, P_a, out_b, P_b = _both(lib, nx, c0)
        print(f"nx={nx}: A={out_b[0]:.10f} x_a={out_b[1]:.6f} k={out_b[2]:.8f}", flush=True)
        assert np.array_equal(out_a, out_b)
        assert np.array_equal(P_a, P_b)
        assert 0.9 < out_b[0] < 1.1 and 0 < out_b[1] < nx


def test_noalloc_rejects_sizes_beyond_its_array(lib):
    import torch
    out = np.zeros(6)
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert lib.lb_cavity_calibrate_noalloc(2049, 0.5, 2 * math.pi * 0.5 / 2049, 1.0, 0.99, 30, 5,
                                           s, _ptr(out), None) == -1
    assert lib.lb_cavity_calibrate_noalloc(64, 0.5, 2 * math.pi * 0.5 / 64, 1.0, 0.99, 30, 5, s,
                                           None, None) == -1
