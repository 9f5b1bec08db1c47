"""Plane interface (eq. c_plane_int) on the GPU library: the coefficients
fitted from the GPU's rho1(x, t) equal the oracle's (FP64 parity), and the
physics bands of tests/test_oracle_interface.py hold for FP64 and FP32."""
import pytest

from paper_2404_02346_amd import validation as V

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_02346_amd as P
    P.lib()
    return P


@pytest.mark.parametrize("storage,tol", [("f64", 1e-10), ("f32", 1e-4)])
def test_interface_gpu_against_oracle(gpu, orc, storage, tol):
    p = V.interface_problem(w=0.5)
    t0, n = V.window(p)
    ref = V.coefficients(p, orc.run(p, t0 + n, line=(t0, n))["rho_line"].reshape(n, p["nx"]), t0)
    got = V.coefficients(p, V.rho_window_gpu(p, t0, n, storage), t0)
    print(f"{storage}: R {got['R']:.6f} (oracle {ref['R']:.6f}), T {got['T']:.6f}, "
          f"energy {got['energy']:.5f}, continuity p {got['pressure_continuity']:.2e} "
          f"u {got['velocity_continuity']:.2e}", flush=True)
    assert abs(got["R"] - ref["R"]) < tol and abs(got["T"] - ref["T"]) < tol
    assert abs(got["energy"] - 1) < 0.01
    assert got["pressure_continuity"] < 0.01 and got["velocity_continuity"] < 0.01
