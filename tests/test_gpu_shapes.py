"""Objects of other shapes (workloads/shapes.py) on the GPU library.

* Parity: an ellipsoid, and a non-convex peanut whose sound speed comes from
  the signed distance to its triangle mesh, each given as a per-cell
  sound-speed field with a triangle-mesh integration surface, GPU against the
  FP64 oracle element by element (one and two steps per launch).
* Physics: a density-matched object scatters as a monopole to leading order
  in kR, so its force depends on its volume, not its shape: prolate and
  oblate ellipsoids of the sphere's volume, in any orientation, feel the
  sphere's force within the finite-kR and resolution error (kR = 0.12 here),
  with no transverse force; so does the non-convex peanut of the sphere's
  volume, with its lobes along x or along y.  The mesh-integrated sphere must
  also agree with the Fibonacci-integrated one.
"""
import math

import numpy as np
import pytest

import workloads
from workloads import shapes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_02346_amd as P
    P.lib()
    return P


def say(*a):
    print(*a, flush=True)


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(b).max())


def small_ellipsoid():
    nz, ny, nx = 24, 32, 64
    c0 = 0.45
    center = (35.2, 16.3, 11.8)
    xyz, nrm, area = workloads.fibonacci_surface(center, 5.0, 8)  # replaced below
    base = {"dim": 3, "nx": nx, "ny": ny, "nz": nz, "xbc": "driven", "c0": c0, "rho0": 1.0,
            "center": center, "radius": 3.0, "cp": 0.55, "d": 4.0, "rho_a": 1.0,
            "omega": 2 * np.pi * c0 / nx, "wall_phi": 0.99, "surf_xyz": xyz,
            "surf_normal": nrm, "surf_area": area, "avg_start": 4}
    return shapes.ellipsoid_problem(base, (5.0, 3.0, 2.5), level=3)


def small_peanut():
    base = small_ellipsoid()
    V, F = shapes.peanut(4.5, 0.3, level=2)
    return shapes.mesh_problem(base, V, F)


@pytest.mark.parametrize("shape", ["ellipsoid", "peanut"])
@pytest.mark.parametrize("storage,spl,tol", [("f64", 1, 1e-12), ("f64", 2, 1e-12),
                                             ("f32", 1, 1e-5), ("f32", 2, 1e-5)])
def test_ellipsoid_parity(P, orc, shape, storage, spl, tol):
    p = small_ellipsoid() if shape == "ellipsoid" else small_peanut()
    n = 20
    init = workloads.random_state(91, p["nx"] * p["ny"] * p["nz"], 7)
    say(f"{shape} parity {storage}, {spl} steps per launch, {len(p['surf_area'])} elements")
    ref = orc.run(p, n, fnew_init=init, want_fields=True, want_trace=True)
    h = P.LBWave([p], storage=storage, trace_steps=n)
    h.set_steps_per_launch(spl)
    h.set_state(0, init)
    h.step(n)
    ef, et = rel(h.get_state(0), ref["fnew"]), rel(h.trace(0, n), ref["F_trace"])
    F, nacc = h.force()
    h.close()
    say(f"  field {ef:.2e} trace {et:.2e}")
    assert ef <= tol and et <= 10 * tol and nacc[0] == ref["n_acc"]


def test_force_depends_on_volume_not_shape(P):
    from paper_2404_02346_amd import sweeps as SW
    lam = 256
    cal = P.cavity_calibrate(lam, SW.C0, 2 * math.pi * SW.C0 / lam)
    sphere = SW.problem(3, cal, lam, R=5.0)                  # analytic object, Fibonacci surface
    b = math.sqrt(125.0 / 7.5)
    shapes_axes = {"sphere (mesh)": (5.0, 5.0, 5.0), "prolate along x": (7.5, b, b),
                   "prolate along y": (b, 7.5, b), "oblate, thin along x": (3.2, 6.25, 6.25)}
    probs = [sphere] + [shapes.ellipsoid_problem(sphere, ax, level=4) for ax in shapes_axes.values()]
    # the non-convex peanut of the sphere's volume, lobes along x, then turned to lie along y
    V1, F1 = shapes.peanut(1.0, 0.3, level=3)
    Rp = (4.0 / 3.0 * math.pi * 125.0 / shapes.mesh_volume(V1, F1)) ** (1.0 / 3.0)
    PV, PF = shapes.peanut(Rp, 0.3, level=3)
    PVy = np.stack([-PV[:, 1], PV[:, 0], PV[:, 2]], axis=1)       # 90 degrees about z
    shapes_axes["peanut, lobes along x"] = f"R = {Rp:.3f}"
    shapes_axes["peanut, lobes along y"] = f"R = {Rp:.3f}"
    probs += [shapes.mesh_problem(sphere, PV, PF), shapes.mesh_problem(sphere, PVy, PF)]
    h = P.LBWave(probs, storage="f32")
    h.autotune(2)
    h.set_graph(64)
    h.step(probs[0]["n_steps"])
    F, _ = h.force()
    h.close()
    F0 = F[0, 0]
    say(f"sphere (Fibonacci): F = {F[0]}")
    for (name, ax), Fi in zip(shapes_axes.items(), F[1:]):
        say(f"  {name} {ax}: F_x / F_sphere = {Fi[0] / F0:.4f}, |F_y|, |F_z| / F_x = "
            f"{abs(Fi[1] / Fi[0]):.1e}, {abs(Fi[2] / Fi[0]):.1e}")
        assert abs(Fi[1]) < 0.01 * abs(Fi[0]) and abs(Fi[2]) < 0.01 * abs(Fi[0])
    assert abs(F[1, 0] / F0 - 1) < 0.01          # mesh against Fibonacci integration
    for Fi in F[2:]:
        assert abs(Fi[0] / F0 - 1) < 0.10        # equal volume, other shapes
