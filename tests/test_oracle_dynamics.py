"""Pins of the oracle's time stepping, interpolation and surface integral.

Pinned to: the exact discrete dispersion of the tau = 1/2 scheme, global
conservation, time reversibility, the Fourier stability bound, the exact
one-dimensional reduction of the empty driven box, exact interpolation of
linear fields and closed-form surface integrals (divergence theorem).
"""
import math

import numpy as np
import pytest

import workloads

OPP = {2: [0, 2, 1, 4, 3], 3: [0, 2, 1, 4, 3, 6, 5]}


def _periodic(dim, shape, c0, **kw):
    p = {"dim": dim, "nx": shape[-1], "ny": shape[-2], "nz": shape[0] if dim == 3 else 1,
         "xbc": "periodic", "c0": c0, "cp": c0, "radius": 0.0, "center": (0, 0, 0)}
    p.update(kw)
    return p


def _moments(orc, dim, f):
    _, _, v = orc.lattice(dim)
    return f.sum(axis=1), f @ v


def _feq_field(orc, dim, c2, rho):
    return np.stack([orc.feq(dim, c2, r, [0.0] * dim) for r in rho])


def _unstream(orc, p, f):
    # inverse advection in a periodic box: reverse the velocities, stream, reverse back
    P = OPP[p["dim"]]
    return orc.stream(p, f[:, P])[:, P]


@pytest.mark.parametrize("dim,shape,kvec,c", [
    (2, (6, 48), (2 * np.pi * 3 / 48, 0.0), 0.5),
    (2, (16, 32), (2 * np.pi * 2 / 32, 2 * np.pi * 1 / 16), 0.6),
    (3, (8, 8, 32), (2 * np.pi * 2 / 32, 2 * np.pi / 8, 2 * np.pi / 8), 0.5),
    (3, (4, 4, 64), (2 * np.pi / 64, 0.0, 0.0), 0.55),
])
def test_exact_dispersion(orc, dim, shape, kvec, c):
    # f(0) = f^eq(rho_a cos(k.x), 0) in a periodic homogeneous box evolves as
    # rho = rho_a cos(k.x) cos(Omega t) with cos Omega = 1 - c^2 sum_a (1 - cos k_a)
    # (exact for this scheme; the wave equation of eq. LB_waves is its long-wave limit).
    p = _periodic(dim, shape, c)
    grids = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    coords = grids[::-1]  # x, y, (z)
    phase = sum(kvec[a] * coords[a] for a in range(dim)).reshape(-1)
    rho0 = 0.7 * np.cos(phase)
    f0 = _feq_field(orc, dim, c * c, rho0)
    X = _unstream(orc, p, f0)  # post-collision state of step -1 that advects into f(0)
    Om = math.acos(1 - c * c * sum(1 - math.cos(k) for k in kvec[:dim]))
    for n in (1, 7, 40):
        r = orc.run(p, n, fnew_init=X, want_fields=True)
        rho, _ = _moments(orc, dim, r["fnew"])
        np.testing.assert_allclose(rho, rho0 * math.cos(Om * (n - 1)), atol=2e-13)


def test_dispersion_against_wave_speed(orc):
    # Long waves travel at c: Omega / k -> c as k -> 0 (eq. LB_waves, read as
    # d2 rho/dt2 = laplacian(c^2 rho)).
    c = 0.5
    for lam in (64, 256, 1024):
        k = 2 * np.pi / lam
        Om = math.acos(1 - c * c * (1 - math.cos(k)))
        assert abs(Om / (c * k) - 1) < 1.3 * (k ** 2) * (1 - c * c) / 24 + 1e-12
    assert orc.lattice_wavenumber(2 * np.pi * 0.5 / 128, 0.5) == pytest.approx(
        2 * np.pi / 128, rel=1e-4)


@pytest.mark.parametrize("dim,shape", [(2, (12, 20)), (3, (6, 8, 10))])
def test_global_conservation(orc, dim, shape):
    # Collision keeps rho1 and J1 per cell, advection only moves populations:
    # sum rho1 and sum J1 are constant in a periodic box for any c field.
    ncell = int(np.prod(shape))
    Q = 2 * dim + 1
    X = workloads.random_state(5, ncell, Q)
    cf = workloads.random_c_field(6, shape, 0.45, 0.1)
    p = _periodic(dim, shape, 0.45, c_field=cf)
    rho_x, J_x = _moments(orc, dim, X)
    for n in (1, 13, 60):
        rho, J = _moments(orc, dim, orc.run(p, n, fnew_init=X, want_fields=True)["fnew"])
        assert rho.sum() == pytest.approx(rho_x.sum(), abs=1e-12)
        np.testing.assert_allclose(J.sum(axis=0), J_x.sum(axis=0), atol=1e-12)
        assert np.abs(rho - rho_x).max() > 1e-3  # it did move


@pytest.mark.parametrize("dim,shape", [(2, (10, 14)), (3, (6, 7, 9))])
def test_time_reversibility(orc, dim, shape):
    # With tau = 1/2 the step is invertible: reversing the velocities runs it
    # backwards (collision is an involution that commutes with the reversal).
    ncell = int(np.prod(shape))
    Q = 2 * dim + 1
    X0 = workloads.random_state(7, ncell, Q)
    cf = workloads.random_c_field(8, shape, 0.4, 0.1)
    p = _periodic(dim, shape, 0.4, c_field=cf)
    P = OPP[dim]
    n = 25
    Y = orc.run(p, n, fnew_init=X0, want_fields=True)["fnew"]
    Z = orc.run(p, n, fnew_init=orc.stream(p, Y)[:, P], want_fields=True)["fnew"]
    X1 = orc.stream(p, Z)[:, P]
    np.testing.assert_allclose(X1, X0, atol=1e-12)


@pytest.mark.parametrize("dim", [2, 3])
def test_fused_run_equals_composition(orc, dim):
    # orc_run gathers, collides and applies the sheets in one pass; it must
    # equal advection (orc_stream) followed by the per-cell rules written out
    # here from the same primitives, including the interpolated force.
    shape = (4, 5, 11) if dim == 3 else (6, 11)
    nx = shape[-1]
    ncell = int(np.prod(shape))
    Q = 2 * dim + 1
    X = workloads.random_state(9, ncell, Q)
    center = (5.2, 2.4, 1.9)
    xyz = np.array([[3.7, 2.2, 1.6], [6.3, 1.1, 3.4], [5.0, 4.6, 0.2]])[:, :3]
    if dim == 2:
        xyz[:, 2] = 0
    nrm = np.array([[0.6, 0.8, 0.0], [0.0, 0.6, 0.8], [1.0, 0.0, 0.0]])
    area = np.array([0.3, 0.7, 1.1])
    p = {"dim": dim, "nx": nx, "ny": shape[-2], "nz": shape[0] if dim == 3 else 1,
         "xbc": "driven", "c0": 0.45, "cp": 0.52, "radius": 1.5, "d": 4.0, "center": center,
         "rho_a": 0.8, "omega": 0.3, "wall_phi": 0.97, "surf_xyz": xyz, "surf_normal": nrm,
         "surf_area": area, "avg_start": 1}
    n = 4
    r = orc.run(p, n, fnew_init=X, want_fields=True, want_trace=True)
    # the same steps composed by hand
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in ([1] if dim == 2 else []) + list(shape)],
                             indexing="ij")
    c = orc.sound_speed(p, xx.reshape(-1), yy.reshape(-1), zz.reshape(-1))
    prev = X.copy()
    trace = []
    _, _, v = orc.lattice(dim)
    for t in range(n):
        f = orc.stream(p, prev)
        rho, J = _moments(orc, dim, f)
        Jf = np.zeros((ncell, 3))
        Jf[:, :dim] = J[:, :dim]
        rI = np.zeros(3)
        JI = np.zeros((3, 3))
        for k in range(3):
            rI[k], JI[k] = orc.interp(p, rho, Jf, xyz[k])
        trace.append(orc.surface_integral(p, rI, JI))
        new = np.stack([orc.collide_cell(dim, c[i] ** 2, f[i]) for i in range(ncell)])
        xcol = np.arange(ncell) % nx
        P = OPP[dim]
        for i in np.where((xcol == 0) | (xcol == nx - 1))[0]:
            new[i] = p["wall_phi"] * f[i, P]
        for i in np.where(xcol == 1)[0]:
            new[i] = orc.feq(dim, c[i] ** 2, p["rho_a"] * math.sin(p["omega"] * t), J[i, :dim])
        prev = new
    np.testing.assert_allclose(r["fnew"], prev, atol=1e-14)
    trace = np.array(trace)
    np.testing.assert_allclose(r["F_trace"], trace, atol=1e-14)
    np.testing.assert_allclose(r["F_avg"], trace[1:].mean(axis=0), atol=1e-14)
    assert r["n_acc"] == n - 1


def _collision_matrix(orc, dim, c2):
    Q = 2 * dim + 1
    return np.stack([orc.collide_cell(dim, c2, np.eye(Q)[j]) for j in range(Q)], axis=1)


@pytest.mark.parametrize("dim,c_ok,c_bad", [(2, 0.70, 0.72), (3, 0.55, 0.60)])
def test_fourier_stability_bound(orc, dim, c_ok, c_bad):
    # Amplification matrix G(k) = S(k) R over the Brillouin zone: all
    # |eigenvalues| equal 1 for c <= 1/sqrt(dim) (no dissipation at tau = 1/2)
    # and some exceed 1 above the bound.
    _, _, v = orc.lattice(dim)
    ks = np.linspace(-np.pi, np.pi, 13)
    grid = np.array(np.meshgrid(*([ks] * dim), indexing="ij")).reshape(dim, -1).T

    def worst(c):
        R = _collision_matrix(orc, dim, c * c)
        mx, mn = 0.0, 9.0
        for k in grid:
            S = np.diag(np.exp(-1j * (v[:, :dim] @ k)))
            ev = np.abs(np.linalg.eigvals(S @ R))
            mx, mn = max(mx, ev.max()), min(mn, ev.min())
        return mx, mn

    mx, mn = worst(c_ok)
    assert mx < 1 + 1e-9 and mn > 1 - 1e-9
    mx, _ = worst(c_bad)
    assert mx > 1 + 1e-3
    assert c_ok <= 1 / math.sqrt(dim) < c_bad


def test_empty_box_reduces_to_one_dimension(orc):
    # The driven empty box with an x-only state is the same 3-population 1D
    # lattice in D2Q5 and D3Q7 (rest weight 1 - c^2 after summing the
    # transverse populations), so rho1(x, t) agrees to rounding.
    nx, c0, om = 40, 0.5, 2 * np.pi * 0.5 / 40
    base = {"nx": nx, "c0": c0, "cp": c0, "radius": 0.0, "center": (0, 0, 0), "rho_a": 1.0,
            "omega": om, "wall_phi": 0.99}
    r2 = orc.run(dict(base, dim=2, ny=3), 300, line=(0, 300))["rho_line"]
    r3 = orc.run(dict(base, dim=3, ny=3, nz=2), 300, line=(0, 300))["rho_line"]
    r1 = orc.run(dict(base, dim=2, ny=1), 300, line=(0, 300))["rho_line"]
    np.testing.assert_allclose(r3, r2, atol=1e-13)
    np.testing.assert_allclose(r1, r2, atol=1e-13)
    assert np.abs(r2).max() > 0.5


def test_cavity_calibration(orc):
    # The driven box settles into a standing wave: antinodes half a lattice
    # wavelength apart, amplitude close to the imposed rho_a (Sec. Results:
    # source sheet at x = 1, reflector at Lx - 1, one nodal plane per half wave).
    cal = orc.cavity_calibration(128, 0.5, 2 * np.pi * 0.5 / 128)
    k = cal["k"]
    a = np.array(cal["antinodes"])
    np.testing.assert_allclose(np.diff(a), np.pi / k, rtol=1e-12)
    assert 0.95 < cal["A"] < 1.05
    assert cal["Pa"] == pytest.approx(0.25 * cal["A"])
    assert 0 < cal["x_mid"] <= 63.5
    # The fitted amplitude profile is a standing wave: |P| at the fitted
    # antinode is A, and near a node it is much smaller.
    P = np.abs(cal["P"])
    xm = int(round(cal["x_mid"]))
    assert P[xm] == pytest.approx(cal["A"], rel=2e-3)
    node = int(round(cal["x_mid"] + 0.5 * np.pi / k))
    assert P[node] < 0.05 * cal["A"]


@pytest.mark.parametrize("dim", [2, 3])
def test_interpolation_exact_for_linear_fields(orc, dim):
    # Partition of unity and zero first moment of the tensor kernel make the
    # interpolation of eq. InterpolatedFields exact for linear fields.
    shape = (9, 10, 12) if dim == 3 else (10, 12)
    zz, yy, xx = np.meshgrid(*[np.arange(s) for s in ([1] if dim == 2 else []) + list(shape)],
                             indexing="ij")
    x, y, z = xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)
    rho = 0.3 + 0.2 * x - 0.1 * y + (0.05 * z if dim == 3 else 0)
    J = np.stack([1 - 0.3 * x, 0.2 * y + 0.1 * x, (0.4 * z - 0.2 * y) if dim == 3 else 0 * x],
                 axis=1)
    p = {"dim": dim, "nx": shape[-1], "ny": shape[-2], "nz": shape[0] if dim == 3 else 1,
         "c0": 0.5}
    rng = np.random.Generator(np.random.PCG64(3))
    for _ in range(10):
        P = [rng.uniform(2, shape[-1] - 3), rng.uniform(2, shape[-2] - 3),
             rng.uniform(2, shape[0] - 3) if dim == 3 else 0.0]
        rI, JI = orc.interp(p, rho, J, P)
        ez = P[2] if dim == 3 else 0
        assert rI == pytest.approx(0.3 + 0.2 * P[0] - 0.1 * P[1] + (0.05 * ez if dim == 3 else 0),
                                   abs=1e-13)
        np.testing.assert_allclose(
            JI, [1 - 0.3 * P[0], 0.2 * P[1] + 0.1 * P[0], (0.4 * ez - 0.2 * P[1]) if dim == 3 else 0],
            atol=1e-13)
    # periodic wrap in y: a constant field is reproduced next to the y edge
    rI, _ = orc.interp(p, np.full_like(rho, 2.5), J, [5.0, 0.3, 4.0 if dim == 3 else 0.0])
    assert rI == pytest.approx(2.5, abs=1e-14)
    with pytest.raises(ValueError):
        orc.interp(p, rho, J, [0.2, 4.0, 4.0])


def test_surface_integral_divergence_theorem_2d(orc):
    # eq. arf_integral_LBM on a circle of N equal segments, for fields whose
    # flux integral has a closed form (divergence theorem, V = pi Rs^2):
    #   rho = a + b x, J = 0:  F_x = -(c0^2/rho0) b rho(x0) V
    #   rho = 0, J = (b x, 0): F_x = -(b^2/rho0) x0 V
    c0, rho0, Rs, x0 = 0.4, 1.3, 5.0, 11.0
    xyz, nrm, area = workloads.circle_surface((x0, 7.0, 0.0), Rs, 256)
    p = {"dim": 2, "nx": 30, "ny": 20, "c0": c0, "rho0": rho0, "surf_xyz": xyz,
         "surf_normal": nrm, "surf_area": area}
    a, b = 0.7, 0.05
    V = np.pi * Rs ** 2
    F = orc.surface_integral(p, a + b * xyz[:, 0], np.zeros((256, 3)))
    assert F[0] == pytest.approx(-(c0 ** 2 / rho0) * b * (a + b * x0) * V, rel=1e-12)
    assert abs(F[1]) < 1e-14
    J = np.zeros((256, 3))
    J[:, 0] = b * xyz[:, 0]
    F = orc.surface_integral(p, np.zeros(256), J)
    assert F[0] == pytest.approx(-(b ** 2 / rho0) * x0 * V, rel=1e-12)
    # a uniform state carries no net flux through a closed surface
    F = orc.surface_integral(p, np.full(256, 0.3), np.tile([0.2, -0.1, 0.0], (256, 1)))
    assert np.abs(F).max() < 1e-14


def test_surface_integral_divergence_theorem_3d(orc):
    # Same closed forms on the Fibonacci sphere (V = 4/3 pi Rs^3); the point
    # set is equal-area but not exactly symmetric, so the tolerance is the
    # quadrature error of N = 4096 points.
    c0, rho0, Rs, x0 = 0.5, 1.0, 6.0, 20.0
    N = 4096
    xyz, nrm, area = workloads.fibonacci_surface((x0, 9.0, 9.0), Rs, N)
    p = {"dim": 3, "nx": 40, "ny": 20, "nz": 20, "c0": c0, "rho0": rho0, "surf_xyz": xyz,
         "surf_normal": nrm, "surf_area": area}
    a, b = 0.7, 0.05
    V = 4 / 3 * np.pi * Rs ** 3
    F = orc.surface_integral(p, a + b * xyz[:, 0], np.zeros((N, 3)))
    assert F[0] == pytest.approx(-(c0 ** 2 / rho0) * b * (a + b * x0) * V, rel=2e-3)
    J = np.zeros((N, 3))
    J[:, 0] = b * xyz[:, 0]
    F = orc.surface_integral(p, np.zeros(N), J)
    assert F[0] == pytest.approx(-(b ** 2 / rho0) * x0 * V, rel=2e-3)


def test_segmented_run_equals_one_run(orc):
    # a driven 3D box with an object and surface measurement across the averaging start,
    # split into uneven pieces: the same time-averaged force, bit for bit
    import workloads
    cal = orc.cavity_calibration(32, 0.5, 2 * math.pi * 0.5 / 32, n_periods=10)
    p = workloads.sphere_3d(cal["x_mid"], cal["k"], 0.5, n_periods=3, avg_periods=1,
                            shape=(32, 16, 16), lam=32.0, R=2.0, n_surf=128)
    one = orc.run(p, p["n_steps"])
    seg = orc.run_segments(p, p["n_steps"], 5)
    assert seg["n_acc"] == one["n_acc"] > 0
    assert np.array_equal(seg["F_avg"], one["F_avg"])
