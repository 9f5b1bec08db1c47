"""Pins of the shape inputs (workloads/shapes.py): mesh topology, closed
surfaces, enclosed volume and area, and the sound-speed field, which for
equal axes must be the sphere of eq. sound_speed_object (checked against the
oracle's own sound speed)."""
import math

import numpy as np
import pytest

from workloads import shapes


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_icosphere_topology(level):
    V, F = shapes.icosphere(level)
    edges = {tuple(sorted(e)) for f in F for e in ((f[0], f[1]), (f[1], f[2]), (f[2], f[0]))}
    assert len(V) - len(edges) + len(F) == 2       # Euler characteristic of a sphere
    assert len(F) == 20 * 4 ** level
    np.testing.assert_allclose(np.linalg.norm(V, axis=1), 1.0, atol=1e-15)
    cen, nrm, area = shapes.mesh_elements(V, F)
    assert np.all(np.sum(cen * nrm, axis=1) > 0)   # outward orientation
    assert np.all(area > 0)


def test_closed_surface_volume_and_area():
    axes = (7.0, 4.0, 3.0)
    for offset in (0.0, 2.0):
        cen, nrm, area = shapes.ellipsoid_surface((30.0, 20.0, 15.0), axes, level=4, offset=offset)
        # a closed surface: sum n dS = 0; the divergence theorem gives the enclosed volume
        np.testing.assert_allclose((nrm * area[:, None]).sum(axis=0), 0.0, atol=1e-10)
        vol = np.sum(np.sum((cen - np.array([30.0, 20.0, 15.0])) * nrm, axis=1) * area) / 3.0
        if offset == 0.0:
            exact = 4.0 / 3.0 * math.pi * np.prod(axes)
            assert abs(vol / exact - 1) < 4e-3           # inscribed polyhedron, 5120 faces
        else:
            inner = 4.0 / 3.0 * math.pi * np.prod(axes)
            assert vol > inner * 1.5                     # the offset surface encloses more
    # sphere: total area -> 4 pi R^2 from below
    cen, nrm, area = shapes.ellipsoid_surface((0, 0, 0), (5.0, 5.0, 5.0), level=4, offset=0.0)
    assert 0.996 < area.sum() / (4 * math.pi * 25.0) < 1.0


def test_offset_surface_stays_two_cells_out():
    axes = np.array([8.0, 4.0, 4.0])
    cen, nrm, area = shapes.ellipsoid_surface((0, 0, 0), axes, level=4, offset=2.0)
    # the element centres lie outside the ellipsoid and at most ~2 cells beyond it along x, y, z
    q = np.sum((cen / axes) ** 2, axis=1)
    assert np.all(q > 1.0)
    assert np.abs(cen).max(axis=0) == pytest.approx(axes + 2.0, abs=0.05)


def test_equal_axes_field_is_the_sphere(orc):
    import workloads
    p = workloads.sphere_3d(40.0, 2 * math.pi / 64, 0.5, shape=(64, 32, 32), lam=64.0, R=6.0,
                            n_surf=64)
    cf = shapes.ellipsoid_c_field((32, 32, 64), p["center"], (6.0, 6.0, 6.0), p["c0"], p["cp"],
                                  p["d"])
    z, y, x = np.meshgrid(np.arange(32), np.arange(32), np.arange(64), indexing="ij")
    ref = orc.sound_speed(p, x.reshape(-1), y.reshape(-1), z.reshape(-1))
    np.testing.assert_allclose(cf, ref, rtol=0, atol=1e-15)
    # c_p at the centre, c0 far outside
    assert cf.max() == pytest.approx(p["cp"], abs=1e-6) and cf.min() == pytest.approx(p["c0"])


# ---------------------------------------------------------------------------
# Any closed mesh: signed distance, inside test, volume and the sound-speed field
# ---------------------------------------------------------------------------

def _sphere_mesh(R, center, level=3):
    V, F = shapes.icosphere(level)
    return V * R + np.asarray(center), F


def test_signed_distance_of_a_sphere_mesh():
    # the inscribed polyhedron lies inside the sphere by at most its sagitta (0.023 cells here)
    R, cen = 5.0, np.array([20.0, 16.0, 16.0])
    V, F = _sphere_mesh(R, cen)
    sd = shapes.mesh_signed_distance_grid(V, F, (8, 4, 4), (32, 28, 28), 7.0)
    z, y, x = np.meshgrid(np.arange(4, 29), np.arange(4, 29), np.arange(8, 33), indexing="ij")
    exact = np.sqrt((x - cen[0]) ** 2 + (y - cen[1]) ** 2 + (z - cen[2]) ** 2) - R
    assert np.abs(sd - np.clip(exact, -7.0, 7.0)).max() < 0.025
    wrong = (np.sign(sd) != np.sign(exact)) & (np.abs(exact) > 0.025)
    assert not wrong.any()
    # the winding-number sign (arbitrary points) agrees with the row-parity sign (grid)
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)[::29].astype(float)
    sw = shapes.mesh_signed_distance(V, F, pts)
    np.testing.assert_array_equal(np.sign(sw), np.sign(sd.ravel()[::29]))
    np.testing.assert_allclose(np.clip(sw, -7, 7), sd.ravel()[::29], atol=1e-12)


def test_peanut_is_closed_non_convex_and_has_its_volume():
    R, eps = 8.0, 0.3
    V, F = shapes.peanut(R, eps, level=3)
    cen, nrm, area = shapes.mesh_elements(V, F)
    np.testing.assert_allclose((nrm * area[:, None]).sum(axis=0), 0.0, atol=1e-10)
    # V = (1/3) int r^3 dOmega = V0 (1 + 3 eps^2 <P4^2> + eps^3 <P4^3>), <P4^2> = 1/9,
    # <P4^3> = 18/1001; the inscribed mesh lies a little below it
    exact = 4 / 3 * math.pi * R ** 3 * (1 + eps ** 2 / 3 + eps ** 3 * 18 / 1001)
    vol = shapes.mesh_volume(V, F)
    assert 0.98 < vol / exact < 1.0
    # non-convex: the chord between the surface points at polar angles 0.34 and 1.33 rad
    # (in the x-y plane) bulges 0.095 R out of the body across the pinch
    def surf(a):
        return R * (1 + eps * (35 * math.cos(a) ** 4 - 30 * math.cos(a) ** 2 + 3) / 8) * \
            np.array([math.cos(a), math.sin(a), 0.0])
    mid = 0.5 * (surf(0.34) + surf(1.33))
    tm = mid[0] / np.linalg.norm(mid)
    assert np.linalg.norm(mid) - R * (1 + eps * (35 * tm ** 4 - 30 * tm ** 2 + 3) / 8) > 0.09 * R
    assert shapes.mesh_signed_distance(V, F, mid[None])[0] > 0.5
    # inside test against the radial definition, away from the facets
    rng = np.random.default_rng(4)
    P = rng.uniform(-11, 11, size=(3000, 3))
    n = np.linalg.norm(P, axis=1)
    t = P[:, 0] / n
    r = R * (1 + eps * (35 * t ** 4 - 30 * t ** 2 + 3) / 8)
    sd = shapes.mesh_signed_distance(V, F, P)
    far = np.abs(n - r) > 0.2
    np.testing.assert_array_equal(sd[far] < 0, (n < r)[far])


def test_mesh_field_of_a_sphere_is_the_sphere(orc):
    # s (s + 2 R) = |r - r0|^2 - R^2 for a sphere: the mesh field reproduces eq. sound_speed_object
    # up to the facets (level 4: sagitta 0.006 cells; slope of c in s about (c_p - c0) R / d)
    nz, ny, nx = 32, 32, 48
    R, cen = 5.0, (22.3, 15.6, 16.2)
    V, F = _sphere_mesh(R, cen, level=4)
    c = shapes.mesh_c_field((nz, ny, nx), V, F, 0.5, 0.6, 4.0)
    p = {"dim": 3, "nx": nx, "ny": ny, "nz": nz, "c0": 0.5, "cp": 0.6, "d": 4.0, "radius": R,
         "center": cen}
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ref = orc.sound_speed(p, x.ravel().astype(float), y.ravel().astype(float),
                          z.ravel().astype(float))
    err = np.abs(c - ref).max()
    cen_f, nrm_f, _ = shapes.mesh_elements(V - np.asarray(cen), F)
    sagitta = R - np.min(np.sum(cen_f * nrm_f, axis=1))      # deepest facet below the sphere
    slope = abs(0.6 - 0.5) / 2 * (2 * R + 2 * sagitta) / 4.0  # max |dc/ds| near s = 0
    print(f"mesh field vs analytic sphere: {err:.2e} (sagitta {sagitta:.4f}, bound "
          f"{slope * sagitta:.2e})")
    assert err <= 1.05 * slope * sagitta
