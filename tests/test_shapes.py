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
