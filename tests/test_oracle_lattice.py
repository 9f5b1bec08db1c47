"""Pins of the oracle's lattice algebra against what the paper and mathematics fix.

Each test names the passage it follows.  A plausible slip (a wrong weight,
a dropped (w0 - 1) term, a sign in the kernel, an inverted tanh) fails at
least one of them.
"""
import numpy as np
import pytest


@pytest.mark.parametrize("dim", [2, 3])
def test_velocity_set_isotropy(orc, dim):
    # eq. velocity_properties: sum w = 1, sum w v = 0, sum w v v = cs2 I, sum w v v v = 0;
    # c_s^2 = 1/3 (D2Q5) and 1/4 (D3Q7) stated after eq. feq_waves.
    w, cs2, v = orc.lattice(dim)
    assert len(w) == 2 * dim + 1
    assert cs2 == pytest.approx(1 / 3 if dim == 2 else 1 / 4, abs=0)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.abs(w @ v).max() == 0
    M2 = np.einsum("i,ia,ib->ab", w, v, v)
    np.testing.assert_allclose(M2[:dim, :dim], cs2 * np.eye(dim), atol=1e-15)
    M3 = np.einsum("i,ia,ib,ic->abc", w, v, v, v)
    assert np.abs(M3).max() == 0
    # velocity vectors: rest plus the unit vectors, in +/- pairs
    assert (v[0] == 0).all()
    for i in range(1, 2 * dim + 1, 2):
        assert (v[i] == -v[i + 1]).all() and np.abs(v[i]).sum() == 1


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_moments(orc, dim):
    # eq. feq_waves must give sum f = rho1, sum v f = J1 and the diagonal
    # momentum flux Pi0 = c^2 rho1 I of eq. Pi0_diagonal (p1 = c^2 rho1, eq. MacroscopicFields).
    rng = np.random.Generator(np.random.PCG64(11))
    _, _, v = orc.lattice(dim)
    for _ in range(20):
        c2 = rng.uniform(0.05, 0.3)
        rho = rng.uniform(-1, 1)
        J = rng.uniform(-1, 1, size=dim)
        f = orc.feq(dim, c2, rho, J)
        assert f.sum() == pytest.approx(rho, abs=1e-14)
        np.testing.assert_allclose(v[:, :dim].T @ f, J, atol=1e-14)
        Pi = np.einsum("ia,ib,i->ab", v[:, :dim], v[:, :dim], f)
        np.testing.assert_allclose(Pi, c2 * rho * np.eye(dim), atol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_equilibrium_rest_population(orc, dim):
    # f0^eq = rho (1 + (c^2/cs^2)(w0 - 1)) = rho (1 - dim c^2) for these sets.
    for c2 in (0.1, 0.25, 0.3):
        f = orc.feq(dim, c2, 1.0, [0.0] * dim)
        assert f[0] == pytest.approx(1.0 - dim * c2, rel=1e-14)
        np.testing.assert_allclose(f[1:], c2 / 2, rtol=1e-14)


@pytest.mark.parametrize("dim", [2, 3])
def test_collision_involution_and_invariants(orc, dim):
    # eq. LBM-Collision with tau = 1/2: f_new = 2 f^eq - f.  It keeps rho1 and J1
    # (the moments of f^eq are those of f) and applying it twice is the identity.
    rng = np.random.Generator(np.random.PCG64(12))
    _, _, v = orc.lattice(dim)
    for _ in range(20):
        c2 = rng.uniform(0.05, 0.3)
        f = rng.uniform(-1, 1, size=2 * dim + 1)
        g = orc.collide_cell(dim, c2, f)
        assert g.sum() == pytest.approx(f.sum(), abs=1e-14)
        np.testing.assert_allclose(v.T @ g, v.T @ f, atol=1e-14)
        np.testing.assert_allclose(orc.collide_cell(dim, c2, g), f, atol=1e-14)
        # the closed form of the post-collision state
        rho = f.sum()
        exp = np.empty_like(f)
        exp[0] = 2 * (1 - dim * c2) * rho - f[0]
        for i in range(1, 2 * dim + 1, 2):
            exp[i] = c2 * rho - f[i + 1]
            exp[i + 1] = c2 * rho - f[i]
        np.testing.assert_allclose(g, exp, atol=1e-14)


def test_roma_kernel_values(orc):
    # The printed 3-point kernel: delta(0) = 2/3, delta(1) = 1/6, delta(1/2) = 1/2,
    # delta(3/2) = 0, continuous at |r| = 1/2, zero beyond 3/2, even.
    r = np.array([0.0, 1.0, 0.5, 1.5, 2.0, -1.0, 0.5 - 1e-12, 0.5 + 1e-12])
    d = orc.roma(r)
    np.testing.assert_allclose(d[:6], [2 / 3, 1 / 6, 1 / 2, 0.0, 0.0, 1 / 6], atol=1e-15)
    assert abs(d[6] - d[7]) < 1e-9


def test_roma_kernel_moments(orc):
    # Partition of unity and zero first moment for every offset (so linear
    # fields are interpolated exactly); second moment 1/3 at a node, 1/4 at
    # a half-node (Roma et al. kernel properties).
    j = np.arange(-3, 4)
    for x in np.linspace(-0.5, 0.5, 41):
        w = orc.roma(x - j)
        assert w.sum() == pytest.approx(1.0, abs=1e-14)
        assert (w * (j - x)).sum() == pytest.approx(0.0, abs=1e-14)
        assert (w >= -1e-15).all()
    assert (orc.roma(0.0 - j) * j ** 2).sum() == pytest.approx(1 / 3, abs=1e-14)
    assert (orc.roma(0.5 - j) * (j - 0.5) ** 2).sum() == pytest.approx(1 / 4, abs=1e-14)


def test_sound_speed_profile(orc):
    # eq. sound_speed_object, sign read so that c = c_p inside and c0 outside,
    # half-way (c0 + c_p)/2 on the sphere |r - r0| = R (tanh(0) = 0).
    p = {"dim": 3, "nx": 8, "ny": 8, "nz": 8, "c0": 0.5, "cp": 0.6, "radius": 5.0, "d": 4.0,
         "center": (10.0, 20.0, 30.0)}
    inner = 0.5 - 0.5 * (0.5 - 0.6) * (1 + np.tanh(25.0 / 4.0))
    assert orc.sound_speed(p, 10.0, 20.0, 30.0) == pytest.approx(inner, abs=1e-15)
    assert abs(inner - 0.6) < 1e-5
    assert orc.sound_speed(p, 30.0, 20.0, 30.0) == pytest.approx(0.5, abs=1e-15)
    assert orc.sound_speed(p, 15.0, 20.0, 30.0) == pytest.approx(0.55, abs=1e-15)
    assert orc.sound_speed(p, 10.0, 23.0, 34.0) == pytest.approx(0.55, abs=1e-15)
    # monotone in r, tanh width set by d: at r^2 - R^2 = d, c = c0 - (c0-cp)/2 (1 - tanh 1)
    r = np.sqrt(25.0 + 4.0)
    exp = 0.5 - 0.5 * (0.5 - 0.6) * (1 - np.tanh(1.0))
    assert orc.sound_speed(p, 10.0 + r, 20.0, 30.0) == pytest.approx(exp, abs=1e-15)
    # 2D ignores z
    p2 = dict(p, dim=2)
    assert orc.sound_speed(p2, 10.0, 20.0, 99.0) == pytest.approx(inner, abs=1e-15)
