"""Host checks of the particle-motion integrator (paper_2404_02346_amd/motion.py) with the
small-sphere closed form F = F0 Psi' sin 2kh as the force: symmetry folding, convergence to the
node or the antinode by the sign of the contrast, and the exact solution of the overdamped
equation, tan(kh(t)) = tan(kh0) exp(2 F0 t / gamma')."""
import math

import numpy as np
import pytest

from paper_2404_02346_amd import motion as M


def test_fold_reproduces_the_symmetries():
    F = M.extended(lambda kh: np.sin(2 * kh))
    kh = np.linspace(-7, 7, 301)
    np.testing.assert_allclose(F(kh), np.sin(2 * kh), atol=1e-12)


@pytest.mark.parametrize("f1", [0.3, -0.3])
def test_drift_to_node_or_antinode(f1):
    F = M.extended(lambda kh: f1 * np.sin(2 * kh))
    t, kh = M.integrate(F, [0.2, 0.7, 1.2, 2.0, 2.9], gamma_over_k=1.0, t_end=40.0, dt=0.01)
    target = math.pi / 2 if f1 > 0 else 0.0    # nodes pi/2 + m pi, or antinodes m pi
    d = np.mod(kh[-1] - target, math.pi)
    np.testing.assert_allclose(np.minimum(d, math.pi - d), 0.0, atol=1e-6)


def test_exact_overdamped_solution():
    # dkh/dt = a sin 2kh  =>  tan kh(t) = tan kh0 exp(2 a t)
    a, kh0 = 0.4, 0.3
    t, kh = M.integrate(M.extended(lambda x: a * np.sin(2 * x)), [kh0], 1.0, 3.0, 0.005)
    exact = np.arctan(np.tan(kh0) * np.exp(2 * a * t))
    np.testing.assert_allclose(kh[:, 0], exact, atol=1e-9)
