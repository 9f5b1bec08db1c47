"""Host checks of the sweep fits (power laws, linear law) on exact synthetic data."""
import math

import numpy as np
import pytest

from paper_2404_02346_amd import sweeps as SW


def test_power_fit_recovers_exact_exponents():
    x = np.array([0.5, 1.0, 2.0, 3.0, 7.0])
    for e in (1.0, 2.0, 3.0, -0.5):
        got, r2 = SW.fit_power(x, 3.7 * x ** e)
        assert got == pytest.approx(e, abs=1e-12) and r2 == pytest.approx(1.0, abs=1e-12)
    got, _ = SW.fit_power(x, -2.0 * x ** 2)  # sign does not enter the exponent
    assert got == pytest.approx(2.0, abs=1e-12)


def test_linear_fit_and_r2():
    x = np.linspace(-8, 8, 5)
    a, b, r2 = SW.fit_linear(x, 0.3 * x - 0.1)
    assert a == pytest.approx(0.3) and b == pytest.approx(-0.1) and r2 == pytest.approx(1.0)
    rng = np.random.Generator(np.random.PCG64(1))
    y = 0.3 * x + rng.normal(0, 0.5, 5)
    _, _, r2n = SW.fit_linear(x, y)
    assert 0.0 < r2n < 1.0


def test_contrast_factor_and_sweep_layout():
    assert SW.psi(0.25, 0.25) == 0.0
    for v in SW.SWEEPS["Psi"]:
        cp = 1.0 / math.sqrt(1.0 / SW.PSI_C0 ** 2 - v)
        assert SW.psi(SW.PSI_C0, cp) == pytest.approx(v, abs=1e-12)
        assert cp < 1 / math.sqrt(3)  # stable on D3Q7 with tau = 1/2
    # every box's drive period is a whole number of steps and the objects clear the sheets
    import workloads
    cal = {"x_mid": 126.63, "k": 2 * math.pi / 256, "A": 0.99}
    for dim in (2, 3):
        for lam in SW.SWEEPS["k"]:
            c = {"x_mid": lam / 2 - 1.37, "k": 2 * math.pi / lam, "A": 0.99}
            assert workloads.geometry_ok(SW.problem(dim, c, lam))
        for R in SW.SWEEPS["R"]:
            assert workloads.geometry_ok(SW.problem(dim, cal, SW.LAM_DEF, R=R))
