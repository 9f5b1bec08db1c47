"""Plane interface between two media (eq. c_plane_int) on the FP64 oracle.

The paper checks pressure and normal-velocity continuity across the
interface to 1%; here also the energy flux balance, the sharp-interface
coefficients (for a narrow interface, w = 0.5 cell) and the weaker reflection
of a wider one (w = 2 cells).  paper_2404_02346_amd/validation.py holds the
set-up and the fit (no method arithmetic: it reads rho1(x, t))."""
import numpy as np
import pytest

from paper_2404_02346_amd import validation as V


def run_oracle(orc, w):
    p = V.interface_problem(w=w)
    t0, n = V.window(p)
    r = orc.run(p, t0 + n, line=(t0, n))
    return p, V.coefficients(p, r["rho_line"].reshape(n, p["nx"]), t0)


def test_narrow_interface(orc):
    p, c = run_oracle(orc, 0.5)
    print(c)
    assert c["backward"] < 1e-6                     # no wave back from the far wall yet
    assert abs(c["energy"] - 1) < 0.01
    assert c["pressure_continuity"] < 0.01 and c["velocity_continuity"] < 0.01
    assert abs(abs(c["R"]) / abs(c["R_sharp"]) - 1) < 0.015
    assert abs(abs(c["T"]) / c["T_sharp"] - 1) < 0.01
    assert c["R"].real < 0                          # slower medium: pressure reflects inverted


def test_wide_interface_reflects_less(orc):
    _, narrow = run_oracle(orc, 0.5)
    _, wide = run_oracle(orc, 2.0)
    assert abs(wide["energy"] - 1) < 0.01
    assert abs(wide["R"]) < 0.95 * abs(narrow["R"])


def test_lattice_wavenumber():
    # exact discrete dispersion against the continuum k = w / c for long waves
    w = 2 * np.pi * 0.5 / 64
    assert V.lattice_k(w, 0.5) == pytest.approx(w / 0.5, rel=1e-3)
    assert V.lattice_k(w, 0.25) == pytest.approx(w / 0.25, rel=2e-3)
    assert np.cos(w) == pytest.approx(1 - 0.25 ** 2 * (1 - np.cos(V.lattice_k(w, 0.25))), abs=1e-15)
