"""The oracle's oscillating point source against the Green's function of the wave equation.

Pins (Sec. "Lattice-Boltzmann for acoustics", eq. waves_with_pointSource and the
solution after it): one node of a periodic cube imposed with rho1 = rho_a sin(w t)
(the source-sheet rule, eq. imposingfields) radiates the outgoing spherical wave
rho1 = A sin(w t - k r + phi) / r of the 3D wave equation.  Before any image from
the periodic copies arrives, the complex amplitude P(r) at the drive frequency
therefore has
  * |P| r constant along a ray (the 1/r decay of the Green's function),
  * phase -k r + const, with k the wavenumber of the exact lattice dispersion
    1 - cos w = c^2 sum_a (1 - cos k_a) along that ray (axis and face diagonal
    differ by 0.6%, the continuum value w / c by 0.9% on the axis and 0.3% on the
    diagonal at 12 cells per wavelength, so the fitted k tells them apart).  Near
    a node-sized source the lattice adds a small near-field phase b / r (about
    0.17 rad at r = 1), fitted beside k,
  * the same values on all six axis rays (the lattice symmetries), and amplitudes
    on the face diagonal within the lattice anisotropy (3% at 12 cells per
    wavelength) of the axis ones;
and the source node's post-collision state carries exactly rho_a sin(w t).  The amplitude A has no
prediction here: the printed prefactor is dimensionally inconsistent and a
node-sized source has no continuum strength.  In 2D the exact outgoing Green's
function H0^(2)(k r), near field included, fits each ray with one complex constant.
"""
import math

import numpy as np
import pytest

import oracle

N, LAM, C0, RHO_A = 64, 12.0, 0.5, 1.0
OM = 2 * math.pi * C0 / LAM
T = int(round(2 * math.pi / OM))
S = N // 2
R_FIT = 16
T_END = int((N - R_FIT) / C0) - 4      # before the first image reaches r = 16
T0 = T_END - T                        # one period after the direct wave passed r = 16


def cell(x, y, z):
    return (z * N + y) * N + x


def k_along(u):
    # bisection on the exact lattice dispersion for the wave vector k u / |u|
    u = np.asarray(u, float) / np.linalg.norm(u)
    lo, hi = 0.0, math.pi
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if C0 ** 2 * np.sum(1 - np.cos(mid * u)) < 1 - math.cos(OM):
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


@pytest.fixture(scope="module")
def run():
    p = {"dim": 3, "nx": N, "ny": N, "nz": N, "xbc": "periodic", "c0": C0, "rho_a": RHO_A,
         "omega": OM, "radius": 0.0, "center": (0, 0, 0), "src_cell": (S, S, S)}
    m = np.arange(1, R_FIT + 1)
    rays = {
        "+x": [cell(S + i, S, S) for i in m], "-x": [cell(S - i, S, S) for i in m],
        "+y": [cell(S, S + i, S) for i in m], "-y": [cell(S, S - i, S) for i in m],
        "+z": [cell(S, S, S + i) for i in m], "-z": [cell(S, S, S - i) for i in m],
        "xy": [cell(S + i, S + i, S) for i in range(1, 12)],
    }
    names = list(rays)
    probes = sum((rays[k] for k in names), []) + [cell(S, S, S)]
    out = oracle.run(p, T_END, line=(T0, T), probes=probes, want_fields=True)
    rp = out["rho_probe"]
    t = np.arange(T0, T_END)
    P = (2.0 / T) * (rp * np.exp(-1j * OM * t)[:, None]).sum(axis=0)
    res, j = {}, 0
    for k in names:
        n = len(rays[k])
        res[k] = P[j: j + n]
        j += n
    return res, out["fnew"][cell(S, S, S)].sum()


def fit_phase(P, r):
    # phase = a - k r + b / r by least squares
    ph = np.unwrap(np.angle(P))
    A = np.stack([np.ones_like(r), -r, 1.0 / r], axis=1)
    c, *_ = np.linalg.lstsq(A, ph, rcond=None)
    return c[1], c[2], float(np.abs(A @ c - ph).max())


def test_source_node_carries_the_drive(run):
    _, src = run
    assert src == pytest.approx(RHO_A * math.sin(OM * (T_END - 1)), abs=1e-14)


def test_one_over_r_decay_on_the_axis(run):
    res, _ = run
    r = np.arange(1, R_FIT + 1, dtype=float)
    far = (np.abs(res["+x"]) * r)[3:]          # r = 4 .. 16
    print(f"|P| r on the axis, r = 4..16: {far.min():.5f} .. {far.max():.5f}")
    assert far.max() / far.min() - 1 < 0.02
    # a constant or a 1/r^2 amplitude would fail by far
    assert abs(res["+x"][3]) / abs(res["+x"][15]) == pytest.approx(4.0, rel=0.02)


@pytest.mark.parametrize("ray,d,m_max", [("+x", (1, 0, 0), R_FIT), ("xy", (1, 1, 0), 11)])
def test_phase_advances_at_the_lattice_wavenumber(run, ray, d, m_max):
    res, _ = run
    r = np.linalg.norm(d) * np.arange(1, m_max + 1, dtype=float)
    sel = r >= 4
    k, b, resid = fit_phase(res[ray][sel], r[sel])
    k_lat = k_along(d)
    print(f"{ray}: fitted k {k:.5f}, lattice {k_lat:.5f}, w/c {OM / C0:.5f}, near-field b {b:.3f}, "
          f"residual {resid:.1e} rad")
    assert k == pytest.approx(k_lat, rel=1.5e-3)
    assert abs(k - OM / C0) > 2 * abs(k - k_lat)
    assert resid < 1e-2


def test_symmetric_and_nearly_isotropic(run):
    res, _ = run
    for k in ("-x", "+y", "-y", "+z", "-z"):
        assert np.allclose(res[k], res["+x"], rtol=1e-10, atol=1e-14), k
    r_ax = np.arange(1, R_FIT + 1)
    r_d = math.sqrt(2) * np.arange(1, 12)
    a_ax = np.mean(np.abs(res["+x"][5:]) * r_ax[5:])
    a_d = np.mean(np.abs(res["xy"][4:]) * r_d[4:])
    print(f"|P| r: axis {a_ax:.5f}, face diagonal {a_d:.5f}")
    assert a_d / a_ax - 1 == pytest.approx(0.0, abs=0.04)


def test_2d_field_is_the_hankel_function():
    # In 2D the outgoing Green's function is H0^(2)(k r) (times e^{i w t}), near field included:
    # with the lattice k of each ray, one complex constant C fits the whole ray within 1% from
    # r = 4 on (0.62% at most), and the axis and the face diagonal give the same C (isotropy).
    # The continuum wavenumber w / c leaves 6% on the axis and 1.7% on the diagonal (whose
    # lattice k is closer to it) even with C refitted.
    from scipy.special import hankel2
    n, lam, r_fit = 256, 16.0, 48
    om = 2 * math.pi * C0 / lam
    period = int(round(2 * math.pi / om))
    s = n // 2
    p = {"dim": 2, "nx": n, "ny": n, "xbc": "periodic", "c0": C0, "rho_a": RHO_A, "omega": om,
         "radius": 0.0, "center": (0, 0, 0), "src_cell": (s, s, 0)}
    m_ax = np.arange(1, r_fit + 1)
    m_d = np.arange(1, int(r_fit / math.sqrt(2)) + 1)
    cells = [s * n + s + i for i in m_ax] + [(s + i) * n + s + i for i in m_d]
    t_end = int((n - r_fit) / C0) - 4
    t0 = t_end - period
    rp = oracle.run(p, t_end, line=(t0, period), probes=cells)["rho_probe"]
    t = np.arange(t0, t_end)
    P = (2.0 / period) * (rp * np.exp(-1j * om * t)[:, None]).sum(axis=0)
    fits = []
    for Pr, r, u in ((P[:m_ax.size], m_ax.astype(float), (1, 0, 0)),
                     (P[m_ax.size:], math.sqrt(2) * m_d, (1, 1, 0))):
        u = np.asarray(u, float) / np.linalg.norm(u)
        lo, hi = 0.0, math.pi
        for _ in range(200):
            mid = 0.5 * (lo + hi)
            if C0 ** 2 * np.sum(1 - np.cos(mid * u)) < 1 - math.cos(om):
                lo = mid
            else:
                hi = mid
        k = 0.5 * (lo + hi)
        sel = r >= 4
        for kk, must_fit in ((k, True), (om / C0, False)):
            H = hankel2(0, kk * r[sel])
            C = np.vdot(H, Pr[sel]) / np.vdot(H, H)
            resid = np.max(np.abs(Pr[sel] - C * H) / np.abs(Pr[sel]))
            print(f"2D ray ({u[0]:.3f}, {u[1]:.3f}), k {kk:.5f}: C = {C:.5f}, "
                  f"max residual {resid:.2e}")
            if must_fit:
                assert resid < 8e-3
                fits.append(C)
            else:
                assert resid > 1.2e-2
    assert abs(fits[1] / fits[0] - 1) < 0.02
