"""Particle motion driven by the trained surrogate's force (paper_2404_02346_amd/motion.py).

A density-matched sphere (kR = 0.3, R = 8 cells) in the overdamped regime
drifts to the pressure node when c_p > c_0 (Psi > 0) and to the antinode
when c_p < c_0, from any starting phase, up to where the network's force
vanishes (within its accuracy of the node); near the node the approach is
exponential with the rate -F'(node)/gamma given by the surrogate's own slope.
"""
import json
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu
DATA = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                    "paper_2404_02346_amd", "data")
HELD_OUT_MAX = 0.0056  # the surrogate's held-out maximum error, in units of TEST_F_SCALE
TEST_F_SCALE = 0.5596  # largest |F/F0| of the 600 held-out LB forces


@pytest.fixture(scope="module")
def net():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02346_amd import surrogate as S
    if not all(os.path.exists(f) for f in S.data_paths(S.TRAIN_FILES)):
        pytest.skip("no LB force data")
    mlp, _, _ = S.fit(S.load_sets(S.TRAIN_FILES))
    yield mlp
    mlp.close()


@pytest.mark.parametrize("ratio,target", [(1.2, math.pi / 2), (0.85, 0.0)])
def test_drift_to_node_or_antinode(net, ratio, target):
    from paper_2404_02346_amd import motion as M
    F = M.extended(M.surrogate_force(net, 0.3, ratio, 8.0))
    kh0 = [0.15, 0.6, 1.0, 1.4, 2.2, 2.9]
    t, kh = M.integrate(F, kh0, gamma_over_k=1.0, t_end=60.0, dt=0.02)
    end = np.mod(kh[-1] - target + math.pi / 2, math.pi) - math.pi / 2  # offset from the target
    print(f"c_p/c0 = {ratio}: stops at {'node' if target else 'antinode'} + "
          f"{np.array2string(end, precision=6)}", flush=True)
    # every start ends the same distance from the node or antinode (from either side, by the
    # mirror symmetry of the folded force): at the network's own zero of the force.  The
    # network runs in BF16, so near its zero the force is resolved to a few 1e-5 of F0 and
    # the stopping points of different starts spread by about that over the slope (~1e-5 rad).
    # Where that zero lies: the network's error moves it (near a zero F/F0 ~ 2 f1 (kh - kh*),
    # f1 = 1 - (c0/c_p)^2, so an error e in F/F0 moves it by e / (2 |f1|); the stated held-out
    # error, at most 0.56% of the test set's largest |F/F0| (0.5596), allows 5.1e-3 rad at
    # c_p/c0 = 1.2 and 4.1e-3 rad at 0.85), and the driven box itself does not put the zero
    # exactly on the ideal antinode: its standing wave carries a small travelling part, and the
    # FP64 oracle's force on the small sphere of the test below is F(0)/F0 = 3.7e-3 at the
    # antinode (a shift of 6e-3 rad) but -1e-4 at the node.  The sum, 1.2e-2, bounds the stop.
    # (The test below compares the stops with the oracle's own force table instead.)
    allowance = HELD_OUT_MAX * TEST_F_SCALE / (2 * abs(1 - 1 / ratio ** 2))
    assert np.ptp(np.abs(end)) < 1e-4
    assert np.abs(end).max() < allowance + 6e-3


def test_relaxation_rate_near_the_node(net):
    from paper_2404_02346_amd import motion as M
    Fh = M.surrogate_force(net, 0.3, 1.2, 8.0)
    F = M.extended(Fh)
    e = 0.05
    slope = (Fh(np.array([math.pi / 2 - e]))[0] - Fh(np.array([math.pi / 2 - 3 * e]))[0]) / (2 * e)
    t, kh = M.integrate(F, [math.pi / 2 - 0.2], gamma_over_k=1.0, t_end=4.0, dt=0.01)
    dist = math.pi / 2 - kh[:, 0]
    sel = (dist < 0.15) & (dist > 0.05)
    rate = -np.polyfit(t[sel], np.log(dist[sel]), 1)[0]
    print(f"approach rate {rate:.4f}, slope of F below the node {slope:.4f}", flush=True)
    assert rate == pytest.approx(-slope, rel=0.1)


GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                    "motion_sphere60_oracle_forces.json")


def test_against_the_oracle_force_table(net):
    # Reference: the FP64 oracle's time-averaged force on a sphere R = 4 cells in a 60^3 box
    # (lambda = 60, k R = 0.419, c_p/c0 = 1.2, c0 = 1/3) at kh_j = j (pi/2)/8, written by
    # tests/golden/make_motion_goldens.py.  The table is smoothed by least squares in
    # {1, cos 2kh, sin 2kh, cos 4kh, sin 4kh} and folded by the same symmetries as the
    # surrogate's force; the same RK4 then drives both.  Required: the surrogate's F/F0 at the
    # nine phases within the 2% force-error target of the table's largest |F/F0|, the stopping
    # phases within the allowance of the surrogate's stated error (see above), and the final
    # approach rates within 10%.
    from paper_2404_02346_amd import motion as M
    d = json.load(open(GOLD))
    lam, R, ratio, c0 = d["lam"], d["R"], d["cp_ratio"], d["c0"]
    kR = 2 * math.pi * R / lam
    F0 = math.pi * R ** 3 * d["Pa"] ** 2 * (2 * math.pi / lam) / (3 * c0 ** 2)
    kh = np.array([q["kh"] for q in d["positions"]])
    Fo = np.array([q["F_avg"][0] for q in d["positions"]]) / F0
    basis = lambda x: np.stack([np.ones_like(x), np.cos(2 * x), np.sin(2 * x), np.cos(4 * x),
                                np.sin(4 * x)], axis=1)
    coef, *_ = np.linalg.lstsq(basis(kh), Fo, rcond=None)
    fit_res = np.abs(basis(kh) @ coef - Fo).max() / np.abs(Fo).max()
    Fs_half = M.surrogate_force(net, kR, ratio, R)
    Fs_tab = Fs_half(kh)
    table_err = np.abs(Fs_tab - Fo).max() / np.abs(Fo).max()
    print(f"oracle table F/F0 {np.array2string(Fo, precision=4)}", flush=True)
    print(f"surrogate     F/F0 {np.array2string(Fs_tab, precision=4)}", flush=True)
    print(f"table error {table_err:.4f} of max |F/F0|, smoothing residual {fit_res:.2e}", flush=True)
    assert fit_res < 1e-2
    assert table_err < 0.02

    Fo_fun = M.extended(lambda x: basis(np.atleast_1d(x)) @ coef)
    Fs_fun = M.extended(Fs_half)
    starts = [0.6, 1.0, 1.3, 1.8, 2.2]
    _, kh_s = M.integrate(Fs_fun, starts, gamma_over_k=1.0, t_end=80.0, dt=0.02)
    _, kh_o = M.integrate(Fo_fun, starts, gamma_over_k=1.0, t_end=80.0, dt=0.02)
    end_s = np.mod(kh_s[-1], math.pi) - math.pi / 2
    end_o = np.mod(kh_o[-1], math.pi) - math.pi / 2
    allowance = HELD_OUT_MAX * TEST_F_SCALE / (2 * abs(1 - 1 / ratio ** 2))
    print(f"stops at the node + {np.array2string(end_s, precision=6)} (surrogate), "
          f"+ {np.array2string(end_o, precision=6)} (oracle table); allowance {allowance:.2e}",
          flush=True)
    assert np.abs(end_s - end_o).max() < allowance

    # final approach from below: distance to each trajectory's own end point, exponential rate
    t, ks = M.integrate(Fs_fun, [math.pi / 2 - 0.2], gamma_over_k=1.0, t_end=6.0, dt=0.01)
    _, ko = M.integrate(Fo_fun, [math.pi / 2 - 0.2], gamma_over_k=1.0, t_end=6.0, dt=0.01)

    def rate(k, stop):
        dist = stop - k[:, 0]
        sel = (dist < 0.15) & (dist > 0.05)
        return -np.polyfit(t[sel], np.log(dist[sel]), 1)[0]

    rs, ro = rate(ks, math.pi / 2 + end_s[0]), rate(ko, math.pi / 2 + end_o[0])  # from below
    print(f"approach rate: surrogate {rs:.4f}, oracle table {ro:.4f}", flush=True)
    assert rs == pytest.approx(ro, rel=0.1)
