"""Particle motion driven by the trained surrogate's force (paper_2404_02346_amd/motion.py).

A density-matched sphere (kR = 0.3, R = 8 cells) in the overdamped regime
drifts to the pressure node when c_p > c_0 (Psi > 0) and to the antinode
when c_p < c_0, from any starting phase; near the node the approach is
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


@pytest.fixture(scope="module")
def net():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02346_amd import surrogate as S
    path = os.path.join(DATA, "lb_forces_seed2405_n4096.json")
    if not os.path.exists(path):
        pytest.skip("no LB force data")
    mlp, _, _ = S.fit([json.load(open(path))])
    yield mlp
    mlp.close()


@pytest.mark.parametrize("ratio,target", [(1.2, math.pi / 2), (0.85, 0.0)])
def test_drift_to_node_or_antinode(net, ratio, target):
    from paper_2404_02346_amd import motion as M
    F = M.extended(M.surrogate_force(net, 0.3, ratio, 8.0))
    kh0 = [0.15, 0.6, 1.0, 1.4, 2.2, 2.9]
    t, kh = M.integrate(F, kh0, gamma_over_k=1.0, t_end=60.0, dt=0.02)
    d = np.mod(kh[-1] - target, math.pi)
    d = np.minimum(d, math.pi - d)
    print(f"c_p/c0 = {ratio}: final distance to the {'node' if target else 'antinode'} {d.max():.2e}",
          flush=True)
    assert d.max() < 1e-3


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
