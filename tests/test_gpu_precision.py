"""GPU force accuracy per storage precision against the FP64 oracle.

FP64 storage is the oracle's arithmetic (parity tests bound it at 1e-10 and
below).  FP32 storage must stay within 1% of the FP64 oracle on the 3D
sphere workload (the target); FP16 and BF16 store each population in 16
bits (FP32 collision, FP64 measurement).  Measured largest errors, and the
bound each test sets (the kernels are deterministic: the same inputs give the
same bits on every run, so a bound a few times the measurement is safe):

  workload (error measure)                 FP32           FP16           BF16
  full-size sphere, 16 positions:
    |dF| / max_j |F_j|                     1.3e-7 (1e-6)  2.4e-4 (1e-3)  1.4e-2 (3e-2)
    |dF| / |F|, |F| >= max / 5             1.5e-7 (1e-6)  5.5e-4 (2e-3)  3.4e-2 (5e-2)
  3D sphere 64x32x32, 3 positions, rel     2.2e-7 (1e-6)  6.8e-4 (3e-3)  1.3e-2 (5e-2)
  2D cylinder, rel                         1.2e-7 (1e-6)  1.8e-4 (1e-3)  2.2e-3 (1e-2)
  seed-2404 batch, edges 64-192, rel       3.6e-5 (2e-4)

BF16 misses the 2% target at three full-size positions: 3.4% at kh_2, 2.1%
at kh_3 and kh_14 (relative to the force there).  Its force comes out too
small at 15 of the 16 positions (0.1-1.4% of the largest force), unevenly
from one position to the next: a systematic loss, not noise.  FP16 stays
within 0.06% everywhere.  The time-averaged force is a
second-order, time-averaged quantity: the rounding noise of the stored
populations largely averages out over the window.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden", "sphere3d_oracle_forces.json")

BOUND = {
    # full-size sphere: |dF| / max_j |F_j| at every position, |dF| / |F| where |F| >= max / 5
    "full_scale": {"f32": 1e-6, "f16": 1e-3, "bf16": 3e-2},
    "full_rel": {"f32": 1e-6, "f16": 2e-3, "bf16": 5e-2},
    "reduced": {"f32": 1e-6, "f16": 3e-3, "bf16": 5e-2},
    "cylinder": {"f64": 1e-12, "f32": 1e-6, "f16": 1e-3, "bf16": 1e-2},
    "batch": {"f32": 2e-4},
}


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_02346_amd as P
    return P


def say(*a):
    print(*a, flush=True)


def run(P, p, storage, spl=1):
    h = P.LBWave([p], storage=storage)
    h.set_steps_per_launch(spl)
    h.step(p["n_steps"])
    F, nacc = h.force()
    h.close()
    assert nacc[0] == p["n_steps"] - p["avg_start"]
    return F[0]


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_sixteen_positions_against_oracle_goldens(P, storage):
    # The 3D workload at full size (256 x 128 x 128, 15360 steps), all 16 positions kh_j in one
    # handle with two steps per launch and graph replay (the benchmark's configuration), against
    # the FP64 oracle's forces written by tests/golden/make_sphere_goldens.py.  Per position:
    # |dF_x| / max_j |F_x| (bounded everywhere) and |dF_x| / |F_x| (bounded where |F_x| is at
    # least a fifth of the largest: near kh = 0 and pi/2 the force crosses zero).
    if not os.path.exists(GOLD):
        pytest.skip("no oracle goldens")
    g = json.load(open(GOLD))
    khs = workloads.sphere_3d_positions(16)
    probs = [workloads.sphere_3d(g["x_mid"], g["k"], kh) for kh in khs]
    h = P.LBWave(probs, storage=storage)
    h.set_steps_per_launch(2)
    h.set_graph(64)
    h.step(probs[0]["n_steps"])
    F, nacc = h.force()
    h.close()
    assert np.all(nacc == probs[0]["n_steps"] - probs[0]["avg_start"])
    gold = {int(j): rec for j, rec in g["positions"].items()}
    scale = max(abs(rec["F_avg"][0]) for rec in gold.values())
    for j in sorted(gold):
        rec = gold[j]
        np.testing.assert_allclose(probs[j]["center"], rec["center"], atol=1e-12)
        ref = rec["F_avg"][0]
        d = abs(F[j, 0] - ref)
        say(f"kh_{j} {storage}: F_x {F[j, 0]:.8e} oracle {ref:.8e} "
            f"|dF|/max|F| {d / scale:.2e} rel {d / abs(ref):.2e}")
        assert d / scale <= BOUND["full_scale"][storage]
        if abs(ref) >= 0.2 * scale:
            assert d / abs(ref) <= BOUND["full_rel"][storage]
    if storage == "f32":
        # the shape the paper reports: sin 2kh, largest near kh = pi/4, zero at the node
        fx = F[:, 0]
        say("F_x by position", np.array2string(fx, precision=4))
        assert np.argmax(fx) in (6, 7, 8)
        assert abs(fx[15]) < 0.05 * fx.max()
        assert np.all(fx[1:15] > 0)


@pytest.mark.parametrize("storage", ["f32", "f16", "bf16"])
def test_reduced_sphere_against_oracle(P, orc, storage):
    cal = orc.cavity_calibration(64, 0.5, 2 * np.pi * 0.5 / 64)
    for kh in (math.pi / 8, math.pi / 4, 3 * math.pi / 8):
        p = workloads.sphere_3d(cal["x_mid"], cal["k"], kh, n_periods=12, avg_periods=5,
                                shape=(64, 32, 32), lam=64.0, R=3.0, n_surf=512)
        ref = orc.run(p, p["n_steps"])["F_avg"][0]
        F = run(P, p, storage)
        e = abs(F[0] - ref) / abs(ref)
        say(f"reduced kh={kh:.3f} {storage}: rel {e:.2e}")
        assert e <= BOUND["reduced"][storage]


def test_cylinder_all_storages(P, orc):
    cal = orc.cavity_calibration(128, 0.5, 2 * np.pi * 0.5 / 128)
    p = workloads.cylinder_2d(cal["x_mid"], cal["k"])
    ref = orc.run(p, p["n_steps"])["F_avg"][0]
    for storage in ("f64", "f32", "f16", "bf16"):
        F = run(P, p, storage)
        e = abs(F[0] - ref) / abs(ref)
        say(f"cylinder {storage}: rel {e:.2e}")
        assert e <= BOUND["cylinder"][storage]


def test_batch_instances_against_oracle_goldens(P):
    # Instances of the seeded uneven batch (seed 2404) run together in one
    # handle, each to its own length, against the FP64 oracle's forces
    # written by tests/golden/make_batch_goldens.py.
    path = os.path.join(HERE, "golden", "batch2404_oracle_forces.json")
    if not os.path.exists(path):
        pytest.skip("no oracle goldens")
    g = json.load(open(path))
    c0 = workloads.BATCH_C0
    probs, refs = [], []
    for i, rec in sorted(g["instances"].items()):
        e = int(rec["edge"])
        p = workloads._problem(3, e, e, e, c0, rec["cp_ratio"] * c0, rec["radius"],
                               rec["center"], float(e), 30, 10, 2048, kh=rec["kh"])
        assert p["n_steps"] == rec["n_steps"] and p["avg_start"] == rec["avg_start"]
        probs.append(p)
        refs.append(rec["F_avg"])
    # two steps per launch, so that rows of 96 and 192 cells (two and three wavefronts per row
    # in the two-step kernel) meet the oracle directly
    h = P.LBWave(probs, storage="f32", freeze_at_n_steps=True)
    h.set_steps_per_launch(2)
    h.set_graph(64)
    h.step(max(p["n_steps"] for p in probs))
    F, nacc = h.force()
    h.close()
    for p, Fi, ref, n in zip(probs, F, refs, nacc):
        e = abs(Fi[0] - ref[0]) / abs(ref[0])
        say(f"edge {p['nx']}: F_x {Fi[0]:.8e} oracle {ref[0]:.8e} rel {e:.2e}")
        assert n == p["n_steps"] - p["avg_start"]
        assert e <= BOUND["batch"]["f32"]
