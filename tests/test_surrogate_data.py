"""Host checks of the surrogate's LB force data and its generators (no GPU).

The network is trained on forces from two seeded generators (Sec. Results and discussion sets the
channel width L_y = L_z = 64): cubic boxes of edge 64 .. 192 (workloads.batch) and, for the small
k R the cubic boxes cannot reach, channel boxes lambda x 64 x 64 (workloads.channel_draws).  The
stored data sets must be the generators' own draws, and together they must cover the input box on
which the network is trusted.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads
from paper_2404_02346_amd import surrogate as S

KR_SPLIT = 2 * math.pi * 4 / 192   # smallest k R of the cubic boxes (R >= 4, edge <= 192)


def test_channel_draws_ranges_and_rounding():
    d1, rej1 = workloads.channel_draws(11, 300)
    d2, rej2 = workloads.channel_draws(11, 300)
    assert d1 == d2 and rej1 == rej2          # seeded
    for lam, R, ratio, kh in d1:
        assert lam % 8 == 0
        kr = 2 * math.pi * R / lam
        assert 0.05 <= kr < KR_SPLIT
        assert 4.0 <= R <= 16.0 and 0.8 <= ratio <= 1.5 and 0.0 <= kh <= math.pi / 2
    krs = np.array([2 * math.pi * R / lam for lam, R, _, _ in d1])
    assert krs.min() < 0.06 and krs.max() > 0.12   # the whole range is drawn


def test_channel_object_fits_the_channel():
    # the object with its integration surface and the 3-point stencil fits across 64 cells, and
    # stays off the x sheets wherever kh puts it between the central antinode and the node (the
    # calibrated antinode of a driven box of length lambda lies within 2 cells below lambda / 2)
    for lam, R, ratio, kh in workloads.channel_draws(12, 200)[0]:
        reach = R + workloads.SURFACE_OFFSET + workloads.KERNEL_REACH
        assert 2 * reach < workloads.CHANNEL_WIDTH
        x_lo, x_hi = lam / 2 - 2 - reach, lam / 2 + lam / 4 + reach
        assert x_lo >= 2 and x_hi <= lam - 3


@pytest.mark.parametrize("name,seed,n", [("lb_forces_channel_seed2408_n704.json", 2408, 704),
                                         ("lb_forces_channel_seed2409_n88.json", 2409, 88)])
def test_stored_channel_data_are_the_generators_draws(name, seed, n):
    path = os.path.join(S.DATA_DIR, name)
    d = json.load(open(path))
    assert d["generator"] == "channel" and d["seed"] == seed and d["n"] == n == len(d["rows"])
    draws, rejected = workloads.channel_draws(seed, n)
    assert rejected == d["rejected_draws"]
    for row, (lam, R, ratio, kh) in zip(d["rows"], draws):
        assert (row["edge"], row["R"], row["ratio"], row["kh"]) == (lam, R, ratio, kh)
        assert row["kR"] == pytest.approx(2 * math.pi * R / lam, rel=1e-12)
        assert np.all(np.isfinite(row["F"]))


def test_data_cover_the_trusted_box():
    assert S.TRUST == S.BOX
    tr = S.table(*S.load_sets(S.TRAIN_FILES))
    te = S.table(*S.load_sets(S.TEST_FILES))
    assert len(tr[0]) == 4800 and len(te[0]) == 600
    for kR, kh, ratio, R, _ in (tr, te):
        assert S.in_box(kR, kh, ratio, R).all()
        assert kR.min() < 0.06 and kR.max() > 0.59       # k R from 0.05 to 0.6
        assert np.sum(kR < KR_SPLIT) > 0.1 * len(kR)     # the channel boxes' share
    # the held-out sets are not training samples
    key = lambda t: set(zip(np.round(t[0], 12), np.round(t[1], 12), np.round(t[2], 12)))
    assert not key(tr) & key(te)
