"""GPU: two lattice steps per launch (step2_kernel) against one step per launch.

The fused kernel must give the same bits as two one-step launches: state,
per-step force trace and time average, for every storage, for rows of one
to four wavefronts (nx = 64, 70, 150, 256), rows longer than 256 cells cut
into strips of 254 cells (nx = 257, 300, 378, 520, 1016: two to four strips,
the last one partial or full), the object's surface across a strip boundary,
z extents that end in a partial
plane chunk, several uneven instances in one handle, odd step counts (the
last step then runs alone), graph replay and instances that stop inside the
run.  FP64 cases are also compared with the oracle directly.
"""
import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

# (z, y, x) shapes: nx -> pitch 64/128/192/256 -> 1/2/3/4 wavefronts per row
SHAPES = [(12, 16, 64), (40, 16, 70), (10, 12, 150), (9, 12, 256)]
# rows longer than 256 cells: strips of 254 owned cells, with the object across a strip boundary
# (x = 254 or 508) in the last three
STRIP_SHAPES = [((8, 16, 257), None), ((6, 16, 300), None), ((5, 16, 520), 253.6),
                ((8, 16, 378), 254.3), ((8, 16, 1016), 508.4)]


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2404_02346_amd as P
    P.lib()
    return P


def say(*a):
    print(*a, flush=True)


def problem(shape, R=2.0, avg_start=3, max_steps=0, seed=0, cx=None):
    nz, ny, nx = shape
    c0 = 0.45
    center = (nx * 0.55 if cx is None else cx, ny / 2.0 + 0.3, nz / 2.0 - 0.2)
    xyz, nrm, area = workloads.fibonacci_surface(center, R + 2.0, 96)
    return {"dim": 3, "nx": nx, "ny": ny, "nz": nz, "xbc": "driven", "c0": c0, "rho0": 1.0,
            "center": center, "radius": R, "cp": 0.55, "d": 4.0, "rho_a": 1.0,
            "omega": 2 * np.pi * c0 / nx, "wall_phi": 0.99, "surf_xyz": xyz,
            "surf_normal": nrm, "surf_area": area, "avg_start": avg_start,
            "max_steps": max_steps}


def run(P, probs, storage, spl, n_steps, graph=0, chunks=None, trace=60):
    h = P.LBWave(probs, storage=storage, trace_steps=trace)
    h.set_steps_per_launch(spl)
    h.set_graph(graph)
    for i, p in enumerate(probs):
        h.set_state(i, workloads.random_state(70 + i, p["nx"] * p["ny"] * p["nz"], 7))
    for n in (chunks or [n_steps]):
        h.step(n)
    st = [h.get_state(i) for i in range(len(probs))]
    tr = [h.trace(i, trace) for i in range(len(probs))]
    F, nacc = h.force()
    h.close()
    return st, tr, F, nacc


def same(a, b):
    for x, y in zip(a[0], b[0]):
        assert np.array_equal(x, y)
    for x, y in zip(a[1], b[1]):
        assert np.array_equal(x, y)
    assert np.array_equal(a[2], b[2]) and np.array_equal(a[3], b[3])


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
def test_two_step_is_bitwise_one_step_batched(P, storage):
    probs = [problem(s) for s in SHAPES]
    say(f"two-step vs one-step, {storage}, shapes {SHAPES}")
    one = run(P, probs, storage, 1, 37)
    two = run(P, probs, storage, 2, 37)
    same(one, two)


@pytest.mark.parametrize("storage", ["f32", "f64", "f16", "bf16"])
def test_two_step_strips_are_bitwise_one_step(P, storage):
    probs = [problem(shape, cx=cx) for shape, cx in STRIP_SHAPES]
    say(f"two-step strips vs one-step, {storage}, shapes {[s for s, _ in STRIP_SHAPES]}")
    same(run(P, probs, storage, 1, 37), run(P, probs, storage, 2, 37))


@pytest.mark.parametrize("shape", SHAPES)
def test_two_step_single_instances(P, shape):
    p = problem(shape)
    say(f"two-step single instance {shape}")
    same(run(P, [p], "f32", 1, 24), run(P, [p], "f32", 2, 24))


def test_two_step_graph_replay_and_stopping_instances(P):
    # instances stop at odd and even steps inside graph chunks; pieces of odd length
    probs = [problem((8, 16, 70), max_steps=0), problem((6, 16, 64), max_steps=29),
             problem((8, 16, 70), max_steps=51), problem((6, 16, 64), max_steps=12)]
    say("two-step graph replay with stopping instances")
    ref = run(P, probs, "f32", 1, 0, graph=0, chunks=[37, 3, 40], trace=80)
    for graph in (0, 8, 64):
        same(ref, run(P, probs, "f32", 2, 0, graph=graph, chunks=[37, 3, 40], trace=80))


def test_two_step_longest_chunks_with_a_partial_chunk(P):
    # 16 boxes of 96 x 128 x 256 give 1024 blocks with the longest FP32 plane chunk (64 planes), so
    # the chunk is kept and the last one of every box is a partial chunk of 32 planes: the launch
    # shape of the 16-sphere workload, plus a ragged end in z.  Two boxes start from seeded random
    # states, the others from rest; 7 steps (the last one runs alone).
    shape = (96, 128, 256)
    probs = [problem(shape, R=6.0) for _ in range(16)]
    ncell = shape[0] * shape[1] * shape[2]
    seeded = {0: 91, 9: 92}
    say("two-step, 16 boxes of 96 x 128 x 256, 64-plane chunks with a partial last chunk")
    out = []
    for spl in (1, 2):
        h = P.LBWave(probs, storage="f32", trace_steps=8)
        h.set_steps_per_launch(spl)
        for i, seed in seeded.items():
            h.set_state(i, workloads.random_state(seed, ncell, 7, scale=0.05))
        h.step(7)
        out.append(([h.get_state(i) for i in (0, 3, 9)], [h.trace(i, 7) for i in range(16)]))
        h.close()
    for x, y in zip(out[0][0], out[1][0]):
        assert np.array_equal(x, y)
    assert np.any(out[0][0][0] != 0) and np.any(out[0][0][1] != 0)
    for x, y in zip(out[0][1], out[1][1]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("shape,cx", [((40, 16, 70), None), ((10, 16, 300), 254.2)])
def test_two_step_against_oracle_fp64(P, orc, shape, cx):
    p = problem(shape, avg_start=5, cx=cx)
    n = 30
    init = workloads.random_state(70, p["nx"] * p["ny"] * p["nz"], 7)
    h = P.LBWave([p], storage="f64", trace_steps=n)
    h.set_steps_per_launch(2)
    h.set_state(0, init)
    h.step(n)
    st, tr = h.get_state(0), h.trace(0, n)
    F, nacc = h.force()
    h.close()
    ref = orc.run(p, n, fnew_init=init, want_fields=True, want_trace=True)
    ef = np.abs(st - ref["fnew"]).max() / np.abs(ref["fnew"]).max()
    et = np.abs(tr - ref["F_trace"]).max() / np.abs(ref["F_trace"]).max()
    say(f"two-step FP64 vs oracle {shape}: field {ef:.2e} trace {et:.2e}")
    assert ef <= 1e-12 and et <= 1e-11
    assert nacc[0] == ref["n_acc"]


def test_two_step_rejected_where_it_does_not_apply(P):
    cases = [problem((6, 10, 70)),            # ny not a multiple of the row block
             problem((6, 10, 300))]           # the same with rows cut into strips
    p2 = dict(problem((6, 16, 64)))
    p2["xbc"] = "periodic"
    for key in ("surf_xyz", "surf_normal", "surf_area"):
        p2.pop(key)
    cases.append(p2)
    for p in cases:
        h = P.LBWave([p], storage="f32")
        with pytest.raises(P.LBError):
            h.set_steps_per_launch(2)
        assert h.steps_per_launch() == 1
        h.close()
    cyl = workloads.cylinder_2d(62.63, 2 * np.pi / 128)
    h = P.LBWave([cyl], storage="f64")
    with pytest.raises(P.LBError):
        h.set_steps_per_launch(2)
    h.close()

