"""GPU tests of the surrogate network kernels against the FP64 oracle.

The GPU rounds weights, activations and back-propagated errors to BF16 and
accumulates in FP32 on MFMA; the oracle is FP64 with the same BF16-rounded
weights and inputs.  Bounds: relative 2-norm error 2e-2 for outputs and for
each layer's gradient (a few BF16 roundings, 2^-8 relative each, through five
layers).
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2404_02346_amd import surrogate as S
    return S


def say(*a):
    print(*a, flush=True)


def _bf16_bits(a):
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def test_mfma_tile_layout(S):
    rng = np.random.Generator(np.random.PCG64(5))
    A = M.bf16_round(rng.normal(size=(16, 32)))
    B = M.bf16_round(rng.normal(size=(32, 16)))
    D = S.mfma_probe(_bf16_bits(A), _bf16_bits(B))
    np.testing.assert_allclose(D, A @ B, rtol=1e-5, atol=1e-5)


def _layers(params):
    return M.unpack(params)


def test_forward_matches_oracle(S):
    p = S.init_params(11)
    rng = np.random.Generator(np.random.PCG64(12))
    x = rng.uniform(-1, 1, size=(300, 4)).astype(np.float32)
    net = S.MLP(max_batch=512, params=p)
    y = net.predict(x)
    ref, _ = M.forward(M.bf16_round(p), M.bf16_round(x))
    e = _rel(y, ref)
    say(f"forward rel err {e:.3e}")
    assert e < 2e-2
    net.close()


def test_gradients_match_oracle(S):
    p = S.init_params(13)
    rng = np.random.Generator(np.random.PCG64(14))
    x = rng.uniform(-1, 1, size=(257, 4)).astype(np.float32)
    t = np.sin(2 * x[:, 1]) * x[:, 2]
    net = S.MLP(max_batch=512, params=p)
    loss, g = net.grad(x, t)
    # biases enter in FP32 on the GPU: the oracle uses the BF16-rounded weights, FP32 biases
    pr = p.astype(np.float64).copy()
    off = 0
    for i in range(len(M.DIMS) - 1):
        n, k = M.DIMS[i + 1], M.DIMS[i]
        pr[off: off + n * k] = M.bf16_round(pr[off: off + n * k])
        off += n * k + n
    lref, gref = M.loss_and_grad(pr, M.bf16_round(x), t.astype(np.float32))
    say(f"loss gpu {loss:.6e} oracle {lref:.6e}")
    assert loss == pytest.approx(lref, rel=2e-2)
    off = 0
    for i in range(len(M.DIMS) - 1):
        n, k = M.DIMS[i + 1], M.DIMS[i]
        ew = _rel(g[off: off + n * k], gref[off: off + n * k])
        eb = _rel(g[off + n * k: off + n * k + n], gref[off + n * k: off + n * k + n])
        say(f"  layer {i}: dW rel {ew:.3e} db rel {eb:.3e}")
        assert ew < 2e-2 and eb < 2e-2
        off += n * k + n
    net.close()


def test_training_fits_a_smooth_target(S):
    rng = np.random.Generator(np.random.PCG64(21))
    kR = rng.uniform(0.05, 0.6, 1024)
    kh = rng.uniform(0, math.pi / 2, 1024)
    ratio = rng.uniform(0.8, 1.5, 1024)
    R = rng.uniform(4.0, 16.0, 1024)
    x = S.normalize(kR, kh, ratio, R)
    t = S.closed_form_ratio(kh, ratio) * (1 - 0.3 * kR ** 2) * (1 - 0.2 / R)
    net = S.MLP(max_batch=1024, seed=3)
    log = net.train(x, t, steps=4000, lr=3e-3, lr_final=1e-4, log_every=500)
    say("loss curve", log)
    assert log[-1][1] < 1e-3 * log[0][1]
    pred = net.predict(x)
    err = S.error_metric(pred, t)
    say("fit error", err)
    assert err["max"] < 0.05 and err["rms"] < 0.01
    net.close()


def test_batch_limits(S):
    import paper_2404_02346_amd as P
    net = S.MLP(max_batch=16)
    with pytest.raises(P.LBError):
        net.grad(np.zeros((17, 4)), np.zeros(17))
    # the layered forward splits into max_batch chunks; inference takes any batch
    assert len(net.predict(np.zeros((40, 4)), layered=True)) == 40
    assert len(net.predict(np.zeros((40, 4)))) == 40
    net.close()


@pytest.mark.parametrize("B", [1, 127, 300, 4096 + 77])
def test_fused_inference_matches_layered_forward(S, B):
    # One fused launch (activations in LDS) against one GEMM launch per layer:
    # the same MFMA sequence per output (sums start at the bias, K in the same
    # 32-wide steps) and the same roundings, so the outputs agree bit for bit
    # (1e-6 of their scale allows for a last-place difference).
    p = S.init_params(31)
    rng = np.random.Generator(np.random.PCG64(32))
    x = rng.uniform(-1, 1, size=(B, 4)).astype(np.float32)
    net = S.MLP(max_batch=8192, params=p)
    yf = net.predict(x)
    yl = net.predict(x, layered=True)
    scale = max(np.abs(yl).max(), 1e-3)
    e = np.abs(yf - yl).max() / scale
    say(f"B={B}: fused vs layered max diff / scale {e:.2e}")
    assert np.isfinite(yf).all() and e < 1e-6
    net.close()


def test_activation_matches_the_exact_gelu(S):
    # the device GELU against z Phi(z) with the exact erf, and its derivative against
    # Phi(z) + z phi(z): Hastings' erf form keeps Phi within 3e-7 in FP32
    z = np.concatenate([np.linspace(-14.0, 14.0, 400001), [0.0, -0.0, 1e-30, -1e-30, 40.0, -40.0]])
    z = z.astype(np.float32)
    z64 = z.astype(np.float64)
    phi = 0.5 * (1.0 + np.array([math.erf(v / math.sqrt(2.0)) for v in z64]))
    g = S.activation(z)
    gd = S.activation(z, derivative=True)
    eg = np.abs(g - z64 * phi)
    ed = np.abs(gd - (phi + z64 * np.exp(-0.5 * z64 * z64) / math.sqrt(2.0 * math.pi)))
    say(f"GELU max |error| / max(|z|, 1) {np.max(eg / np.maximum(np.abs(z64), 1.0)):.2e}, "
        f"derivative max |error| {ed.max():.2e}")
    assert np.all(eg <= 5e-7 * np.maximum(np.abs(z64), 1.0))
    assert np.all(ed <= 6e-7)
    assert g[-2] == 40.0 and g[-1] == 0.0 and gd[-2] == 1.0 and gd[-1] == 0.0
