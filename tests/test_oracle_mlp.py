"""Pins of the FP64 surrogate-network oracle: finite differences, autograd, GELU."""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as M

SMALL = (3, 7, 5, 1)


def _params(seed, dims):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.normal(0, 0.5, size=M.num_params(dims))


def test_num_params():
    assert M.num_params() == 198913


def test_gelu_values():
    # exact GELU z Phi(z): g(0) = 0, g'(0) = 1/2, g(z) -> z and g'(z) -> 1 for large z,
    # g(-z) = g(z) - z (Phi(z) + Phi(-z) = 1)
    assert M.gelu(0.0) == 0.0 and M.gelu_prime(0.0) == pytest.approx(0.5)
    assert M.gelu(9.0) == pytest.approx(9.0, rel=1e-15)
    assert M.gelu_prime(9.0) == pytest.approx(1.0, rel=1e-15)
    z = np.linspace(-4, 4, 17)
    np.testing.assert_allclose(M.gelu(-z), M.gelu(z) - z, atol=1e-15)
    assert M.gelu(1.0) == pytest.approx(0.5 * (1 + math.erf(1 / math.sqrt(2))), rel=1e-15)
    e = 1e-6
    np.testing.assert_allclose(M.gelu_prime(z), (M.gelu(z + e) - M.gelu(z - e)) / (2 * e),
                               rtol=1e-8, atol=1e-9)


def test_gradient_by_finite_differences():
    p = _params(1, SMALL)
    rng = np.random.Generator(np.random.PCG64(2))
    x = rng.uniform(-1, 1, size=(9, 3))
    t = rng.normal(size=9)
    loss, g = M.loss_and_grad(p, x, t, SMALL)
    e = 1e-6
    for i in range(p.size):
        q = p.copy()
        q[i] += e
        lp, _ = M.loss_and_grad(q, x, t, SMALL)
        q[i] -= 2 * e
        lm, _ = M.loss_and_grad(q, x, t, SMALL)
        assert g[i] == pytest.approx((lp - lm) / (2 * e), rel=1e-6, abs=1e-9), i


def test_gradient_against_autograd():
    torch = pytest.importorskip("torch")
    p = _params(3, M.DIMS) * 0.1
    rng = np.random.Generator(np.random.PCG64(4))
    x = rng.uniform(-1, 1, size=(33, M.DIMS[0]))
    t = rng.normal(size=33)
    loss, g = M.loss_and_grad(p, x, t)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    a = torch.tensor(x, dtype=torch.float64)
    off = 0
    dims = M.DIMS
    for i in range(len(dims) - 1):
        n, k = dims[i + 1], dims[i]
        W = pt[off: off + n * k].reshape(n, k)
        off += n * k
        b = pt[off: off + n]
        off += n
        a = a @ W.T + b
        if i < len(dims) - 2:
            a = torch.nn.functional.gelu(a)  # exact (erf) form
    lt = ((a[:, 0] - torch.tensor(t)) ** 2).mean()
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-13)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-10, atol=1e-14)


def test_bf16_round():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -2.5, 3.140625, 1e-3])
    r = M.bf16_round(v)
    assert r[0] == 1.0 and r[3] == -2.5 and r[4] == 3.140625
    assert r[1] == 1.0 + 2 ** -7 or r[1] == 1.0  # exact tie: to even
    assert r[1] == 1.0
    assert r[2] == 1.0 + 2 ** -7
    assert abs(r[5] - 1e-3) / 1e-3 < 2 ** -8
