"""FP64 CPU reference of the force surrogate network (test infrastructure).

TEST INFRASTRUCTURE ONLY (part of the oracle package; shares no code with
the GPU library).  Plain numpy, float64 throughout.

Network: 4 -> 256 -> 256 -> 256 -> 256 -> 1, exact GELU
g(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2 after each hidden layer, linear
output.  Parameters are one flat vector, layer by layer: W_l (out x in,
row-major) then b_l.  Loss: mean squared error L = (1/B) sum (y - t)^2.
Gradients by reverse-mode differentiation written out layer by layer.

Pinned by finite differences and by PyTorch's autograd in
tests/test_oracle_mlp.py.
"""
from __future__ import annotations

import math

import numpy as np

DIMS = (4, 256, 256, 256, 256, 1)


def num_params(dims=DIMS) -> int:
    return sum(dims[i + 1] * dims[i] + dims[i + 1] for i in range(len(dims) - 1))


def unpack(params, dims=DIMS):
    """Split the flat parameter vector into [(W_l, b_l)]."""
    params = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for i in range(len(dims) - 1):
        n, k = dims[i + 1], dims[i]
        W = params[off: off + n * k].reshape(n, k)
        off += n * k
        b = params[off: off + n]
        off += n
        out.append((W, b))
    assert off == params.size
    return out


_erf = np.vectorize(math.erf, otypes=[np.float64])


def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_prime(z):
    z = np.asarray(z, dtype=np.float64)
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def forward(params, x, dims=DIMS):
    """y (B,) and the per-layer cache (inputs a_l, pre-activations z_l)."""
    layers = unpack(params, dims)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for i, (W, b) in enumerate(layers):
        z = a @ W.T + b
        cache.append((a, z))
        a = gelu(z) if i < len(layers) - 1 else z
    return a[:, 0], cache


def loss_and_grad(params, x, t, dims=DIMS):
    """Mean squared error and its gradient (same flat layout as params)."""
    layers = unpack(params, dims)
    y, cache = forward(params, x, dims)
    t = np.asarray(t, dtype=np.float64)
    B = y.size
    loss = float(np.mean((y - t) ** 2))
    delta = (2.0 * (y - t) / B)[:, None]  # dL/dz of the output layer
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        a, z = cache[i]
        W, _ = layers[i]
        grads[i] = (delta.T @ a, delta.sum(axis=0))
        if i > 0:
            delta = (delta @ W) * gelu_prime(cache[i - 1][1])
    flat = np.concatenate([np.concatenate([gw.reshape(-1), gb]) for gw, gb in grads])
    return loss, flat


def bf16_round(a) -> np.ndarray:
    """Round float64 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
