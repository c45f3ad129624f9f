"""Four-layer MLP of the learned far-field form, FP64 forward and analytic backward
(oracle; test infrastructure only).

Layers 8 -> 128 -> 128 -> 128 -> 12 with SiLU activations (silu(z) = z / (1 + e^-z)),
mean-squared-error loss.  Parameters are one flat array, layer by layer: W_l [out][in]
row-major, then b_l [out].  The same layout is used by the HIP kernels.
"""
from __future__ import annotations

import numpy as np

SIZES = (8, 128, 128, 128, 12)


def n_params(sizes=SIZES) -> int:
    return sum(o * i + o for i, o in zip(sizes[:-1], sizes[1:]))


def unpack(params: np.ndarray, sizes=SIZES):
    out, off = [], 0
    for i, o in zip(sizes[:-1], sizes[1:]):
        w = params[off:off + o * i].reshape(o, i)
        off += o * i
        b = params[off:off + o]
        off += o
        out.append((w, b))
    return out


def init_params(rng: np.random.Generator, sizes=SIZES) -> np.ndarray:
    parts = []
    for i, o in zip(sizes[:-1], sizes[1:]):
        parts.append(rng.normal(0.0, 1.0 / np.sqrt(i), size=(o, i)).ravel())
        parts.append(np.zeros(o))
    return np.concatenate(parts)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward(params: np.ndarray, x: np.ndarray, sizes=SIZES):
    """x [n, 8] -> y [n, 12]; returns (y, cache of pre-activations and inputs)."""
    layers = unpack(params, sizes)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for li, (w, b) in enumerate(layers):
        z = a @ w.T + b
        cache.append((a, z))
        a = z if li == len(layers) - 1 else z * _sig(z)
    return a, cache


def loss(params, x, t, weight=None, sizes=SIZES) -> float:
    y, _ = forward(params, x, sizes)
    d = y - t
    if weight is not None:
        d = d * weight[:, None]
    return float(np.mean(np.sum(d * d, axis=1)))


def loss_grad(params, x, t, weight=None, sizes=SIZES):
    """Mean over samples of sum over outputs of (w (y - t))^2, and its gradient."""
    y, cache = forward(params, x, sizes)
    n = x.shape[0]
    d = y - t
    wv = np.ones(n) if weight is None else weight
    g = 2.0 * d * (wv * wv)[:, None] / n
    layers = unpack(params, sizes)
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        w, b = layers[li]
        a_in, z = cache[li]
        if li != len(layers) - 1:
            s = _sig(z)
            g = g * (s * (1.0 + z * (1.0 - s)))
        grads.append((g.T @ a_in, g.sum(axis=0)))
        g = g @ w
    grads.reverse()
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    return float(np.mean(np.sum((d * wv[:, None]) ** 2, axis=1))), flat
