"""FP64 reference of the warm-start network (test infrastructure only).

Plain numpy: Fourier features, the forward pass (linear layers with SiLU
between them) and its backward pass written out by the chain rule, and the
weighted mean-squared error.  ``quant`` optionally rounds the operands of
every matrix product to bfloat16 and the stored activations, at the points
where the GPU kernels hold them in bfloat16, so that GPU and reference take
the same quantisation decisions.
"""
from __future__ import annotations

import numpy as np


def bf16(a: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) and return as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def features(p: np.ndarray, B: np.ndarray) -> np.ndarray:
    z = 2.0 * np.pi * (p @ B.T)
    return np.concatenate([np.sin(z), np.cos(z)], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(W, b, x, quant: bool = False):
    """Returns the output and the cache (inputs and pre-activations per layer)."""
    q = bf16 if quant else (lambda a: a)
    h = q(x)
    cache = []
    for i in range(len(W)):
        z = q(h) @ q(W[i]).T + b[i]
        cache.append((h, z))
        if i < len(W) - 1:
            h = q(silu(z))
        else:
            h = z
    return h, cache


def mse(y, t, w):
    r = y - t
    return float(np.sum(w[None, :] * r * r) / y.shape[0]), 2.0 * w[None, :] * r / y.shape[0]


def backward(W, cache, dout, quant: bool = False):
    """dL/dW and dL/db of every layer from dL/d(out)."""
    q = bf16 if quant else (lambda a: a)
    gW = [None] * len(W)
    gb = [None] * len(W)
    dz = dout
    for i in range(len(W) - 1, -1, -1):
        h, z = cache[i]
        gW[i] = q(dz).T @ q(h)
        gb[i] = dz.sum(axis=0)
        if i > 0:
            _, zprev = cache[i - 1]
            dz = (q(dz) @ q(W[i])) * dsilu(zprev)
    return gW, gb


def adam(w, g, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
         wd: float = 0.0):
    """One Adam step (Kingma & Ba, 2015) with decoupled weight decay
    (Loshchilov & Hutter, 2019) in FP64; returns the new (w, m, v).
    m and v are the biased first and second moment estimates, corrected by
    1 - b1^t and 1 - b2^t at step t (t counts from 1); the decay term wd * w
    uses the parameters before the step."""
    w, g, m, v = (np.asarray(a, dtype=np.float64) for a in (w, g, m, v))
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    w = w - lr * (mhat / (np.sqrt(vhat) + eps) + wd * w)
    return w, m, v
