"""Seeded synthetic inputs shared by the oracle and the GPU tests.

Holds none of the method's arithmetic: only random smooth fields and
population arrays built from a caller-supplied base vector.
"""
from __future__ import annotations

import numpy as np


def smooth_field(shape, rng: np.random.Generator, nmodes: int = 4) -> np.ndarray:
    """Sum of ``nmodes`` separable low Fourier modes with random
    coefficients, scaled to max |value| = 1."""
    axes = [np.linspace(0.0, 1.0, s) for s in shape]
    out = np.zeros(shape)
    for _ in range(nmodes):
        term = np.array(rng.normal())
        for d, g in enumerate(axes):
            k = rng.integers(1, 4)
            f = np.cos(np.pi * k * g + rng.uniform(0, 2 * np.pi))
            term = term[..., None] * f if term.ndim else term * f
        out += term
    m = np.abs(out).max()
    return out / m if m > 0 else out


def random_populations(shape, base, amp: float, seed: int, noise: float = 1e-3) -> np.ndarray:
    """[q, *shape] float64: base_i * (1 + amp * smooth_i + noise * white_i)."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64)
    out = np.empty((len(base),) + tuple(shape))
    for i, b in enumerate(base):
        out[i] = b * (1.0 + amp * smooth_field(shape, rng) + noise * rng.normal(size=shape))
    return out


def random_scalar_populations(shape, q: int, scale: float, seed: int,
                              noise: float = 1e-3) -> np.ndarray:
    """[q, *shape] float64 with values scale/q * (smooth in [-1,1] + noise)."""
    rng = np.random.default_rng(seed)
    out = np.empty((q,) + tuple(shape))
    for i in range(q):
        out[i] = scale / q * (smooth_field(shape, rng) + noise * rng.normal(size=shape))
    return out


def _separable(shape, rng: np.random.Generator, jitter: float) -> np.ndarray:
    """One separable low Fourier mode plus ``jitter`` times a separable
    product of per-axis uniform random vectors (node-to-node variation),
    built by outer products only; max |value| <= 1 + jitter."""
    smooth = None
    rough = None
    for s in shape:
        g = np.linspace(0.0, 1.0, s)
        c = np.cos(np.pi * rng.integers(1, 4) * g + rng.uniform(0, 2 * np.pi))
        r = rng.uniform(-1.0, 1.0, s)
        smooth = c if smooth is None else smooth[..., None] * c
        rough = r if rough is None else rough[..., None] * r
    return smooth + jitter * rough


def separable_populations(shape, base, amp: float, seed: int, jitter: float = 0.2) -> np.ndarray:
    """[q, *shape] float64: base_i * (1 + amp * field_i) with a separable
    field per population (cheap enough for meshes of 10^8 nodes)."""
    rng = np.random.default_rng(seed)
    base = np.asarray(base, dtype=np.float64)
    out = np.empty((len(base),) + tuple(shape))
    for i, b in enumerate(base):
        out[i] = _separable(shape, rng, jitter)
        out[i] *= amp * b
        out[i] += b
    return out


def separable_scalar_populations(shape, q: int, scale: float, seed: int,
                                 jitter: float = 0.2) -> np.ndarray:
    """[q, *shape] float64 with values scale/q * field_i (separable fields)."""
    rng = np.random.default_rng(seed)
    out = np.empty((q,) + tuple(shape))
    for i in range(q):
        out[i] = _separable(shape, rng, jitter)
        out[i] *= scale / q
    return out
