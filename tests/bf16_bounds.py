"""Rounding-error bars of the warm-start network evaluated with bfloat16
operands and FP32 accumulation, against the same network in exact arithmetic
(the FP64 reference of oracle/mlp.py with quant=False).

The bars come from Monte Carlo arithmetic (D. S. Parker, "Monte Carlo
arithmetic: exploiting randomness in floating-point arithmetic", 1997): every
value that the kernels hold in bfloat16 -- the Fourier features, the hidden
activations, the bfloat16 copies of the weights, the loss gradient and the
back-propagated gradients -- is replaced by value * (1 + d) with d uniform in
[-u, u], u = 2^-8 (the unit roundoff of bfloat16's 8-bit significand:
round-to-nearest moves a value by at most u of its magnitude).  The FP32
accumulation of the products (K 2^-24 per sum, K <= 300) is two orders of
magnitude below u and is left out.  The network is evaluated in FP64 with
these perturbations for a number of independent draws; the spread of the
results over the draws sizes the bars:
  * outputs: elementwise, LAMBDA standard deviations of the draws;
  * loss, weight and bias gradients: relative (Frobenius) error, SAFETY times
    the largest relative error met over the draws.
Round-to-nearest is one realisation of such perturbations (its errors are
bounded by u and, for data like these, centred), so the kernels' results
should fall inside the bars; the CPU test of this module checks that the
deterministic round-to-nearest model of oracle/mlp.py (quant=True) does.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp

U = 2.0 ** -8      # bfloat16 unit roundoff
LAMBDA = 6.0       # standard deviations of the elementwise output bar
SAFETY = 2.0       # factor on the largest relative gradient / loss error of the draws
DRAWS = 32


def _pert(a, rng):
    return a * (1.0 + rng.uniform(-U, U, size=np.shape(a)))


def perturbed_pass(W, b, x0, t, wvec, rng):
    """Forward, loss and backward of the network with every bfloat16-held
    value perturbed by a random relative amount of at most u.
    Returns (y, loss, gW, gb)."""
    L = len(W)
    Wq = [_pert(Wi, rng) for Wi in W]
    h = _pert(x0, rng)
    hs, zs = [], []
    for i in range(L):
        z = h @ Wq[i].T + b[i]
        hs.append(h)
        zs.append(z)
        if i < L - 1:
            h = _pert(mlp.silu(z), rng)
    y = zs[-1]
    loss, dout = mlp.mse(y, t, wvec)
    dzf, dzb = dout, _pert(dout, rng)
    gW, gb = [None] * L, [None] * L
    for i in range(L - 1, -1, -1):
        gW[i] = dzb.T @ hs[i]
        gb[i] = dzf.sum(axis=0)
        if i > 0:
            dzf = (dzb @ Wq[i]) * mlp.dsilu(zs[i - 1])
            dzb = _pert(dzf, rng)
    return y, loss, gW, gb


def bars(W, b, x0, t, wvec, seed: int = 0, draws: int = DRAWS):
    """Reference (exact) results and their bars.  Returns a dict with the
    exact y, loss, gW, gb and the bars: y_bar (elementwise), loss_bar
    (relative), gW_bar / gb_bar (relative Frobenius, per layer)."""
    y, cache = mlp.forward(W, b, x0)
    loss, dout = mlp.mse(y, t, wvec)
    gW, gb = mlp.backward(W, cache, dout)
    rng = np.random.default_rng(seed)
    ys, el, egW, egb = [], [], [], []
    for _ in range(draws):
        yp, lp, gWp, gbp = perturbed_pass(W, b, x0, t, wvec, rng)
        ys.append(yp)
        el.append(abs(lp - loss) / abs(loss))
        egW.append([np.linalg.norm(a - r) / np.linalg.norm(r) for a, r in zip(gWp, gW)])
        egb.append([np.linalg.norm(a - r) / np.linalg.norm(r) for a, r in zip(gbp, gb)])
    ys = np.array(ys)
    return {
        "y": y, "loss": loss, "gW": gW, "gb": gb,
        "y_bar": LAMBDA * ys.std(axis=0) + 1e-7 * np.abs(y),
        "loss_bar": SAFETY * max(el),
        "gW_bar": SAFETY * np.max(np.array(egW), axis=0),
        "gb_bar": SAFETY * np.max(np.array(egb), axis=0),
        "y_rel_rms": float(np.sqrt(np.mean((ys - y) ** 2)) / np.sqrt(np.mean(y ** 2))),
    }
