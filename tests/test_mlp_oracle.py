"""Pins of the FP64 network reference: gradients against central finite
differences, features against their closed form, bf16 rounding against the
definition of the format."""
import numpy as np

from oracle import mlp


def small_net(rng, dims=(6, 5, 4, 3)):
    W = [rng.normal(size=(dims[i + 1], dims[i])) * 0.7 for i in range(len(dims) - 1)]
    b = [rng.normal(size=dims[i + 1]) * 0.1 for i in range(len(dims) - 1)]
    return W, b


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(0)
    W, b = small_net(rng)
    x = rng.normal(size=(7, 6))
    t = rng.normal(size=(7, 3))
    w = np.array([1.0, 2.0, 0.5])

    def loss(W, b):
        y, _ = mlp.forward(W, b, x)
        return mlp.mse(y, t, w)[0]

    y, cache = mlp.forward(W, b, x)
    _, dout = mlp.mse(y, t, w)
    gW, gb = mlp.backward(W, cache, dout)
    h = 1e-6
    for i in range(len(W)):
        for (r, c) in [(0, 0), (W[i].shape[0] - 1, W[i].shape[1] - 1), (1, 2)]:
            Wp = [a.copy() for a in W]
            Wm = [a.copy() for a in W]
            Wp[i][r, c] += h
            Wm[i][r, c] -= h
            fd = (loss(Wp, b) - loss(Wm, b)) / (2 * h)
            assert abs(fd - gW[i][r, c]) < 1e-7 * max(1.0, abs(fd))
        bp = [a.copy() for a in b]
        bm = [a.copy() for a in b]
        bp[i][0] += h
        bm[i][0] -= h
        fd = (loss(W, bp) - loss(W, bm)) / (2 * h)
        assert abs(fd - gb[i][0]) < 1e-7 * max(1.0, abs(fd))


def test_features_closed_form():
    p = np.array([[0.25, 0.0, 0.0], [0.0, 0.5, 1.0]])
    B = np.array([[1.0, 0.0, 0.0], [0.0, 1.0, 0.5]])
    f = mlp.features(p, B)
    # <B_0, p_0> = 0.25 -> sin(pi/2) = 1, cos = 0; <B_1, p_1> = 1 -> sin 0, cos 1
    assert np.allclose(f[0], [1.0, 0.0, 0.0, 1.0], atol=1e-15)
    assert np.allclose(f[1], [0.0, 0.0, 1.0, 1.0], atol=1e-15)


def test_bf16_rounding():
    # exactly representable values stay; ties go to even; 8 significant bits
    assert mlp.bf16(np.array([1.0, -2.5, 3.0]))[1] == -2.5
    assert mlp.bf16(np.array([1.0 + 2 ** -8]))[0] == 1.0          # tie -> even (1.0)
    assert mlp.bf16(np.array([1.0 + 3 * 2 ** -8]))[0] == 1.0 + 2 ** -6  # tie -> even
    assert mlp.bf16(np.array([1.0 + 2 ** -7]))[0] == 1.0 + 2 ** -7
    x = np.random.default_rng(1).normal(size=1000)
    assert np.max(np.abs(mlp.bf16(x) - x) / np.abs(x)) <= 2 ** -8 + 1e-12   # half an ulp


def test_adam_first_step_by_hand():
    """w = 1, g = 0.5, zero moments, lr 0.1, wd 0.01: m = 0.05, v = 0.00025,
    the bias-corrected moments are 0.5 and 0.25, so the step is
    0.1 * (0.5 / (0.5 + 1e-8) + 0.01) and w becomes 0.89900000199999996."""
    w, m, v = mlp.adam(np.array([1.0]), np.array([0.5]), np.zeros(1), np.zeros(1), 1, 0.1,
                       wd=0.01)
    assert abs(m[0] - 0.05) < 1e-16 and abs(v[0] - 0.00025) < 1e-18  # 1 - 0.9 is inexact in FP64
    assert abs(w[0] - 0.89900000199999996) < 1e-15


def test_adam_constant_gradient_moves_lr_per_step():
    """With a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so (eps = 0, no decay) each step moves w by exactly lr against
    the sign of g, whatever the magnitude of g."""
    g = np.array([3.0, -1e-3, 250.0])
    w, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
    for t in range(1, 8):
        w, m, v = mlp.adam(w, g, m, v, t, 0.01, eps=0.0)
    assert np.allclose(w, -7 * 0.01 * np.sign(g), rtol=0, atol=1e-14)


def test_adam_without_moments_is_normalised_sgd():
    """b1 = b2 = 0: m = g, v = g^2, and the step is lr * g / (|g| + eps)."""
    rng = np.random.default_rng(2)
    g = rng.normal(size=5)
    w0 = rng.normal(size=5)
    w, _, _ = mlp.adam(w0, g, rng.normal(size=5), rng.random(5), 4, 0.3, b1=0.0, b2=0.0, eps=0.1)
    assert np.allclose(w, w0 - 0.3 * g / (np.abs(g) + 0.1), rtol=0, atol=1e-15)


def test_bf16_bars_cover_round_to_nearest():
    """The Monte Carlo arithmetic bars of tests/bf16_bounds.py, sized from the
    bfloat16 unit roundoff alone, cover the deterministic round-to-nearest
    model (quant=True: the same values rounded to bfloat16 instead of
    randomly perturbed), on a network of the warm start's shape
    (64 -> 4 x 256 -> 3)."""
    import math

    from tests import bf16_bounds as bb

    rng = np.random.default_rng(3)
    dims = [64, 256, 256, 256, 256, 3]
    W, b = [], []
    for i in range(5):
        lim = math.sqrt(6 / dims[i]) if i < 4 else math.sqrt(1 / dims[i])
        W.append(rng.uniform(-lim, lim, size=(dims[i + 1], dims[i])))
        b.append(rng.normal(size=dims[i + 1]) * 0.05)
    B = rng.normal(size=(32, 3)) * np.array([6.0, 6.0, 1.0])
    n = 300
    p = np.column_stack([rng.random(n), rng.random(n), rng.uniform(-1, 1, n)])
    t = rng.normal(size=(n, 3)) * 0.1
    w = np.array([2.0, 3.0, 1.0])
    x0 = mlp.features(p, B)
    R = bb.bars(W, b, x0, t, w)
    yq, cq = mlp.forward(W, b, x0, quant=True)
    Lq, dq = mlp.mse(yq, t, w)
    gWq, gbq = mlp.backward(W, cq, dq, quant=True)
    assert np.all(np.abs(yq - R["y"]) <= R["y_bar"])
    assert abs(Lq - R["loss"]) <= R["loss_bar"] * R["loss"]
    for i in range(5):
        assert np.linalg.norm(gWq[i] - R["gW"][i]) <= R["gW_bar"][i] * np.linalg.norm(R["gW"][i])
        assert np.linalg.norm(gbq[i] - R["gb"][i]) <= R["gb_bar"][i] * np.linalg.norm(R["gb"][i])
    # the bars are informative: a few bfloat16 roundoffs, not order one
    assert max(R["gW_bar"]) < 8 * U_BF16 and R["loss_bar"] < 4 * U_BF16


U_BF16 = 2.0 ** -8
