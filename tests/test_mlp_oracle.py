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
