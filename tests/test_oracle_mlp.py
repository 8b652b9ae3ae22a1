"""Pins of the emulator-network oracle (oracle/mlp.py): BF16 rounding, the
chain rule against finite differences, Adam against its closed form."""
import numpy as np

from oracle import mlp as O


def test_bf16_round_to_nearest_even():
    x = np.array([1.0, 1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 3.14159, -2.5 - 2.0 ** -7, 65504.0, 1e-30])
    want = np.array([1.0, 1.0, 1 + 2.0 ** -6, 3.140625, -2.5, 65536.0, 1.0005271035279193e-30])
    got = O.bf16_round(x)
    assert np.array_equal(got[:6], want[:6])
    assert abs(got[6] - 1e-30) <= 2 ** -8 * 1e-30


def test_bf16_split_carries_sixteen_bits():
    """hi + lo reproduces values of up to 16 significant bits exactly and
    every FP32 value to within 2^-16 of its magnitude."""
    x = np.array([1 + 2.0 ** -8 + 2.0 ** -12, 3.0 + 2.0 ** -14, -0.7 * (1 + 2.0 ** -15)])
    exact = np.array([1 + 2.0 ** -8 + 2.0 ** -12, 3.0 + 2.0 ** -14])
    assert np.array_equal(O.bf16_split(exact), exact)
    rng = np.random.default_rng(9)
    y = rng.standard_normal(10000).astype(np.float32).astype(np.float64) * 10.0 ** rng.integers(-3, 4, 10000)
    assert np.all(np.abs(O.bf16_split(y) - y) <= 2.0 ** -16 * np.abs(y))
    assert np.abs(O.bf16_split(x) - x).max() <= 2.0 ** -16


def test_gradients_match_finite_differences():
    rng = np.random.default_rng(4)
    widths = [3, 5, 4, 2]
    n = sum(widths[i] * widths[i + 1] + widths[i + 1] for i in range(3))
    p = rng.standard_normal(n) * 0.7
    X = rng.standard_normal((6, 3))
    T = rng.standard_normal((6, 2))
    loss, g = O.loss_and_grads(p, widths, X, T)
    h = 1e-6
    for i in range(n):
        e = np.zeros(n)
        e[i] = h
        lp, _ = O.loss_and_grads(p + e, widths, X, T)
        lm, _ = O.loss_and_grads(p - e, widths, X, T)
        assert abs((lp - lm) / (2 * h) - g[i]) <= 1e-7 * max(1.0, abs(g[i])), i


def test_adam_constant_gradient_closed_form():
    g = np.array([0.3, -2.0, 1e-3])
    p = np.zeros(3)
    m1 = np.zeros(3)
    m2 = np.zeros(3)
    for t in range(1, 6):
        p, m1, m2 = O.adam_step(p, g, m1, m2, t, lr=0.01)
    # bias-corrected moments are exactly g and g^2: every step moves lr g/(|g| + eps)
    want = -5 * 0.01 * g / (np.abs(g) + 1e-8)
    assert np.allclose(p, want, rtol=1e-12, atol=0)


def test_forward_single_linear_layer_and_silu():
    rng = np.random.default_rng(2)
    W = rng.standard_normal((4, 3))
    b = rng.standard_normal(4)
    X = rng.standard_normal((5, 3))
    p = np.concatenate([W.ravel(), b])
    assert np.allclose(O.forward(p, [3, 4], X), X @ W.T + b, rtol=1e-14, atol=1e-14)
    # two layers: silu(0) = 0 and silu(z) = z / (1 + e^-z)
    W2 = rng.standard_normal((2, 4))
    p2 = np.concatenate([W.ravel(), b, W2.ravel(), np.zeros(2)])
    z = X @ W.T + b
    assert np.allclose(O.forward(p2, [3, 4, 2], X), (z / (1 + np.exp(-z))) @ W2.T, rtol=1e-13, atol=1e-13)
