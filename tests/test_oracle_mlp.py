"""Pins for the oracle's control-variate network (forward, backward, Adam).

Independent facts used: central finite differences of the fp64 loss for
every gradient (a dropped term, a wrong transpose or a wrong ReLU mask
fails them); bfloat16 rounding against its bit-level definition on
exhaustive edge patterns; Adam's first step, which moves every weight by
lr * g / (|g| + eps) (Kingma and Ba 2015); convergence on a toy fit.
"""
import numpy as np

from oracle import mlp


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 18049


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(0)
    X = rng.normal(size=(7, 10))
    y = rng.normal(size=7)
    theta = _theta(1)
    g, _ = mlp.backward(theta, X, y, bf16=False)
    idx = np.concatenate([rng.choice(np.arange(0, 1280), 40, replace=False),  # W1
                          np.arange(1280, 1290),  # b1
                          rng.choice(np.arange(1408, 1408 + 16384), 60, replace=False),  # W2
                          np.arange(17792, 17800),  # b2
                          np.arange(17920, 17930),  # W3
                          [18048]])  # b3
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, y, bf16=False) - mlp.loss(tm, X, y, bf16=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, i


def test_bf16_rounding_definition():
    # bf16 keeps the top 16 bits; round to nearest, ties to even
    vals = np.array([1.0, 1.00390625, 1.005859375, 1.0078125 + 2**-9, -3.14159265, 0.0,
                     65504.0, 1e-30], np.float32)
    got = mlp.bf16_round(vals)
    bits = vals.view(np.uint32)
    for v, b, r in zip(vals, bits, got):
        lo = int(b) & 0xFFFF
        hi = int(b) >> 16
        if lo > 0x8000 or (lo == 0x8000 and (hi & 1)):
            hi += 1
        expect = np.array([hi << 16], np.uint32).view(np.float32)[0]
        assert r == expect, (v, r, expect)
    assert mlp.bf16_round(np.float32(1.0 + 2**-8))[()] == 1.0  # tie to even (down)
    assert mlp.bf16_round(np.float32(1.0 + 3 * 2**-8))[()] == 1.0 + 2**-6  # tie to even (up)


def test_bf16_forward_close_to_fp64_forward():
    rng = np.random.default_rng(2)
    X = rng.normal(size=(64, 10)).astype(np.float32)
    theta = _theta(3, 0.2)
    a, _ = mlp.forward(theta, X, bf16=True)
    b, _ = mlp.forward(theta, X, bf16=False)
    assert np.max(np.abs(a - b)) < 0.05 * (np.max(np.abs(b)) + 1)


def test_adam_first_step_is_sign_step():
    rng = np.random.default_rng(4)
    theta = rng.normal(size=100)
    g = rng.normal(size=100)
    new, m, v = mlp.adam_step(theta, np.zeros(100), np.zeros(100), g, 1, lr=1e-3)
    assert np.allclose(theta - new, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_training_reduces_loss():
    rng = np.random.default_rng(5)
    X = rng.normal(size=(256, 10)).astype(np.float32)
    y = (X[:, 0] * 2.0 - X[:, 3] + 0.5).astype(np.float32)
    theta = _theta(6, 0.1)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, y)
    for step in range(1, 201):
        g, _ = mlp.backward(theta, X, y)
        theta, m, v = mlp.adam_step(theta, m, v, g, step, lr=3e-3)
    assert mlp.loss(theta, X, y) < 0.05 * l0
