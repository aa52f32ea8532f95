"""Pins for the oracle's control-variate network (forward, backward, Adam).

Independent facts used: central finite differences of the fp64 loss for
every gradient (a dropped term, a wrong transpose or a wrong ReLU mask
fails them); bfloat16 rounding against its bit-level definition on
exhaustive edge patterns; Adam's first step, which moves every weight by
lr * g / (|g| + eps) (Kingma and Ba 2015); convergence on a toy fit.
"""
import numpy as np
import pytest

from oracle import mlp


def _theta(seed, scale=0.3):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, mlp.N_PARAMS)


def test_param_count():
    assert mlp.N_PARAMS == 128 * 10 + 128 + 128 * 128 + 128 + 4 * 128 + 4 == 18436


@pytest.mark.parametrize("mult", [False, True])
def test_gradient_matches_finite_differences(mult):
    rng = np.random.default_rng(0)
    X = rng.normal(size=(7, 10))
    y = rng.normal(size=7)
    z = rng.normal(size=(7, 4)) if mult else None
    theta = _theta(1)
    g, _ = mlp.backward(theta, X, y, bf16=False, z=z)
    idx = np.concatenate([rng.choice(np.arange(0, 1280), 40, replace=False),  # W1
                          np.arange(1280, 1290),  # b1
                          rng.choice(np.arange(1408, 1408 + 16384), 60, replace=False),  # W2
                          np.arange(17792, 17800),  # b2
                          rng.choice(np.arange(17920, 18432), 40, replace=False),  # W3
                          np.arange(18432, 18436)])  # b3
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (mlp.loss(tp, X, y, bf16=False, z=z) - mlp.loss(tm, X, y, bf16=False, z=z)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, i
    if not mult:  # without multipliers only the first output is trained
        assert np.all(g[18048:18432] == 0.0) and np.all(g[18433:] == 0.0)


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


# The rounding points of the bf16 reading: both operands of every matrix
# product are rounded to bfloat16 (X, W1, H1, W2, H2, W3 forward; dy, dZ2,
# dZ1 backward); biases, ReLU masks and sums stay unrounded.
_POINTS = ("X", "W1", "H1", "W2", "H2", "W3", "dy", "dZ2", "dZ1")


def _layerwise(theta, X, y, z, points):
    """The network written out layer by layer in fp64, rounding to bfloat16
    with torch's own conversion (an implementation independent of the
    oracle's bit arithmetic) exactly at `points`; z: (n, 4) multipliers."""
    import torch

    def r(name, v):
        v = np.asarray(v, np.float64)
        if name not in points:
            return v
        t = torch.from_numpy(v.astype(np.float32)).to(torch.bfloat16)
        return t.to(torch.float64).numpy()

    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)  # noqa: E731
    W1 = theta[:1280].reshape(128, 10)
    b1 = theta[1280:1408]
    W2 = theta[1408:17792].reshape(128, 128)
    b2 = theta[17792:17920]
    W3 = theta[17920:18432].reshape(4, 128)
    b3 = theta[18432:18436]
    Xr = r("X", X)
    z1 = Xr @ r("W1", W1).T + b1
    h1 = r("H1", f32(np.maximum(z1, 0.0)))
    z2 = h1 @ r("W2", W2).T + b2
    h2 = r("H2", f32(np.maximum(z2, 0.0)))
    out = h2 @ r("W3", W3).T + b3
    n = X.shape[0]
    pred = np.einsum("nk,nk->n", out, z)
    dy = f32(2.0 * (pred - y)[:, None] * z / n)
    dyr = r("dy", dy)
    gW3 = dyr.T @ h2
    gb3 = dy.sum(0)
    dz2 = f32((dyr @ r("W3", W3)) * (z2 > 0))
    dz2r = r("dZ2", dz2)
    gW2 = dz2r.T @ h1
    gb2 = dz2.sum(0)
    dz1 = f32((dz2r @ r("W2", W2)) * (z1 > 0))
    gW1 = r("dZ1", dz1).T @ Xr
    gb1 = dz1.sum(0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return out, grad


def test_bf16_path_rounds_exactly_at_the_stated_points():
    rng = np.random.default_rng(11)
    X = rng.normal(size=(48, 10)).astype(np.float32)
    y = rng.normal(size=48).astype(np.float32)
    z = rng.normal(size=(48, 4)).astype(np.float32).astype(np.float64)
    theta = _theta(12, 0.25).astype(np.float32).astype(np.float64)
    got_y, _ = mlp.forward(theta, X, bf16=True)
    got_g, _ = mlp.backward(theta, X, y, bf16=True, z=z)
    want_y, want_g = _layerwise(theta, X, y, z, set(_POINTS))
    scale = np.max(np.abs(want_g))
    assert np.allclose(got_y, want_y, rtol=1e-9, atol=1e-12)
    assert np.max(np.abs(got_g - want_g)) <= 1e-9 * scale
    # the comparison sees each rounding point: leaving any one out moves the
    # prediction or some gradient far beyond the tolerance above
    for p in _POINTS:
        y2, g2 = _layerwise(theta, X, y, z, set(_POINTS) - {p})
        moved = max(np.max(np.abs(y2 - want_y)) / np.max(np.abs(want_y)),
                    np.max(np.abs(g2 - want_g)) / scale)
        assert moved > 1e-6, p


def test_one_hot_multipliers_select_an_output():
    # z = e_k for every sample is the plain regression of output k; e_0 is
    # the default
    rng = np.random.default_rng(13)
    X = rng.normal(size=(9, 10)).astype(np.float32)
    y = rng.normal(size=9)
    theta = _theta(14)
    out, _ = mlp.forward(theta, X)
    for k in range(4):
        e = np.zeros((9, 4), np.float32)
        e[:, k] = 1.0
        assert mlp.loss(theta, X, y, z=e) == float(np.mean((out[:, k] - y) ** 2))
    e0 = np.zeros((9, 4), np.float32)
    e0[:, 0] = 1.0
    g1, _ = mlp.backward(theta, X, y, bf16=True, z=e0)
    g0, _ = mlp.backward(theta, X, y, bf16=True)
    assert np.array_equal(g0, g1)


def test_multipliers_fit_a_coefficient_law():
    # y = sum_k c_k(x) z_k with coefficients that depend on x: training on
    # (x, z, y) recovers the coefficients, whatever the z
    rng = np.random.default_rng(15)
    n = 512
    X = rng.normal(size=(n, 10)).astype(np.float32)
    Z = rng.normal(size=(n, 4)).astype(np.float32)
    C = np.stack([1.0 + 0.5 * X[:, 0], -0.7 * np.ones(n), 0.3 * X[:, 1], 0.2 + 0 * X[:, 2]], 1)
    y = np.sum(C * Z, axis=1)
    theta = _theta(16, 0.1)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    l0 = mlp.loss(theta, X, y, z=Z)
    for step in range(1, 401):
        g, _ = mlp.backward(theta, X, y, z=Z)
        theta, m, v = mlp.adam_step(theta, m, v, g, step, lr=3e-3)
    assert mlp.loss(theta, X, y, z=Z) < 0.05 * l0
    out, _ = mlp.forward(theta, X)
    assert np.sqrt(np.mean((out - C) ** 2)) < 0.2
