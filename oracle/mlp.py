"""Learned control variate, oracle side -- TEST INFRASTRUCTURE ONLY.

The paper has no variance reduction; the control variate is the growth path
the method's statement of work adds. What is computed:

  network   10 -> 128 -> 128 -> 4, ReLU after the two hidden layers; the
            four outputs are the coefficients of four zero-mean controls.
  operands  every matrix product rounds both of its operands to bfloat16
            (round to nearest, ties to even) and accumulates exactly here
            (fp64); biases and the ReLU masks stay in fp32/fp64.
  loss      mean squared error over the batch of sum_k g_k(x) z_k, with a
            per-sample multiplier vector z (the sample's controls); without
            multipliers, of the first output g_0(x) alone (z = e_0).
  optimizer Adam (Kingma and Ba, 2015, Algorithm 1) on fp32 master weights.

Parameters are the flat fp32 vector [W1 (128x10), b1 (128), W2 (128x128),
b2 (128), W3 (4x128), b3 (4)], row-major, 18436 values.

`bf16=False` turns the rounding off, which is what the finite-difference
gradient pin uses.
"""
import numpy as np

D_IN, H, D_OUT = 10, 128, 4
SHAPES = (("W1", (H, D_IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (D_OUT, H)),
          ("b3", (D_OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (N_PARAMS,)
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[off:off + n].reshape(shape)
        off += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1)
                           for name, _ in SHAPES])


def bf16_round(x):
    """Round fp32 values to the nearest bfloat16 (ties to even), returned as fp64."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def _op(x, bf16):
    return bf16_round(x) if bf16 else np.asarray(x, dtype=np.float64)


def forward(theta, X, bf16=True):
    """Prediction and the intermediates backward() needs. X: (n, 10)."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float32 if bf16 else np.float64)
    z1 = _op(X, bf16) @ _op(p["W1"], bf16).T + p["b1"]
    h1 = np.maximum(z1, 0.0)
    if bf16:
        h1 = h1.astype(np.float32)
    z2 = _op(h1, bf16) @ _op(p["W2"], bf16).T + p["b2"]
    h2 = np.maximum(z2, 0.0)
    if bf16:
        h2 = h2.astype(np.float32)
    y = _op(h2, bf16) @ _op(p["W3"], bf16).T + p["b3"]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def _mult(z, n):
    """Per-sample multipliers as fp64 (n, 4); None is e_0 for every sample."""
    if z is None:
        m = np.zeros((n, D_OUT))
        m[:, 0] = 1.0
        return m
    z = np.asarray(z, np.float32).astype(np.float64)
    assert z.shape == (n, D_OUT)
    return z


def predict(theta, X, bf16=True, z=None):
    """sum_k g_k(x) z_k per sample (g_0(x) without multipliers)."""
    yh, _ = forward(theta, X, bf16)
    return np.sum(yh * _mult(z, yh.shape[0]), axis=1)


def loss(theta, X, y, bf16=True, z=None):
    return float(np.mean((predict(theta, X, bf16, z) - np.asarray(y, np.float64)) ** 2))


def backward(theta, X, y, bf16=True, z=None):
    """Gradient of the mean squared error of sum_k g_k(x) z_k, flat like
    theta, and the loss. The output gradient dy_k = 2 (pred - y) z_k / n is
    rounded to fp32 before it enters the products."""
    p = unpack(theta)
    yh, c = forward(theta, X, bf16)
    n = yh.shape[0]
    y = np.asarray(y, np.float64)
    zz = _mult(z, n)
    err = np.sum(yh * zz, axis=1) - y
    dy = (2.0 * err / n)[:, None] * zz
    if bf16:
        dy = dy.astype(np.float32)
    g = {}
    g["W3"] = _op(dy, bf16).T @ _op(c["h2"], bf16)
    g["b3"] = np.sum(np.asarray(dy, np.float64), axis=0)
    dh2 = _op(dy, bf16) @ _op(p["W3"], bf16)
    dz2 = dh2 * (c["z2"] > 0)
    if bf16:
        dz2 = dz2.astype(np.float32)
    g["W2"] = _op(dz2, bf16).T @ _op(c["h1"], bf16)
    g["b2"] = np.sum(np.asarray(dz2, np.float64), axis=0)
    dh1 = _op(dz2, bf16) @ _op(p["W2"], bf16)
    dz1 = dh1 * (c["z1"] > 0)
    if bf16:
        dz1 = dz1.astype(np.float32)
    g["W1"] = _op(dz1, bf16).T @ _op(c["X"], bf16)
    g["b1"] = np.sum(np.asarray(dz1, np.float64), axis=0)
    return pack(g), float(np.mean(err ** 2))


def adam_step(theta, m, v, grad, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step counts from 1). Returns new (theta, m, v) in fp64."""
    g = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    theta = np.asarray(theta, np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def normalize(X, mean, std):
    """z-score features with the training set's mean and std (std 0 -> 1)."""
    std = np.where(np.asarray(std) > 0, std, 1.0)
    return ((np.asarray(X, np.float64) - mean) / std).astype(np.float32)
