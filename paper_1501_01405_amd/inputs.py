"""Seeded synthetic inputs for MRIP runs.

Holds none of the method's arithmetic: it only draws the factor levels and
run lengths of experimental plans, the design of the control-variate
training and application sets, and initial network weights, from numpy's
seeded generator. Both the GPU library and the CPU oracle consume the same
tables.
"""
import math

import numpy as np

ITEM_DTYPE = np.dtype([("dp", "<u4"), ("rep", "<u4"), ("customers", "<u8"),
                       ("lambda_", "<f4"), ("mu", "<f4")])


def plan_table(n_dp=64, reps=32, rho_lo=0.5, rho_hi=0.95, n_lo=1e4, n_hi=1e6, mu=1.0, seed=42,
               dp_base=0):
    """Uneven experimental plan: n_dp design points with rho ~ U[rho_lo, rho_hi]
    (lambda = rho * mu), `reps` replications each, every replication with its
    own log-uniform run length in [n_lo, n_hi] customers. dp-major order."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(rho_lo, rho_hi, n_dp)
    logn = rng.uniform(math.log10(n_lo), math.log10(n_hi), (n_dp, reps))
    n = np.rint(10.0 ** logn).astype(np.uint64)
    items = np.zeros(n_dp * reps, ITEM_DTYPE)
    items["dp"] = np.repeat(np.arange(n_dp, dtype=np.uint32) + dp_base, reps)
    items["rep"] = np.tile(np.arange(reps, dtype=np.uint32), n_dp)
    items["customers"] = n.reshape(-1)
    items["lambda_"] = np.repeat((rho * mu).astype(np.float32), reps)
    items["mu"] = np.float32(mu)
    return items


def uniform_items(n_dp, reps, customers, rho, mu=1.0, dp_base=0, rep_base=0):
    """n_dp design points with the given rho values (array-like, length n_dp),
    `reps` replications each of `customers` customers."""
    rho = np.asarray(rho, dtype=np.float64).reshape(n_dp)
    items = np.zeros(n_dp * reps, ITEM_DTYPE)
    items["dp"] = np.repeat(np.arange(n_dp, dtype=np.uint32) + dp_base, reps)
    items["rep"] = np.tile(np.arange(reps, dtype=np.uint32) + rep_base, n_dp)
    items["customers"] = customers
    items["lambda_"] = np.repeat((rho * mu).astype(np.float32), reps)
    items["mu"] = np.float32(mu)
    return items


def cv_design(n_train=100000, train_reps=32, n_apply_dp=256, reps=64, customers=100000,
              rho_lo=0.5, rho_hi=0.95, seed=7):
    """Control-variate experiment: a training set of n_train replications
    (design points with rho ~ U[rho_lo, rho_hi], `train_reps` replications
    each), then new design points with `reps` replications each. Ids never
    overlap: training dps are 0..n_train/train_reps-1, application dps start
    at n_train."""
    rng = np.random.default_rng(seed)
    n_tdp = max(1, n_train // train_reps)
    train = uniform_items(n_tdp, train_reps, customers, rng.uniform(rho_lo, rho_hi, n_tdp))
    rho = rng.uniform(rho_lo, rho_hi, n_apply_dp)
    apply = uniform_items(n_apply_dp, reps, customers, rho, dp_base=n_train)
    return train, apply


def he_uniform_init(seed=3, d_in=10, hidden=128, d_out=4):
    """Flat fp32 weights [W1 (h x d), b1, W2 (h x h), b2, W3 (d_out x h), b3]
    with W ~ U(-sqrt(6/fan_in), +sqrt(6/fan_in)) and zero biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for rows, cols in ((hidden, d_in), (hidden, hidden), (d_out, hidden)):
        lim = math.sqrt(6.0 / cols)
        parts.append(rng.uniform(-lim, lim, rows * cols))
        parts.append(np.zeros(rows))
    return np.concatenate(parts).astype(np.float32)
