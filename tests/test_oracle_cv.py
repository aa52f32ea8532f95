"""Pins for the oracle's two-phase control-variate estimator.

Independent facts used: a constant control (g = c) reduces the estimator
exactly to the plain mean; the estimator is unbiased in a model with a known
mean; its variance matches the Monte Carlo variance over many experiments;
a perfectly correlated control removes the first-phase variance.
"""
import math

import numpy as np

from oracle import cv


def test_constant_control_reduces_to_plain():
    rng = np.random.default_rng(0)
    Y = rng.normal(5.0, 1.0, 64)
    c = 2.5
    G = np.full(64, c)
    Gp = np.full(200, c)
    a = cv.control_variate(Y, G, Gp, beta=1.0)
    b = cv.plain(Y)
    assert abs(a["mean"] - b["mean"]) < 1e-12
    assert abs(a["var"] - b["var"]) < 1e-12


def test_unbiased_and_variance_estimate():
    # Y = X + e with X ~ N(0, 1), e ~ N(0, 0.1^2); control g(X) = X; E[Y] = 0
    rng = np.random.default_rng(1)
    n, M, K = 64, 512, 3000
    ests, vars_ = [], []
    for _ in range(K):
        X = rng.normal(size=n)
        Y = X + 0.1 * rng.normal(size=n)
        Xp = rng.normal(size=M)
        r = cv.control_variate(Y, X, Xp, beta=1.0)
        ests.append(r["mean"])
        vars_.append(r["var"])
    ests = np.array(ests)
    assert abs(ests.mean()) < 4 * ests.std() / math.sqrt(K)
    true_var = 0.01 / n + 1.0 / M
    assert abs(ests.var() / true_var - 1) < 0.1
    assert abs(np.mean(vars_) / true_var - 1) < 0.05


def test_perfect_control_leaves_second_phase_only():
    rng = np.random.default_rng(2)
    X = rng.normal(size=64)
    Xp = rng.normal(size=1000)
    r = cv.control_variate(3 * X + 1, X, Xp, beta=3.0)
    assert abs(r["var"] - 9 * np.var(Xp, ddof=1) / 1000) < 1e-12
