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


# ------------------------------------------------------ training host steps

def test_feature_stats_against_numpy_and_invariants():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(500, 10)) * np.arange(1, 11) + np.arange(10)
    X[:, 1] = 1.0  # a constant column (mu in a plan with one service rate)
    X = X.astype(np.float32)
    mean, std = cv.feature_stats(X)
    x64 = X.astype(np.float64)
    assert np.allclose(mean, x64.mean(0), rtol=1e-13, atol=1e-13)
    want = x64.std(0, ddof=0)
    want[1] = 1.0
    assert np.allclose(std, want, rtol=1e-12)
    z = (x64 - mean) / std
    assert np.allclose(z.mean(0), 0.0, atol=1e-12)
    assert np.allclose(np.delete(z.std(0), 1), 1.0, rtol=1e-12)
    assert np.all(z[:, 1] == 0.0)


def test_standardized_target_is_zero_mean_unit_variance_per_design_point():
    rng = np.random.default_rng(4)
    dp = np.repeat(np.arange(7), 32)
    rng.shuffle(dp)
    Y = rng.gamma(2.0, 3.0, dp.size) + 10.0 * dp
    Y[dp == 5] = 4.25  # a design point with no spread
    t = cv.standardized_target(Y, dp)
    for d in range(7):
        td = t[dp == d]
        if d == 5:
            assert np.all(td == 0.0)
            continue
        assert abs(td.mean()) < 1e-12
        assert abs(td.var(ddof=1) - 1.0) < 1e-12
    # invariant to a positive affine change of Y within each design point
    a = 1.0 + dp * 0.5
    b = -3.0 * dp
    assert np.allclose(cv.standardized_target(a * Y + b, dp), t, atol=1e-12)


def test_holdout_is_the_last_fifth_of_the_design_points():
    assert cv.holdout_design_points(range(3125)) == list(range(2500, 3125))
    assert cv.holdout_design_points([9, 2, 2, 5]) == [9]
    assert cv.holdout_design_points(range(5)) == [4]
    assert cv.holdout_design_points(range(10, 20)) == [18, 19]


def test_rho_bins_edges_and_centres():
    lo, hi = 0.5, 0.95
    assert cv.rho_bin(lo, lo, hi, 16) == 0
    assert cv.rho_bin(hi, lo, hi, 16) == 15
    assert cv.rho_bin(0.1, lo, hi, 16) == 0
    assert cv.rho_bin(1.2, lo, hi, 16) == 15
    for k in range(16):
        assert cv.rho_bin(lo + (k + 0.5) * (hi - lo) / 16, lo, hi, 16) == k


def _binned_design(rng, bins_used, reps=24, per_bin=6, lo=0.5, hi=0.95):
    dp, rho = [], []
    d = 0
    for k in bins_used:
        for _ in range(per_bin):
            r = lo + (k + rng.uniform(0.1, 0.9)) * (hi - lo) / 16
            dp += [d] * reps
            rho += [r] * reps
            d += 1
    return np.array(dp), np.array(rho, np.float32)


def test_pooled_slope_recovers_a_linear_law_and_equals_demeaned_least_squares():
    rng = np.random.default_rng(5)
    dp, rho = _binned_design(rng, range(16))
    k_of = np.array([cv.rho_bin(r, 0.5, 0.95, 16) for r in rho])
    a = 0.2 + 0.1 * k_of  # true slope per bin
    G = rng.normal(size=dp.size) + 3.0 * dp  # per-dp offsets in the control ...
    Y = a * G + 50.0 * dp  # ... and in the response do not matter
    beta = cv.pooled_slope_table(Y, G, dp, rho, 0.5, 0.95)
    assert np.allclose(beta, 0.2 + 0.1 * np.arange(16), rtol=1e-10)
    # with noise: each bin equals least squares on the within-dp deviations
    Yn = Y + 0.3 * rng.normal(size=dp.size)
    beta = cv.pooled_slope_table(Yn, G, dp, rho, 0.5, 0.95)
    for k in range(16):
        sel = k_of == k
        yd = np.concatenate([Yn[sel & (dp == d)] - Yn[sel & (dp == d)].mean()
                             for d in np.unique(dp[sel])])
        gd = np.concatenate([G[sel & (dp == d)] - G[sel & (dp == d)].mean()
                             for d in np.unique(dp[sel])])
        ls = np.linalg.lstsq(gd[:, None], yd, rcond=None)[0][0]
        assert abs(beta[k] - max(ls, 0.0)) < 1e-10
        se = 0.3 / np.sqrt(np.sum(gd * gd))
        assert abs(beta[k] - (0.2 + 0.1 * k)) < 4 * se


def test_pooled_slope_constant_network_negative_slope_and_neighbour_fill():
    rng = np.random.default_rng(6)
    dp, rho = _binned_design(rng, range(16))
    Y = rng.normal(size=dp.size)
    # a network constant within every design point (fp32 outputs, as the
    # network gives them) gives no slope anywhere
    G = (0.7 * dp).astype(np.float32).astype(np.float64)
    assert np.all(cv.pooled_slope_table(Y, G, dp, rho, 0.5, 0.95) == 0.0)
    # a control that moves against Y is clamped to plain MRIP
    G = rng.normal(size=dp.size)
    assert np.all(cv.pooled_slope_table(-2.0 * G, G, dp, rho, 0.5, 0.95) == 0.0)
    # only bins 3 and 9 hold design points: the others borrow the nearest,
    # the lower one on a tie (bin 6 is 3 from both)
    dp, rho = _binned_design(rng, [3, 9])
    G = rng.normal(size=dp.size)
    k_of = np.array([cv.rho_bin(r, 0.5, 0.95, 16) for r in rho])
    Y = np.where(k_of == 3, 1.5, 4.0) * G
    beta = cv.pooled_slope_table(Y, G, dp, rho, 0.5, 0.95)
    assert np.allclose(beta[:7], 1.5) and np.allclose(beta[7:], 4.0)


# ------------------------------------------------- the input control variate

def test_log_grid_mean_equals_exhaustive_average():
    k = np.arange(1, 2 ** 24 + 1, dtype=np.float64)
    exact = -np.mean(np.log(k * 2.0 ** -24))
    assert abs(cv.LOG_GRID_MEAN - exact) < 1e-12
    assert 1.0 - 1e-6 < cv.LOG_GRID_MEAN < 1.0  # the cut tail: about 5.5e-7


def test_input_control_is_standard_and_independent_of_the_features():
    from oracle import core
    N, K, R = 900, 300, 4000
    for lam in (0.6, 0.95):
        _, feat, post = core.mm1_many(11, R, N, lam, 1.0, features=K, threads=8, post=True)
        z = np.array([cv.input_control(p, N, K, lam, 1.0) for p in post])
        assert abs(z.mean()) < 4 / np.sqrt(R)
        assert abs(z.var(ddof=1) - 1.0) < 4 * np.sqrt(2.0 / R)
        for j in range(2, 10):  # the prefix statistics
            c = np.corrcoef(feat[:, j], z)[0, 1]
            assert abs(c) < 4 / np.sqrt(R), (lam, j, c)
        # any fixed function of the features times z has mean 0
        h = np.tanh(feat[:, 9] / 5.0 - 1.0) * z
        assert abs(h.mean()) < 4 * h.std(ddof=1) / np.sqrt(R)
    assert cv.input_control(123.0, 500, 500, 0.9, 1.0) == 0.0


def test_known_mean_estimator_reduces_unbiased_and_matches_variance():
    rng = np.random.default_rng(8)
    Y = rng.normal(3.0, 2.0, 64)
    zero = cv.known_mean_control_variate(Y, np.zeros(64), beta=2.0)
    pl = cv.plain(Y)
    assert abs(zero["mean"] - pl["mean"]) < 1e-12 and abs(zero["var"] - pl["var"]) < 1e-12
    # Y = 1 + 2 H + e with E[H] = 0: unbiased, variance 0.25 / n
    n, K = 64, 2000
    ests, vs = [], []
    for _ in range(K):
        H = rng.normal(size=n)
        Yk = 1.0 + 2.0 * H + 0.5 * rng.normal(size=n)
        r = cv.known_mean_control_variate(Yk, H, beta=2.0)
        ests.append(r["mean"])
        vs.append(r["var"])
    ests = np.array(ests)
    assert abs(ests.mean() - 1.0) < 4 * ests.std() / np.sqrt(K)
    assert abs(ests.var() / (0.25 / n) - 1) < 4 * np.sqrt(2.0 / K)
    assert abs(np.mean(vs) / (0.25 / n) - 1) < 0.05
    H = rng.normal(size=n)
    assert cv.known_mean_control_variate(5.0 + 3.0 * H, H, beta=3.0)["var"] < 1e-28
