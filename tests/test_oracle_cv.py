"""Pins for the oracle's control-variate estimator and training host steps.

Independent facts used: a zero control reduces the estimator exactly to the
plain mean; it is unbiased with the Monte Carlo variance in a model with a
known mean; numpy's own statistics for the z-scores; least squares on the
demeaned data (numpy's lstsq on the stacked deviations) for the pooled
regression, and exact recovery of a noise-free linear law; the exhaustive
average of -ln u over its 2^24-point grid for the variates' mean.
"""
import math

import numpy as np

from oracle import cv


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


def _deviations(v, sel, dp):
    return np.concatenate([v[sel & (dp == d)] - v[sel & (dp == d)].mean(axis=0)
                           for d in np.unique(dp[sel])])


def test_pooled_regression_recovers_a_linear_law_and_equals_demeaned_least_squares():
    rng = np.random.default_rng(5)
    dp, rho = _binned_design(rng, range(16))
    k_of = np.array([cv.rho_bin(r, 0.5, 0.95, 16) for r in rho])
    a = np.stack([0.2 + 0.1 * k_of, -1.0 + 0.05 * k_of, 3.0 - 0.2 * k_of], axis=1)
    # per-dp offsets in the controls and in the response do not matter
    F = rng.normal(size=(dp.size, 3)) + np.stack([3.0 * dp, -dp, 0.5 * dp], axis=1)
    Y = np.sum(a * F, axis=1) + 50.0 * dp
    coef = cv.pooled_regression_table(Y, F, dp, rho, 0.5, 0.95)
    want = np.stack([0.2 + 0.1 * np.arange(16), -1.0 + 0.05 * np.arange(16),
                     3.0 - 0.2 * np.arange(16)], axis=1)
    assert np.allclose(coef, want, rtol=1e-9, atol=1e-10)
    # with noise: each bin equals least squares on the within-dp deviations
    Yn = Y + 0.3 * rng.normal(size=dp.size)
    coef = cv.pooled_regression_table(Yn, F, dp, rho, 0.5, 0.95)
    for k in range(16):
        sel = k_of == k
        ls = np.linalg.lstsq(_deviations(F, sel, dp), _deviations(Yn, sel, dp), rcond=None)[0]
        assert np.allclose(coef[k], ls, rtol=1e-9, atol=1e-12)
    # one column: the pooled slope sum(dy dg) / sum(dg^2), written out
    G = F[:, 0]
    one = cv.pooled_regression_table(Yn, G, dp, rho, 0.5, 0.95)
    for k in range(16):
        sel = k_of == k
        gd, yd = _deviations(G, sel, dp), _deviations(Yn, sel, dp)
        sxy = sxx = 0.0
        for u, v in zip(gd, yd):
            sxy += u * v
            sxx += u * u
        assert abs(one[k, 0] - sxy / sxx) < 1e-10 * abs(sxy / sxx)


def test_pooled_regression_degenerate_columns_and_neighbour_fill():
    rng = np.random.default_rng(6)
    dp, rho = _binned_design(rng, range(16))
    Y = rng.normal(size=dp.size)
    # a column constant within every design point (a constant network's
    # control) gets 0 and leaves the others' fit unchanged
    F = np.stack([(0.7 * dp).astype(np.float32).astype(np.float64), rng.normal(size=dp.size)],
                 axis=1)
    both = cv.pooled_regression_table(Y, F, dp, rho, 0.5, 0.95)
    alone = cv.pooled_regression_table(Y, F[:, 1], dp, rho, 0.5, 0.95)
    assert np.all(both[:, 0] == 0.0) and np.allclose(both[:, 1], alone[:, 0], rtol=1e-12)
    # a control that moves against Y keeps its sign (no clamp)
    G = rng.normal(size=dp.size)
    assert np.allclose(cv.pooled_regression_table(-2.0 * G, G, dp, rho, 0.5, 0.95), -2.0)
    # only bins 3 and 9 hold design points: the others borrow the nearest,
    # the lower one on a tie (bin 6 is 3 from both)
    dp, rho = _binned_design(rng, [3, 9])
    G = rng.normal(size=dp.size)
    k_of = np.array([cv.rho_bin(r, 0.5, 0.95, 16) for r in rho])
    Y = np.where(k_of == 3, 1.5, 4.0) * G
    coef = cv.pooled_regression_table(Y, G, dp, rho, 0.5, 0.95)[:, 0]
    assert np.allclose(coef[:7], 1.5) and np.allclose(coef[7:], 4.0)
    # no design point at all: every coefficient 0
    assert np.all(cv.pooled_regression_table(Y[:0], G[:0], dp[:0], rho[:0], 0.5, 0.95) == 0)


# ------------------------------------------------- the martingale controls

def test_log_grid_mean_equals_exhaustive_average():
    k = np.arange(1, 2 ** 24 + 1, dtype=np.float64)
    exact = -np.mean(np.log(k * 2.0 ** -24))
    assert abs(cv.LOG_GRID_MEAN - exact) < 1e-12
    assert 1.0 - 1e-6 < cv.LOG_GRID_MEAN < 1.0  # the cut tail: about 5.5e-7


def test_control_multipliers_scale_per_customer_and_service_time():
    c = np.array([4.0, -2.0, 8.0, 6.0])
    assert np.array_equal(cv.control_multipliers(c, 4, 1.0), [1.0, -0.5, 2.0, 1.5])
    # mu = 2: the service scale is 1/2, the weighted pair doubles
    assert np.array_equal(cv.control_multipliers(c, 4, 2.0), [1.0, -0.5, 4.0, 3.0])
    # all eight: the prefix four scale the same way, by the whole run length
    c8 = np.concatenate([c, 2.0 * c])
    assert np.array_equal(cv.control_multipliers(c8, 4, 2.0),
                          [1.0, -0.5, 4.0, 3.0, 2.0, -1.0, 8.0, 6.0])


def test_design_point_sd_and_training_multipliers():
    rng = np.random.default_rng(9)
    dp = np.repeat(np.arange(5), 16)
    rng.shuffle(dp)
    Y = rng.normal(size=dp.size) * (1 + dp)
    Y[dp == 3] = 2.0
    sd = cv.design_point_sd(Y, dp)
    for d in range(5):
        assert np.allclose(sd[dp == d], np.std(Y[dp == d], ddof=1), rtol=1e-13)
    Z = rng.normal(size=(dp.size, 4))
    M = cv.training_multipliers(Z, sd)
    assert np.all(M[dp == 3] == 0.0)
    ok = dp != 3
    assert np.allclose(M[ok] * sd[ok, None], Z[ok], rtol=1e-13)
    # the standardised target and the multipliers share the scale: a network
    # predicting g fits t exactly when Y - mean_dp Y = sum_k g_k z_k
    g = np.array([0.5, -1.0, 2.0, 0.25])
    Y2 = Z @ g + 10.0 * dp
    t = cv.standardized_target(Y2, dp)
    M2 = cv.training_multipliers(Z - np.array([Z[dp == d].mean(0) for d in dp]),
                                 cv.design_point_sd(Y2, dp))
    assert np.allclose(cv.control_value(np.tile(g, (dp.size, 1)), M2), t, atol=1e-12)


def test_known_mean_estimator_reduces_unbiased_and_matches_variance():
    rng = np.random.default_rng(8)
    Y = rng.normal(3.0, 2.0, 64)
    zero = cv.known_mean_control_variate(Y, np.zeros(64), 2.0)
    pl = cv.plain(Y)
    assert abs(zero["mean"] - pl["mean"]) < 1e-12 and abs(zero["var"] - pl["var"]) < 1e-12
    # Y = 1 + 2 H + e with E[H] = 0: unbiased, variance 0.25 / n
    n, K = 64, 2000
    ests, vs = [], []
    for _ in range(K):
        H = rng.normal(size=n)
        Yk = 1.0 + 2.0 * H + 0.5 * rng.normal(size=n)
        r = cv.known_mean_control_variate(Yk, H, 2.0)
        ests.append(r["mean"])
        vs.append(r["var"])
    ests = np.array(ests)
    assert abs(ests.mean() - 1.0) < 4 * ests.std() / np.sqrt(K)
    assert abs(ests.var() / (0.25 / n) - 1) < 4 * np.sqrt(2.0 / K)
    assert abs(np.mean(vs) / (0.25 / n) - 1) < 0.05
    H = rng.normal(size=n)
    assert cv.known_mean_control_variate(5.0 + 3.0 * H, H, 3.0)["var"] < 1e-28
    # several columns: Y - F a written out per replication
    F = rng.normal(size=(n, 3))
    a = np.array([0.5, -2.0, 1.25])
    Y = 2.0 + F @ a + 0.1 * rng.normal(size=n)
    r = cv.known_mean_control_variate(Y, F, a)
    d = [Y[i] - (F[i, 0] * a[0] + F[i, 1] * a[1] + F[i, 2] * a[2]) for i in range(n)]
    assert abs(r["mean"] - np.mean(d)) < 1e-12 and abs(r["var"] - np.var(d, ddof=1) / n) < 1e-14
