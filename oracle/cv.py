"""Control-variate estimator, oracle side -- TEST INFRASTRUCTURE ONLY.

Two-phase control variate for one design point (a control variate whose mean
is estimated from a second, independent sample):

  n full replications give (Y_i, g_i = g(X_i)); M prefix-only replications,
  with stream ids disjoint from the full ones, give g'_j = g(X'_j). With a
  fixed coefficient beta,

      Y_cv = mean_i(Y_i - beta g_i) + beta mean_j(g'_j)

  is unbiased for E[Y] for any fixed g, because E[g(X)] = E[g(X')]. Its
  variance estimate is s^2(Y - beta g)/n + beta^2 s^2(g')/M, and the interval
  uses the Welch-Satterthwaite degrees of freedom. The plain estimate
  mean(Y) with a t_{n-1} interval is the fallback.

Training's host steps (feature z-scores, the standardised within-design-
point target, the held-out design points, and the per-bin pooled slope of Y
on the control with its clamp at zero and nearest-bin fill) follow below,
one function each.
"""
import math

import numpy as np

from .stats import t_quantile


def _mean_var(x):
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    s = 0.0
    for v in x:
        s += v
    m = s / n
    ss = 0.0
    for v in x:
        ss += (v - m) * (v - m)
    return m, ss / (n - 1)


def plain(Y, confidence=0.95):
    m, v = _mean_var(Y)
    n = len(Y)
    tq = t_quantile(0.5 + confidence / 2.0, n - 1)
    return dict(mean=m, var=v / n, half_width=tq * math.sqrt(v / n), dof=float(n - 1))


def control_variate(Y, G, Gp, beta, confidence=0.95):
    Y, G, Gp = (np.asarray(a, np.float64) for a in (Y, G, Gp))
    n, M = Y.shape[0], Gp.shape[0]
    m1, v1 = _mean_var(Y - beta * G)
    m2, v2 = _mean_var(Gp)
    est = m1 + beta * m2
    a, b = v1 / n, beta * beta * v2 / M
    var = a + b
    denom = a * a / (n - 1) + b * b / (M - 1)
    dof = var * var / denom if denom > 0 else float(n - 1)
    tq = t_quantile(0.5 + confidence / 2.0, dof)
    return dict(mean=est, var=var, half_width=tq * math.sqrt(var), dof=dof)


# ----------------------------------------------------------------- training
# The host steps of training the control variate, one function each, as the
# method states them (not in the paper; they extend MRIP's estimator).

def feature_stats(X):
    """Per-column mean and population standard deviation of the training
    features, sequential fp64 sums in row order; a column whose deviation is
    not above 1e-12 gets 1 (it is constant and z-scores to 0)."""
    X = np.asarray(X, np.float64)
    n, cols = X.shape
    mean = np.zeros(cols)
    std = np.ones(cols)
    for j in range(cols):
        s = 0.0
        for i in range(n):
            s += X[i, j]
        m = s / n
        ss = 0.0
        for i in range(n):
            ss += (X[i, j] - m) * (X[i, j] - m)
        sd = math.sqrt(ss / n)
        mean[j] = m
        std[j] = sd if sd > 1e-12 else 1.0
    return mean, std


def standardized_target(Y, dp):
    """t_i = (Y_i - mean of Y over i's design point) / (its unbiased standard
    deviation), 0 where that deviation is 0: the within-design-point variation
    a control variate can use, on one scale for every factor level."""
    Y = np.asarray(Y, np.float64)
    dp = np.asarray(dp)
    t = np.zeros(Y.shape[0])
    for d in sorted(set(dp.tolist())):
        idx = np.flatnonzero(dp == d)
        m, v = _mean_var(Y[idx])
        sd = math.sqrt(v)
        for i in idx:
            t[i] = (Y[i] - m) / sd if sd > 0 else 0.0
    return t


def holdout_design_points(dp_ids):
    """The design points held out to fit the coefficients: the last fifth of
    the distinct ids in ascending order (at least one)."""
    ids = sorted(set(int(d) for d in dp_ids))
    g = len(ids)
    k = g // 5 if g >= 5 else 1
    return ids[g - k:]


def rho_bin(rho, lo, hi, bins):
    """Bin of load rho among `bins` equal bins of [lo, hi], clamped at both
    ends (computed in fp32 like the factor levels themselves)."""
    u = (np.float32(rho) - np.float32(lo)) / (np.float32(hi) - np.float32(lo)) * np.float32(bins)
    k = int(math.floor(float(u)))
    return min(max(k, 0), bins - 1)


def pooled_slope_table(Y, G, dp, rho, lo, hi, bins=16):
    """Per bin of rho: the pooled within-design-point least-squares slope of Y
    on the control G, sum (Y - Ybar_dp)(G - Gbar_dp) / sum (G - Gbar_dp)^2
    over the design points in the bin (rho taken per design point), clamped
    at 0 so that a bin where the control does not help uses plain MRIP. A bin
    with no variation of G takes the slope of its nearest bin that has some
    (the lower one on a tie); with none anywhere every slope is 0."""
    Y = np.asarray(Y, np.float64)
    G = np.asarray(G, np.float64)
    dp = np.asarray(dp)
    rho = np.asarray(rho)
    sxy = [0.0] * bins
    sxx = [0.0] * bins
    for d in sorted(set(dp.tolist())):
        idx = np.flatnonzero(dp == d)
        my = sum(Y[i] for i in idx) / len(idx)
        mg = sum(G[i] for i in idx) / len(idx)
        k = rho_bin(rho[idx[0]], lo, hi, bins)
        for i in idx:
            sxy[k] += (Y[i] - my) * (G[i] - mg)
            sxx[k] += (G[i] - mg) * (G[i] - mg)
    beta = np.zeros(bins)
    for k in range(bins):
        src = None
        for dist in range(bins):
            if k - dist >= 0 and sxx[k - dist] > 0.0:
                src = k - dist
                break
            if k + dist < bins and sxx[k + dist] > 0.0:
                src = k + dist
                break
        beta[k] = 0.0 if src is None else max(0.0, sxy[src] / sxx[src])
    return beta


# ------------------------------------------------- the input control variate
# A control whose mean is known: the net input sum over the customers after
# the feature prefix, post = sum_{n >= K} (S_n - A_n). Its expectation
# follows from the variates' definition, and it draws on other customers'
# variates than the features X, so it is independent of X: for any fixed
# network g, h = g(X) z has mean 0 and Y - beta h is unbiased for E[Y]
# without a second sample.

# E[-ln u] for u = (k + 1) 2^-24, k uniform on [0, 2^24): the mean of the
# exponential variate's inversion on its 24-bit grid, in closed form
# 24 ln 2 - ln((2^24)!) / 2^24 (slightly below 1: the tail beyond u = 2^-24
# is cut).
LOG_GRID_MEAN = 24.0 * math.log(2.0) - math.lgamma(2.0 ** 24 + 1.0) / 2.0 ** 24


def variate_mean(rate):
    """Mean of the exponential variate of the given rate as drawn: the fp32
    mean m = (float)(1 / rate) times the grid mean of -ln u."""
    m = float(np.float32(1.0 / float(np.float32(rate))))
    return m * LOG_GRID_MEAN


def input_control(post, customers, K, lam, mu):
    """Standardised input control of one replication: (post / (N - K) minus
    its mean E[S] - E[A]) over its standard deviation sqrt((1/mu^2 +
    1/lambda^2) / (N - K)); 0 when no customer follows the prefix."""
    n_after = int(customers) - int(K)
    if n_after <= 0:
        return 0.0
    mean = variate_mean(mu) - variate_mean(lam)
    ms = float(np.float32(1.0 / float(np.float32(mu))))
    ma = float(np.float32(1.0 / float(np.float32(lam))))
    sd = math.sqrt((ms * ms + ma * ma) / n_after)
    return (float(post) / n_after - mean) / sd


def known_mean_control_variate(Y, H, beta, confidence=0.95):
    """mean(Y - beta H) for a control H of known mean 0, with the variance
    s^2(Y - beta H) / n and a t_{n-1} interval (beta fixed beforehand)."""
    Y, H = (np.asarray(a, np.float64) for a in (Y, H))
    n = Y.shape[0]
    m, v = _mean_var(Y - beta * H)
    tq = t_quantile(0.5 + confidence / 2.0, n - 1)
    return dict(mean=m, var=v / n, half_width=tq * math.sqrt(v / n), dof=float(n - 1))
