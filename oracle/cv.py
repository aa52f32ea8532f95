"""Control-variate estimator, oracle side -- TEST INFRASTRUCTURE ONLY.

For one design point with n replications (Y_i, h_i), where h is a control of
known mean zero fixed before the replications are drawn (up to the
replication's own prefix, see below), and a coefficient beta fixed
beforehand,

    Y_cv = mean_i(Y_i - beta h_i)

is unbiased for E[Y]; its variance estimate is s^2(Y - beta h)/n with a
t_{n-1} interval. The plain estimate mean(Y) with its t_{n-1} interval is
the fallback and the judge of the control's error.

The control is h = sum_k g_k(X) z_k: four martingale controls z of the run
after its first K customers (below), with coefficients g(X) the network
predicts from the design's factor levels and summary statistics of those K
customers.

Training's host steps (feature z-scores, the standardised within-design-
point target and its multipliers, the held-out design points, and the
per-bin pooled slope of Y on the control with its clamp at zero and
nearest-bin fill) follow, one function each.
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


# ------------------------------------------------- the martingale controls
# Four controls over the customers after the feature prefix (n >= K):
#   c0 = sum (S_n - E S), c1 = sum (A_n - E A),
#   c2 = sum T_{n-1} (S_n - E S), c3 = sum T_{n-1} (A_n - E A).
# A_n and S_n are drawn independently of everything before customer n, so
# each term has mean zero given the past (martingale differences). Any
# function of the first K customers, the network's coefficients included,
# times any c_k therefore has mean zero, and Y - h stays unbiased for E[Y]
# with no second sample. The means are the variates' exact ones.

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


def control_multipliers(ctl, customers, mu):
    """The network's per-sample multipliers z from the four controls of a
    replication of N customers: c / N, the two T-weighted controls also
    divided by the service scale (float)(1 / mu), so that all four are in
    time units per customer and the coefficients are plain numbers. A fixed
    rescaling per design point keeps every mean zero."""
    ctl = np.asarray(ctl, np.float64)
    ms = float(np.float32(1.0 / float(np.float32(mu))))
    scale = np.array([1.0, 1.0, 1.0 / ms, 1.0 / ms]) / float(customers)
    return ctl * scale


def design_point_sd(Y, dp):
    """Per row: the unbiased standard deviation of Y over the row's design
    point (the scale of the standardised training target)."""
    Y = np.asarray(Y, np.float64)
    dp = np.asarray(dp)
    sd = np.zeros(Y.shape[0])
    for d in sorted(set(dp.tolist())):
        idx = np.flatnonzero(dp == d)
        _, v = _mean_var(Y[idx])
        sd[idx] = math.sqrt(v)
    return sd


def training_multipliers(Z, sd):
    """The multipliers of the standardised target: z / sd of the row's
    design point (0 where that deviation is 0), so that sum_k g_k z_k / sd
    fits (Y - mean_dp Y) / sd and g_k stays a coefficient of Y itself."""
    Z = np.asarray(Z, np.float64)
    sd = np.asarray(sd, np.float64)
    out = np.zeros_like(Z)
    for i in range(Z.shape[0]):
        if sd[i] > 0:
            out[i] = Z[i] / sd[i]
    return out


def control_value(G, Z):
    """h = sum_k g_k z_k per replication (G: network outputs, Z: multipliers)."""
    G = np.asarray(G, np.float64)
    Z = np.asarray(Z, np.float64)
    return np.sum(G * Z, axis=1)


def known_mean_control_variate(Y, H, beta, confidence=0.95):
    """mean(Y - beta H) for a control H of known mean 0, with the variance
    s^2(Y - beta H) / n and a t_{n-1} interval (beta fixed beforehand)."""
    Y, H = (np.asarray(a, np.float64) for a in (Y, H))
    n = Y.shape[0]
    m, v = _mean_var(Y - beta * H)
    tq = t_quantile(0.5 + confidence / 2.0, n - 1)
    return dict(mean=m, var=v / n, half_width=tq * math.sqrt(v / n), dof=float(n - 1))
