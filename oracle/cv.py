"""Control-variate estimator, oracle side -- TEST INFRASTRUCTURE ONLY.

For one design point with n replications (Y_i, F_i), where the columns of F
are controls of known mean zero, and a coefficient vector a fixed
beforehand (fitted on other replications),

    Y_cv = mean_i(Y_i - a . F_i)

is unbiased for E[Y]; its variance estimate is s^2(Y - a . F)/n with a
t_{n-1} interval. The plain estimate mean(Y) with its t_{n-1} interval is
the fallback and the reference for the control's error.

The controls are F = (h, z_pre): h = sum_k g_k(X) z_k with z the four
martingale controls of the run after its first K customers (below) and
coefficients g(X) the network predicts from the design's factor levels and
summary statistics of those K customers; z_pre the same four controls over
the first K customers. a is the per-bin-of-rho pooled least-squares fit of
Y on F on held-out design points.

Training's host steps (feature z-scores, the standardised within-design-
point target and its multipliers, the held-out design points, and the
per-bin pooled regression of Y on the controls with its nearest-bin fill)
follow, one function each.
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


def pooled_regression_table(Y, F, dp, rho, lo, hi, bins=16):
    """Per bin of rho: the pooled within-design-point least-squares
    coefficients of Y on the columns of F, i.e. the solution a_k of
    (sum_dp Fc' Fc) a = sum_dp Fc' Yc over the design points in the bin
    (rho taken per design point), with Fc, Yc centred on their design
    point's means. A column without within-design-point variation in a bin
    gets coefficient 0 there and leaves the system; a bin with no design
    point takes the coefficients of its nearest bin that has one (the lower
    one on a tie); with none anywhere every coefficient is 0. Returns
    (bins, p) fp64."""
    Y = np.asarray(Y, np.float64)
    F = np.asarray(F, np.float64)
    if F.ndim == 1:
        F = F[:, None]
    dp = np.asarray(dp)
    rho = np.asarray(rho)
    p = F.shape[1]
    A = np.zeros((bins, p, p))
    b = np.zeros((bins, p))
    seen = [False] * bins
    for d in sorted(set(dp.tolist())):
        idx = np.flatnonzero(dp == d)
        Fc = F[idx] - F[idx].mean(axis=0)
        Yc = Y[idx] - Y[idx].mean()
        k = rho_bin(rho[idx[0]], lo, hi, bins)
        A[k] += Fc.T @ Fc
        b[k] += Fc.T @ Yc
        seen[k] = True
    coef = np.zeros((bins, p))
    for k in range(bins):
        if not seen[k]:
            continue
        live = [j for j in range(p) if A[k, j, j] > 0.0]
        if live:
            coef[k, live] = np.linalg.solve(A[k][np.ix_(live, live)], b[k, live])
    out = np.zeros((bins, p))
    for k in range(bins):
        src = None
        for dist in range(bins):
            if k - dist >= 0 and seen[k - dist]:
                src = k - dist
                break
            if k + dist < bins and seen[k + dist]:
                src = k + dist
                break
        if src is not None:
            out[k] = coef[src]
    return out


# ------------------------------------------------- the martingale controls
# Four controls over the customers after the feature prefix (n >= K):
#   c0 = sum (S_n - E S), c1 = sum (A_n - E A),
#   c2 = sum T_{n-1} (S_n - E S), c3 = sum T_{n-1} (A_n - E A),
# and c4..c7, the same sums over the prefix (n < K).
# A_n and S_n are drawn independently of everything before customer n, so
# each term has mean zero given the past (martingale differences). Any
# function of the first K customers, the network's coefficients included,
# times any of c0..c3 therefore has mean zero, c4..c7 have mean zero, and
# Y - a . F stays unbiased for E[Y] with no second sample. The means are
# the variates' exact ones.

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
    """The per-sample multipliers from a replication's controls (4 or 8 of
    them) over a run of N customers: c / N, the T-weighted ones also divided
    by the service scale (float)(1 / mu), so that all are in time units per
    customer and their coefficients are plain numbers. A fixed rescaling per
    design point keeps every mean zero."""
    ctl = np.asarray(ctl, np.float64)
    ms = float(np.float32(1.0 / float(np.float32(mu))))
    scale = np.array([1.0, 1.0, 1.0 / ms, 1.0 / ms] * (ctl.shape[-1] // 4)) / float(customers)
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


def known_mean_control_variate(Y, F, coef, confidence=0.95):
    """mean(Y - F . coef) for controls F (n, or n x p) of known mean 0, with
    the variance s^2(Y - F . coef) / n and a t_{n-1} interval (coef fixed
    beforehand)."""
    Y = np.asarray(Y, np.float64)
    F = np.asarray(F, np.float64)
    if F.ndim == 1:
        F = F[:, None]
    coef = np.atleast_1d(np.asarray(coef, np.float64))
    n = Y.shape[0]
    m, v = _mean_var(Y - F @ coef)
    tq = t_quantile(0.5 + confidence / 2.0, n - 1)
    return dict(mean=m, var=v / n, half_width=tq * math.sqrt(v / n), dof=float(n - 1))
