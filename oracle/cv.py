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
