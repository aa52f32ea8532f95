"""MRIP statistics, oracle side -- TEST INFRASTRUCTURE ONLY.

The paper's section 1 builds a confidence interval from independent
replications through the central limit theorem. The reading taken here is
the Student-t interval, which tends to the Gaussian one as replications
grow:

    mean = sum(x) / R,  var = sum((x - mean)^2) / (R - 1)   (two passes)
    half = t_{(1+conf)/2, R-1} * sqrt(var / R)

The t quantile is found by bisection on the t distribution function, which
is itself the plain integral of the t density (composite Simpson rule in
fp64). Slow and obviously correct; pinned against scipy in the tests.
"""
import math

import numpy as np


def t_density(x, dof):
    x = np.asarray(x, dtype=np.float64)
    logc = math.lgamma((dof + 1.0) / 2.0) - math.lgamma(dof / 2.0) - 0.5 * math.log(dof * math.pi)
    return np.exp(logc - (dof + 1.0) / 2.0 * np.log1p(x * x / dof))


def t_cdf(x, dof, intervals=20000):
    """P(T <= x) for x >= 0 as 1/2 plus the Simpson integral of the density on [0, x]."""
    if x < 0:
        return 1.0 - t_cdf(-x, dof, intervals)
    if x == 0:
        return 0.5
    n = intervals
    xs = np.linspace(0.0, x, n + 1)
    f = t_density(xs, dof)
    h = x / n
    integral = h / 3.0 * (f[0] + f[-1] + 4.0 * f[1:-1:2].sum() + 2.0 * f[2:-1:2].sum())
    return 0.5 + integral


def t_quantile(p, dof):
    """Inverse of t_cdf for 0.5 <= p < 1 by bisection to fp64 resolution."""
    if not (0.5 <= p < 1.0):
        raise ValueError("p must be in [0.5, 1)")
    if p == 0.5:
        return 0.0
    lo, hi = 0.0, 1.0
    while t_cdf(hi, dof) < p:
        lo, hi = hi, hi * 2.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid == lo or mid == hi:
            break
        if t_cdf(mid, dof) < p:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def summarize(x, confidence=0.95):
    """dict(n, mean, var, half_width, t_quantile) of per-replication outputs x."""
    x = np.asarray(x)
    n = x.shape[0]
    if n < 2:
        raise ValueError("need at least two replications")
    if np.issubdtype(x.dtype, np.integer):
        mean = float(int(np.sum(x.astype(np.int64)))) / n  # exact integer sum
    else:
        s = 0.0
        for v in x.astype(np.float64):  # sequential fp64 sum
            s += v
        mean = s / n
    ss = 0.0
    for v in x.astype(np.float64):
        d = v - mean
        ss += d * d
    var = ss / (n - 1)
    tq = t_quantile(0.5 + confidence / 2.0, n - 1)
    return dict(n=n, mean=mean, var=var, half_width=tq * math.sqrt(var / n), t_quantile=tq,
                confidence=confidence)
