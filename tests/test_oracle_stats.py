"""Pins for the oracle's MRIP statistics (paper section 1: a confidence
interval from independent replications).

Independent facts used: scipy's Student-t quantile, numpy's mean and
unbiased variance, the closed-form t quantiles for 1 and 2 degrees of
freedom, convergence to the normal quantile, and the coverage of the
interval over many seeded experiments.
"""
import math

import numpy as np
import pytest
import scipy.stats

from oracle import stats


@pytest.mark.parametrize("dof", [1, 2, 3, 9, 31, 63, 1023, 4095])
@pytest.mark.parametrize("p", [0.9, 0.95, 0.975, 0.995])
def test_t_quantile_vs_scipy(dof, p):
    assert abs(stats.t_quantile(p, dof) - scipy.stats.t.ppf(p, dof)) < 1e-9 * (1 + abs(
        scipy.stats.t.ppf(p, dof)))


def test_t_quantile_closed_forms():
    # dof 1 (Cauchy): tan(pi (p - 1/2)); dof 2: (2p - 1) sqrt(2 / (4p(1-p)))
    for p in (0.8, 0.95, 0.975):
        assert abs(stats.t_quantile(p, 1) - math.tan(math.pi * (p - 0.5))) < 1e-9
        a = 4 * p * (1 - p)
        assert abs(stats.t_quantile(p, 2) - (2 * p - 1) * math.sqrt(2 / a)) < 1e-9
    assert abs(stats.t_quantile(0.975, 10**6) - 1.959963984540054) < 1e-5


def test_summary_vs_numpy():
    rng = np.random.default_rng(1)
    x = rng.normal(3.0, 2.0, 1000).astype(np.float32)
    s = stats.summarize(x, 0.95)
    assert abs(s["mean"] - np.mean(x.astype(np.float64))) < 1e-12
    assert abs(s["var"] - np.var(x.astype(np.float64), ddof=1)) < 1e-11
    tq = scipy.stats.t.ppf(0.975, 999)
    assert abs(s["half_width"] - tq * math.sqrt(np.var(x.astype(np.float64), ddof=1) / 1000)) \
        < 1e-11
    xi = rng.integers(0, 10**7, 64).astype(np.int32)
    si = stats.summarize(xi)
    assert si["mean"] == int(xi.astype(np.int64).sum()) / 64


def test_too_few_replications():
    with pytest.raises(ValueError):
        stats.summarize(np.array([1.0]))


def test_interval_coverage():
    # 95% intervals of 30 normal replications cover the true mean ~95% of the time
    rng = np.random.default_rng(2)
    hits = 0
    K = 2000
    tq = stats.t_quantile(0.975, 29)
    for _ in range(K):
        x = rng.normal(1.0, 1.0, 30)
        h = tq * x.std(ddof=1) / math.sqrt(30)
        hits += abs(x.mean() - 1.0) <= h
    assert abs(hits / K - 0.95) < 4 * math.sqrt(0.95 * 0.05 / K)
