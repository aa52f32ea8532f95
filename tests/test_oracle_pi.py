"""Pins for the oracle's Monte Carlo pi (paper section 5.1, first model).

Independent facts used: hand-checked points inside, on and outside the unit
circle (the integer test against the real inequality evaluated in exact
rational arithmetic), E[hits/N] = pi/4 and the binomial variance
N p (1 - p) of the hit count.
"""
import math
from fractions import Fraction

import numpy as np

from oracle import core


def _exact_inside(wx, wy):
    u = Fraction(2 * (wx >> 8) + 1, 2**25)
    v = Fraction(2 * (wy >> 8) + 1, 2**25)
    return u * u + v * v <= 1


def test_inside_test_against_exact_rationals():
    rng = np.random.default_rng(0)
    words = [0, 0xFF, 0x100, 0xFFFFFFFF, 0xB504F300, 0xB504F400, 0x80000000]
    words += [int(w) for w in rng.integers(0, 2**32, 200, dtype=np.uint64)]
    # points within a few grid steps of the circle
    for k in range(0, 2**24, 2**20):
        y = int(math.isqrt(2**48 - k * k)) if k * k <= 2**48 else 0
        for d in (-1, 0, 1):
            words.append(((max(0, min(2**24 - 1, y + d))) << 8))
            words.append(k << 8)
    for wx in words[:60]:
        for wy in words:
            assert core.pi_inside(wx, wy) == _exact_inside(wx, wy)


def test_corners():
    assert core.pi_inside(0, 0)
    assert not core.pi_inside(0xFFFFFFFF, 0xFFFFFFFF)
    assert core.pi_inside(0xFFFFFFFF, 0)  # u ~ 1 - 2^-25, v ~ 2^-25: inside


def test_mean_is_pi_over_four_and_variance_binomial():
    R, N = 64, 200000
    hits = core.pi_many(42, R, N, threads=core.default_threads()).astype(np.float64)
    p = math.pi / 4
    se = math.sqrt(N * p * (1 - p) / R)
    assert abs(hits.mean() - N * p) < 4 * se
    # sample variance of R binomial counts: chi-square with R-1 dof
    chi2 = hits.var(ddof=1) * (R - 1) / (N * p * (1 - p))
    assert (R - 1) - 5 * math.sqrt(2 * (R - 1)) < chi2 < (R - 1) + 5 * math.sqrt(2 * (R - 1))


def test_stream_convention(philox_ref):
    seed, rep, N = 7, 3, 101
    ctr = np.array([[k, 0, rep, 4] for k in range((N + 1) // 2)], np.uint32)
    key = np.tile(np.array([[seed, 0]], np.uint32), (ctr.shape[0], 1))
    blk = np.empty_like(ctr)
    philox_ref.torch_philox_batch(ctr.shape[0], ctr, key, blk)
    w = blk.reshape(-1)
    expect = sum(_exact_inside(int(w[2 * i]), int(w[2 * i + 1])) for i in range(N))
    assert core.pi_hits(seed, rep, N) == expect
