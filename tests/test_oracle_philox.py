"""Pins for the oracle's Philox4x32-10 and variate transforms.

The oracle's Philox is checked against two independent engines (PyTorch's
at::Philox4_32 and rocRAND's philox4x32_10_engine) on random (key, counter)
pairs, including counters at the 2^32 word boundary. The variate transforms
are checked against their closed forms at the edge inputs.
"""
import math

import numpy as np

from oracle import core


def _random_inputs(n, seed):
    rng = np.random.default_rng(seed)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    # word boundaries: counters near 0 and 2^32 - 1
    ctr[: n // 8, 0] = np.uint32(0xFFFFFFFF) - rng.integers(0, 4, n // 8).astype(np.uint32)
    ctr[n // 8: n // 4] = 0
    key[n // 4: n // 4 + 16] = 0
    return ctr, key


def test_philox_matches_torch_engine(philox_ref):
    ctr, key = _random_inputs(20000, 1)
    ref = np.empty_like(ctr)
    philox_ref.torch_philox_batch(ctr.shape[0], ctr, key, ref)
    got = core.philox(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_matches_rocrand_engine(philox_ref):
    ctr, key = _random_inputs(20000, 2)
    ctr[:, 1] &= 0x3FFFFFFF  # rocRAND's offset counts words: keep 4*offset < 2^64
    ref = np.empty_like(ctr)
    philox_ref.rocrand_philox_batch(ctr.shape[0], ctr, key, ref)
    got = core.philox(ctr, key)
    assert np.array_equal(got, ref)


def test_philox_key_and_counter_sensitivity():
    base = core.philox([[1, 2, 3, 4]], [[5, 6]])[0]
    for i in range(4):
        c = [1, 2, 3, 4]
        c[i] ^= 1
        assert not np.array_equal(core.philox([c], [[5, 6]])[0], base)
    for i in range(2):
        k = [5, 6]
        k[i] ^= 1
        assert not np.array_equal(core.philox([[1, 2, 3, 4]], [k])[0], base)


def test_u01_edges():
    assert core.u01(0) == np.float32(2.0 ** -24)
    assert core.u01(255) == np.float32(2.0 ** -24)
    assert core.u01(256) == np.float32(2.0 ** -23)
    assert core.u01(0xFFFFFFFF) == np.float32(1.0)
    assert core.u01(0x80000000) == np.float32(0.5 + 2.0 ** -24)


def test_u01_is_exact_and_monotone():
    xs = np.arange(0, 2**32, 2**20 + 12345, dtype=np.uint64)
    us = np.array([core.u01(int(x)) for x in xs], dtype=np.float64)
    exact = ((xs >> 8) + 1).astype(np.float64) * 2.0 ** -24
    assert np.array_equal(us, exact)
    assert np.all(np.diff(us) > 0)


def test_exp_variate_closed_form():
    # u = 1 gives 0; u = 2^-24 gives 24 ln 2 / rate; u = 1/2 (+2^-24) gives ~ln 2 / rate
    assert core.exp_variate(0xFFFFFFFF, 0.9) == 0.0
    for rate in (0.5, 0.9, 1.0, 3.0):
        v = float(core.exp_variate(0, rate))
        assert abs(v - 24 * math.log(2) / rate) <= 4e-7 * v
        v = float(core.exp_variate(0x7FFFFF00, rate))
        assert abs(v - math.log(2) / rate) <= 4e-7 * v


def test_exp_variate_distribution():
    # mean and the median of many draws match the exponential law
    ctr = np.zeros((50000, 4), np.uint32)
    ctr[:, 0] = np.arange(50000)
    words = core.philox(ctr, [[42, 0]])[:, 0]
    rate = 0.9
    xs = np.array([core.exp_variate(int(w), rate) for w in words[:20000]], np.float64)
    se = (1 / rate) / math.sqrt(xs.size)
    assert abs(xs.mean() - 1 / rate) < 4 * se
    assert abs(np.median(xs) - math.log(2) / rate) < 0.03
