"""Pins for the oracle's lattice random walk (paper section 5.1, third model).

Independent facts used: the unbiased lattice walk has mean-square
displacement exactly t; the squared displacement has the parity of t; the
exact distribution of visited sites for short walks comes from enumerating
all 4^T paths; hand-traced paths, including one that wraps the torus. The
per-walker site counts: one walker's count is the union's; with several
walkers it is the sum of the union counts of each walker's moves run alone
(the count of a path does not depend on where it starts on the torus).
"""
import itertools
import math

import numpy as np

from oracle import core


def test_hand_traced_paths():
    # +x, +x, +y, -x, -y, -y : ends at (+1, -1), visits 6 distinct sites
    s, d = core.rw_injected(np.array([[0, 0, 2, 1, 3, 3]]))
    assert (s, d) == (2, 6)
    # back and forth on one edge: displacement 0, two sites
    s, d = core.rw_injected(np.array([[0, 1, 0, 1]]))
    assert (s, d) == (0, 2)


def test_wrap_keeps_unwrapped_displacement():
    # 64 moves in +x around a 64-torus: back at the start, displacement 64
    s, d = core.rw_injected(np.zeros((1, 64), np.uint8))
    assert (s, d) == (64 * 64, 64)
    # 70 moves in -y: 70^2, the whole column visited once
    s, d = core.rw_injected(np.full((1, 70), 3, np.uint8))
    assert (s, d) == (70 * 70, 64)


def test_start_lattice_is_distinct_and_counted():
    s, d = core.rw_injected(np.zeros((64, 0), np.uint8))
    assert (s, d) == (0, 64)
    # two walkers with one move each toward each other's region stay distinct
    s, d = core.rw_injected(np.array([[0], [1]]))
    assert (s, d) == (2, 4)


def test_direction_convention_uses_documented_bits(philox_ref):
    # move t of walker w in replication r is bits 2(t&15).. of word (t>>4)&3
    # of block (t>>6, w, r, 1) under key (seed_lo, seed_hi)
    seed = 42
    for r, w, t in [(0, 0, 0), (3, 17, 999), (31, 63, 64), (5, 2, 127), (1, 1, 16)]:
        ctr = np.array([[t >> 6, w, r, 1]], np.uint32)
        key = np.array([[seed, 0]], np.uint32)
        blk = np.empty_like(ctr)
        philox_ref.torch_philox_batch(1, ctr, key, blk)
        expect = (int(blk[0, (t >> 4) & 3]) >> (2 * (t & 15))) & 3
        assert core.rw_direction(seed, r, w, t) == expect


def test_ssd_parity_and_bounds():
    ssd, dist = core.rw_many(42, 8, walkers=64, grid=64, steps=1000)
    assert np.all(ssd % 2 == (64 * 1000) % 2)
    assert np.all((dist >= 64) & (dist <= 4096))


def test_mean_square_displacement_equals_t():
    # E[ssd] = W * T; tolerance 4 standard errors of the sample mean
    W, T, R = 64, 1000, 96
    ssd, _ = core.rw_many(7, R, walkers=W, grid=64, steps=T, threads=core.default_threads())
    se = ssd.std(ddof=1) / math.sqrt(R)
    assert abs(ssd.mean() - W * T) < 4 * se


def _exact_single_walker(T):
    """Exact P(distinct sites = k) and E[squared displacement] over 4^T paths."""
    moves = [(1, 0), (-1, 0), (0, 1), (0, -1)]
    counts = {}
    sd_sum = 0
    for path in itertools.product(range(4), repeat=T):
        x = y = 0
        seen = {(0, 0)}
        for d in path:
            x += moves[d][0]
            y += moves[d][1]
            seen.add((x, y))
        counts[len(seen)] = counts.get(len(seen), 0) + 1
        sd_sum += x * x + y * y
    total = 4 ** T
    return {k: v / total for k, v in counts.items()}, sd_sum / total


def test_exact_distribution_by_enumeration():
    T = 6
    dist, esd = _exact_single_walker(T)
    assert esd == T  # the closed form MSD = t, here exactly by enumeration
    R = 6000
    obs = {}
    sds = []
    for r in range(R):
        s, d = core.rw(11, r, walkers=1, grid=64, steps=T)
        obs[d] = obs.get(d, 0) + 1
        sds.append(s)
    # chi-square goodness of fit over the support of the exact law
    chi2 = 0.0
    for k, p in dist.items():
        e = R * p
        chi2 += (obs.get(k, 0) - e) ** 2 / e
    assert set(obs) <= set(dist)
    dof = len(dist) - 1
    assert chi2 < dof + 6 * math.sqrt(2 * dof)
    assert abs(np.mean(sds) - T) < 4 * np.std(sds) / math.sqrt(R)


def test_walker_sites_hand_traced():
    # two walkers: a 6-site path and a back-and-forth on one edge
    dirs = np.array([[0, 0, 2, 1, 3, 3], [0, 1, 0, 1, 0, 1]])
    s, d, v = core.rw_injected(dirs, walker_sites=True)
    assert v == 6 + 2
    assert d == 8  # the two walkers start on different lattice points
    # one walker: the per-walker count is the union count
    for moves in ([0, 0, 2, 1, 3, 3], [3] * 70, [0] * 64):
        s, d, v = core.rw_injected(np.array([moves]), walker_sites=True)
        assert v == d


def test_walker_sites_is_the_sum_of_single_walker_runs():
    rng = np.random.default_rng(4)
    for W, T in ((5, 37), (64, 200), (17, 1)):
        dirs = rng.integers(0, 4, (W, T)).astype(np.uint8)
        _, _, v = core.rw_injected(dirs, walker_sites=True)
        assert v == sum(core.rw_injected(dirs[w:w + 1])[1] for w in range(W))


def test_walker_sites_of_a_philox_run_agree_with_single_walkers():
    # the Philox-driven oracle walk against its own moves injected walker by walker
    seed, rep, W, T = 5, 3, 9, 150
    _, _, v = core.rw(seed, rep, W, 64, T, walker_sites=True)
    dirs = np.array([[core.rw_direction(seed, rep, w, t) for t in range(T)] for w in range(W)],
                    np.uint8)
    assert v == sum(core.rw_injected(dirs[w:w + 1])[1] for w in range(W))
    ssd, distinct, vs = core.rw_many(seed, 40, 64, 64, 1000, threads=core.default_threads(),
                                     walker_sites=True)
    assert np.all(vs >= distinct) and np.all(vs <= 64 * 1001)
