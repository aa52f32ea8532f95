"""Pins for the oracle's second generator: taus88 with Random Spacing.

Independent facts used:
  * a Tausworthe component is a linear feedback shift register: its bit
    sequence obeys x_n = x_{n-k} xor x_{n-k+q} (trinomial z^k + z^q + 1), the
    state after step j holds bits x_{js} .. x_{js+31}; built here bit by bit
    from that recurrence, not from the word-level algorithm;
  * the three trinomials are primitive over GF(2) (maximal period 2^k - 1),
    checked by polynomial arithmetic modulo each trinomial;
  * Random Spacing seeds equal PyTorch's Philox words under the stated rule;
  * each model on a stream built from the bit-serial definition, and the
    models' laws (pi/4, Wq = rho/(mu - lambda), E[ssd] = W T).
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import core

COMPONENTS = [(31, 13, 12), (29, 2, 4), (28, 3, 17)]  # (k, q, s), L'Ecuyer 1996


def lfsr_words(seed_word, k, q, s, steps):
    """Words after steps 1..steps of one component, from its bit recurrence."""
    x = [(seed_word >> (31 - j)) & 1 for j in range(k)]  # x_0 .. x_{k-1}
    need = steps * s + 32
    while len(x) < need:
        n = len(x)
        x.append(x[n - k] ^ x[n - k + q])
    out = []
    for j in range(1, steps + 1):
        w = 0
        for b in x[j * s: j * s + 32]:
            w = (w << 1) | b
        out.append(w)
    return out


def reference_stream(state, n):
    """taus88 outputs 0..n-1 from a start state, via three bit-serial LFSRs."""
    parts = [lfsr_words(int(state[c]), *COMPONENTS[c], n) for c in range(3)]
    return np.array([parts[0][i] ^ parts[1][i] ^ parts[2][i] for i in range(n)], np.uint32)


def test_components_follow_their_trinomial_recurrence():
    rng = np.random.default_rng(11)
    for _ in range(8):
        st = rng.integers(16, 2**32, 3, dtype=np.uint64).astype(np.uint32)
        out, _ = core.taus88_outputs(st, 60)
        assert np.array_equal(out, reference_stream(st, 60))


def test_state_carries_over_between_calls():
    st = np.array([12345, 67890, 13579], np.uint32)
    a, st2 = core.taus88_outputs(st, 50)
    b, _ = core.taus88_outputs(st2, 50)
    c, _ = core.taus88_outputs(st, 100)
    assert np.array_equal(np.concatenate([a, b]), c)


def _polymulmod(a, b, mod, k):
    r = 0
    while b:
        if b & 1:
            r ^= a
        b >>= 1
        a <<= 1
        if a >> k & 1:
            a ^= mod
    return r


def _polypow(e, mod, k):
    """z^e modulo the degree-k polynomial mod (bit i = coefficient of z^i)."""
    result, base = 1, 2
    while e:
        if e & 1:
            result = _polymulmod(result, base, mod, k)
        base = _polymulmod(base, base, mod, k)
        e >>= 1
    return result


def _prime_factors(n):
    f, p = set(), 2
    while p * p <= n:
        while n % p == 0:
            f.add(p)
            n //= p
        p += 1
    if n > 1:
        f.add(n)
    return f


@pytest.mark.parametrize("k,q,s", COMPONENTS)
def test_trinomials_are_primitive(k, q, s):
    mod = (1 << k) | (1 << q) | 1
    order = (1 << k) - 1
    assert _polypow(order, mod, k) == 1
    for p in _prime_factors(order):
        assert _polypow(order // p, mod, k) != 1
    # the step size is coprime with the period, so the word sequence has it too
    assert math.gcd(s, order) == 1 and 0 < 2 * q < k and s <= k - q


def test_random_spacing_seeds_against_independent_philox(philox_ref):
    seed = 0x1234_5678_9ABC
    for model, tag in (("pi", 4), ("mm1", 2), ("rw", 1)):
        for dp, rep in ((0, 0), (3, 17), (0, 2**20 + 5)):
            ctr = np.array([[tag, dp, rep, 5]], np.uint32)
            key = np.array([[seed & 0xFFFFFFFF, seed >> 32]], np.uint32)
            blk = np.empty_like(ctr)
            philox_ref.torch_philox_batch(1, ctr, key, blk)
            st = core.taus88_seed(seed, model, rep, dp)
            assert list(st) == [int(v) for v in blk[0, :3]]


def test_pi_on_reference_stream():
    seed, rep, n = 9, 4, 301
    words = reference_stream(core.taus88_seed(seed, "pi", rep), 2 * n)

    def inside(wx, wy):
        u = Fraction(2 * (int(wx) >> 8) + 1, 2**25)
        v = Fraction(2 * (int(wy) >> 8) + 1, 2**25)
        return u * u + v * v <= 1

    expect = sum(inside(words[2 * i], words[2 * i + 1]) for i in range(n))
    assert core.pi_taus(seed, rep, n) == expect


def test_rw_on_reference_stream():
    seed, rep, W, T = 5, 6, 5, 37  # T not a multiple of 16: words partly used
    per = (T + 15) // 16
    words = reference_stream(core.taus88_seed(seed, "rw", rep), W * per)
    dirs = np.zeros((W, T), np.uint8)
    for w in range(W):
        for t in range(T):
            dirs[w, t] = (int(words[w * per + (t >> 4)]) >> (2 * (t & 15))) & 3
    # the injected walk on a 64 x 64 torus is pinned separately
    assert core.rw_taus(seed, rep, W, 64, T) == core.rw_injected(dirs)
    _, _, v = core.rw_taus(seed, rep, W, 64, T, walker_sites=True)
    assert v == sum(core.rw_injected(dirs[w:w + 1])[1] for w in range(W))


def test_mm1_on_reference_stream():
    seed, rep, dp, n, lam, mu = 3, 7, 2, 257, 0.8, 1.1
    words = reference_stream(core.taus88_seed(seed, "mm1", rep, dp), 2 * n)
    A = np.array([core.exp_variate(int(words[2 * i]), lam) for i in range(n)], np.float32)
    S = np.array([core.exp_variate(int(words[2 * i + 1]), mu) for i in range(n)], np.float32)
    _, _, _, ref = core.mm1_injected(A, S)
    got = core.mm1_taus(seed, rep, n, lam, mu, dp)
    assert np.array_equal(got, ref)


def test_pi_law():
    R, N = 64, 200000
    hits = core.pi_many(8, R, N, threads=core.default_threads(), rng="taus88").astype(float)
    p = math.pi / 4
    se = math.sqrt(N * p * (1 - p) / R)
    assert abs(hits.mean() - N * p) < 4 * se
    chi2 = hits.var(ddof=1) * (R - 1) / (N * p * (1 - p))
    assert (R - 1) - 5 * math.sqrt(2 * (R - 1)) < chi2 < (R - 1) + 5 * math.sqrt(2 * (R - 1))


def test_mm1_law():
    lam, mu, N, R = 0.5, 1.0, 20000, 64
    out = core.mm1_many(1, R, N, lam, mu, threads=core.default_threads(), rng="taus88")
    wq = out[:, 0].astype(np.float64)
    se = wq.std(ddof=1) / math.sqrt(R)
    # Wq = rho / (mu - lambda); the empty start biases the mean of a finite
    # run slightly low, far inside the 5-sigma band at this length
    assert abs(wq.mean() - (lam / mu) / (mu - lam)) < 5 * se
    idle = out[:, 2].astype(np.float64)
    assert abs(idle.mean() - (1 - lam / mu) / lam) < 5 * idle.std(ddof=1) / math.sqrt(R)


def test_rw_law():
    W, T, R = 64, 1000, 64
    ssd, distinct = core.rw_many(2, R, W, 64, T, threads=core.default_threads(), rng="taus88")
    ssd = ssd.astype(np.float64)
    assert abs(ssd.mean() - W * T) < 5 * ssd.std(ddof=1) / math.sqrt(R)
    assert np.all(ssd % 2 == (W * T) % 2)
    assert np.all((distinct >= 1) & (distinct <= 64 * 64))
