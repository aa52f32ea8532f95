"""Pins for the oracle's M/M/1 queue (paper section 5.1, second model).

Independent facts used: a hand-traced three-customer case; an absolute-clock
event simulation in fp64 (arrival and departure epochs, a different
formulation from Lindley's recursion); the degenerate inputs S = 0 and
A = 0; the flow-balance identity; the M/M/1 closed forms
Wq = rho/(mu - lambda), W = 1/(mu - lambda) and mean idle (1 - rho)/lambda.
"""
import math

import numpy as np

from oracle import core


def test_hand_traced_three_customers():
    W, I, T, out = core.mm1_injected([1.0, 2.0, 0.5], [3.0, 1.0, 1.0])
    assert W.tolist() == [0.0, 1.0, 1.5]
    assert I.tolist() == [1.0, 0.0, 0.0]
    assert T.tolist() == [3.0, 2.0, 2.5]
    assert out[0] == np.float32(2.5 / 3)
    assert out[1] == np.float32(7.5 / 3)
    assert out[2] == np.float32(1.0 / 3)


def _event_clock(A, S):
    """Absolute-time FIFO single server: arrival epochs and departure epochs."""
    arrival = 0.0
    last_departure = 0.0
    W, I = [], []
    for a, s in zip(A.astype(np.float64), S.astype(np.float64)):
        arrival += a
        start = max(arrival, last_departure)
        W.append(start - arrival)
        I.append(max(0.0, arrival - last_departure))
        last_departure = start + s
    return np.array(W), np.array(I), last_departure


def test_matches_absolute_clock_simulation():
    rng = np.random.default_rng(3)
    for rho in (0.5, 0.9, 1.2):
        A = rng.exponential(1 / rho, 1000).astype(np.float32)
        S = rng.exponential(1.0, 1000).astype(np.float32)
        W, I, T, _ = core.mm1_injected(A, S)
        We, Ie, dep = _event_clock(A, S)
        assert np.allclose(W, We, rtol=0, atol=2e-4 * (1 + We.max()))
        assert np.allclose(I, Ie, rtol=0, atol=2e-4 * (1 + We.max()))


def test_flow_balance_identity():
    rng = np.random.default_rng(4)
    A = rng.exponential(1 / 0.9, 5000).astype(np.float32)
    S = rng.exponential(1.0, 5000).astype(np.float32)
    W, I, T, _ = core.mm1_injected(A, S)
    busy_plus_idle = I.astype(np.float64).sum() + S.astype(np.float64).sum()
    last_departure = A.astype(np.float64).sum() + float(W[-1]) + float(S[-1])
    assert abs(busy_plus_idle - last_departure) < 1e-6 * last_departure + 1e-2


def test_degenerate_inputs():
    rng = np.random.default_rng(5)
    A = rng.exponential(1.0, 200).astype(np.float32)
    S = rng.exponential(1.0, 200).astype(np.float32)
    W, I, T, _ = core.mm1_injected(A, np.zeros(200, np.float32))
    assert np.all(W == 0) and np.array_equal(I, A)
    W, I, T, _ = core.mm1_injected(np.zeros(200, np.float32), S)
    expect = np.concatenate([[0.0], np.cumsum(S.astype(np.float64))[:-1]])
    assert np.allclose(W, expect, rtol=1e-5, atol=1e-5)
    assert np.all(I == 0)


def test_stream_convention(philox_ref):
    # customer n draws from block (n>>1, dp, rep, 2): A_n = word 2(n&1), S_n = word 2(n&1)+1
    seed, dp, rep, N, lam, mu = 42, 3, 7, 257, 0.8, 1.0
    ctr = np.array([[k, dp, rep, 2] for k in range((N + 1) // 2)], np.uint32)
    key = np.tile(np.array([[seed, 0]], np.uint32), (ctr.shape[0], 1))
    blk = np.empty_like(ctr)
    philox_ref.torch_philox_batch(ctr.shape[0], ctr, key, blk)
    words = blk.reshape(-1)
    A = np.array([core.exp_variate(int(words[2 * n]), lam) for n in range(N)], np.float32)
    S = np.array([core.exp_variate(int(words[2 * n + 1]), mu) for n in range(N)], np.float32)
    W, I, T, out = core.mm1_injected(A, S)
    got, feat = core.mm1(seed, rep, N, lam, mu, dp=dp, features=100)
    assert np.array_equal(got, out)
    K = 100
    expect = [lam / mu, mu, A[:K].astype(np.float64).mean(), S[:K].astype(np.float64).mean(),
              W[:K].astype(np.float64).mean(), T[:K].astype(np.float64).mean(),
              np.mean(W[:K] == 0), W[:K].max(), I[:K].astype(np.float64).mean(), T[K - 1]]
    assert np.array_equal(feat, np.array(expect, np.float32))


def test_closed_form_waiting_time():
    # lambda = 0.9, mu = 1: Wq = 9, W = 10, idle per customer (1-rho)/lambda = 1/9.
    # Starting empty biases the mean down by ~0.01 at N = 1e5 (transient).
    R, N = 96, 100000
    out = core.mm1_many(42, R, N, 0.9, 1.0, threads=core.default_threads()).astype(np.float64)
    m, se = out.mean(axis=0), out.std(axis=0, ddof=1) / math.sqrt(R)
    assert abs(m[0] - 9.0) < 4 * se[0] + 0.03
    assert abs(m[1] - 10.0) < 4 * se[1] + 0.03
    assert abs(m[2] - 1 / 9) < 4 * se[2] + 1e-3


def test_closed_form_light_load():
    # rho = 0.5: Wq = 1, negligible transient
    R, N = 64, 50000
    out = core.mm1_many(9, R, N, 0.5, 1.0, threads=core.default_threads()).astype(np.float64)
    m, se = out[:, 0].mean(), out[:, 0].std(ddof=1) / math.sqrt(R)
    assert abs(m - 1.0) < 4 * se + 1e-3


def test_post_prefix_net_input_obeys_flow_balance():
    # T_n - T_{n-1} = S_n - A_n + I_n, so the net input after customer K-1 is
    # T_{N-1} - T_{K-1} - sum_{n >= K} I_n (up to the fp32 rounding of T)
    rng = np.random.default_rng(21)
    N = 1500
    for K, lam in ((0, 0.9), (200, 0.9), (700, 0.6), (N, 0.8), (N - 1, 1.2)):
        A = rng.exponential(1 / lam, N).astype(np.float32)
        S = rng.exponential(1.0, N).astype(np.float32)
        W, I, T, _, post = core.mm1_injected(A, S, post_after=K)
        T64, I64 = T.astype(np.float64), I.astype(np.float64)
        tk = T64[K - 1] if K > 0 else 0.0
        want = T64[-1] - tk - I64[K:].sum()
        tol = 2.0 ** -23 * np.abs(T64).sum() + 1e-9
        assert abs(post - want) <= tol, (K, post, want)


def test_post_prefix_net_input_has_the_variates_mean():
    # E[post] = (N - K)(E[S] - E[A]) with the variates' exact means
    from oracle import cv
    N, K, lam, mu, R = 1200, 200, 0.8, 1.0, 3000
    _, _, post = core.mm1_many(7, R, N, lam, mu, features=K, threads=8, post=True)
    per = post / (N - K)
    mean = cv.variate_mean(mu) - cv.variate_mean(lam)
    se = np.sqrt((1.0 + 1.0 / lam ** 2) / (N - K) / R)
    assert abs(per.mean() - mean) < 4 * se
    assert abs(per.var(ddof=1) / ((1.0 + 1.0 / lam ** 2) / (N - K)) - 1) < 0.1
