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


def test_controls_hand_traced():
    # (A, S) = ((1, 3), (2, 1), (0.5, 1)): T = (3, 2, 2.5); with means 1, 1
    A = np.array([1.0, 2.0, 0.5], np.float32)
    S = np.array([3.0, 1.0, 1.0], np.float32)
    # K = 0: c0 = 2 + 0 + 0, c1 = 0 + 1 - 0.5, c2 = 0*2 + 3*0 + 2*0,
    # c3 = 0*0 + 3*1 + 2*(-0.5); nothing in the prefix
    assert list(core.mm1_injected(A, S, ctl_after=0)[4]) == [2.0, 0.5, 0.0, 2.0, 0, 0, 0, 0]
    # K = 1: customer 0 (ds 2, da 0, T_{-1} = 0) moves to the prefix four
    assert list(core.mm1_injected(A, S, ctl_after=1)[4]) == [0.0, 0.5, 0.0, 2.0, 2, 0, 0, 0]
    # K = 2: the prefix holds customers 0, 1: (2 + 0, 0 + 1, 0 + 3*0, 0 + 3*1)
    assert list(core.mm1_injected(A, S, ctl_after=2)[4]) == [0.0, -0.5, 0.0, -1.0, 2, 1, 0, 3]
    assert list(core.mm1_injected(A, S, ctl_after=3)[4]) == [0.0, 0.0, 0.0, 0.0, 2, 0.5, 0, 2]
    # other means: c2 = 0*(3-0.5) + 3*(1-0.5) + 2*(1-0.5) = 2.5
    c = core.mm1_injected(A, S, ctl_after=0, es=0.5, ea=2.0)[4]
    assert list(c[:4]) == [3.5, -2.5, 2.5, -3.0]


def test_prefix_and_post_prefix_controls_partition_the_run():
    # every customer's terms go to exactly one of the two sets: for any K
    # the prefix four plus the post-prefix four are the whole run's four
    rng = np.random.default_rng(23)
    N, es, ea = 900, 0.99, 1.2
    A = rng.exponential(1.2, N).astype(np.float32)
    S = rng.exponential(1.0, N).astype(np.float32)
    whole = core.mm1_injected(A, S, ctl_after=0, es=es, ea=ea)[4][:4]
    scale = np.abs(whole).max() + N
    for K in (1, 17, 450, N - 1, N):
        c = core.mm1_injected(A, S, ctl_after=K, es=es, ea=ea)[4]
        assert np.all(np.abs(c[:4] + c[4:] - whole) <= 1e-12 * scale), K
    # K = N: the prefix four are the whole run's
    assert np.array_equal(core.mm1_injected(A, S, ctl_after=N, es=es, ea=ea)[4][4:], whole)


def test_controls_degenerate_inputs():
    rng = np.random.default_rng(22)
    N, K, es, ea = 700, 150, 1.0, 1.25
    A = rng.exponential(1.25, N).astype(np.float32)
    S = rng.exponential(1.0, N).astype(np.float32)
    # S == 0: the system is always empty, T == 0, the weighted controls vanish
    c = core.mm1_injected(A, np.zeros(N, np.float32), ctl_after=K, es=es, ea=ea)[4]
    assert c[0] == -(N - K) * es and c[2] == 0.0 and c[3] == 0.0
    assert abs(c[1] - (A[K:].astype(np.float64) - ea).sum()) < 1e-9
    # A == 0: everyone arrives at once, T_n = S_0 + ... + S_n
    _, _, T, _, c = core.mm1_injected(np.zeros(N, np.float32), S, ctl_after=K, es=es, ea=ea)
    cum = np.cumsum(S.astype(np.float64))
    prev = np.concatenate([[0.0], cum[:-1]])
    want2 = np.sum(prev[K:] * (S[K:].astype(np.float64) - es))
    want3 = np.sum(prev[K:] * (0.0 - ea))
    # the oracle's T is the fp32 running sum: each T_n within n ulps of cum
    tol = 2.0 ** -23 * N * np.sum(cum * (np.abs(S.astype(np.float64) - es) + ea))
    assert abs(c[2] - want2) <= tol and abs(c[3] - want3) <= tol
    assert np.max(np.abs(T - cum) / cum) < 2.0 ** -23 * N


def test_controls_obey_flow_balance():
    # T_n - T_{n-1} = S_n - A_n + I_n, so c0 - c1 + (N - K)(es - ea), the net
    # input after customer K-1, is T_{N-1} - T_{K-1} - sum_{n >= K} I_n (up
    # to the fp32 rounding of T)
    rng = np.random.default_rng(21)
    N, es, ea = 1500, 0.997, 1.11
    for K, lam in ((0, 0.9), (200, 0.9), (700, 0.6), (N, 0.8), (N - 1, 1.2)):
        A = rng.exponential(1 / lam, N).astype(np.float32)
        S = rng.exponential(1.0, N).astype(np.float32)
        W, I, T, _, c = core.mm1_injected(A, S, ctl_after=K, es=es, ea=ea)
        T64, I64 = T.astype(np.float64), I.astype(np.float64)
        tk = T64[K - 1] if K > 0 else 0.0
        want = T64[-1] - tk - I64[K:].sum()
        got = c[0] - c[1] + (N - K) * (es - ea)
        tol = 2.0 ** -23 * np.abs(T64).sum() + 1e-9
        assert abs(got - want) <= tol, (K, got, want)


def test_variate_mean_is_the_grid_closed_form():
    from oracle import cv
    # the C oracle's lgamma and Python's agree to a few ulps
    for rate in (0.5, 0.9, 1.0, 1.3, 3.7):
        assert abs(core.variate_mean(rate) / cv.variate_mean(rate) - 1) < 1e-14
    assert abs(core.variate_mean(1.0) - cv.LOG_GRID_MEAN) < 1e-14


def test_controls_have_mean_zero_given_the_prefix():
    # every post-prefix control, alone or times a function of the first K
    # customers' features, averages to zero over replications (the variates'
    # exact means; the weight T_{n-1} precedes customer n's draws), and so
    # does every prefix control alone
    N, K, R = 900, 300, 4000
    for lam in (0.6, 0.95):
        _, feat, ctl = core.mm1_many(11, R, N, lam, 1.0, features=K, threads=8, ctl=True)
        fs = [np.ones(R), np.tanh(feat[:, 9] / 5.0 - 1.0), feat[:, 6] - 0.5, feat[:, 4]]
        for k in range(4):
            for f in fs:
                h = f * ctl[:, k]
                assert abs(h.mean()) < 4 * h.std(ddof=1) / np.sqrt(R), (lam, k)
        for k in range(4, 8):
            h = ctl[:, k]
            assert abs(h.mean()) < 4 * h.std(ddof=1) / np.sqrt(R), (lam, k)
        # the prefix statistics are independent of the unweighted pair
        for j in range(2, 10):
            for k in (0, 1):
                assert abs(np.corrcoef(feat[:, j], ctl[:, k])[0, 1]) < 4 / np.sqrt(R)


def test_controls_explain_the_mean_wait():
    # perturbation analysis: a unit more work at load T delays the rest of
    # its busy period, about lambda T / (1 - rho) customers, so the
    # T-weighted pair carries coefficients near +-lambda / ((1 - rho) N) and
    # the four controls explain most of the variance of the mean wait
    N, K, R, lam = 20000, 1000, 1500, 0.9
    out, _, ctl = core.mm1_many(12, R, N, lam, 1.0, features=K, threads=8, ctl=True)
    Y = out[:, 0].astype(np.float64)
    Xc = ctl[:, :4] - ctl[:, :4].mean(0)
    b, *_ = np.linalg.lstsq(Xc, Y - Y.mean(), rcond=None)
    r2 = 1.0 - np.var(Y - Y.mean() - Xc @ b) / np.var(Y)
    assert r2 > 0.85, r2
    want = lam / (1 - lam) / N
    assert abs(b[2] / want - 1) < 0.25 and abs(-b[3] / want - 1) < 0.25, b * N
