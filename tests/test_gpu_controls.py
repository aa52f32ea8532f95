"""GPU parity of the M/M/1 engines' eight martingale controls (output 4:
four over the customers after the feature prefix, four over the prefix)
against the oracle, in every mapping and launch form: WAVE shapes, split
replications with their corrections, SIMT, one working lane, taus88
streams, and plans in both persistent kernels; prefixes ending inside a
chunk, a one-customer prefix, a prefix that is the whole run, rho >= 1.

Tolerance. A control is a sum of m terms, x_n = S_n - E S (or A_n - E A),
or T_{n-1} times it. The GPU draws the oracle's variates to a few ulps (the
fp32 scale, log2 against logf, the product), holds T to the scan's
rounding, centres with E S rounded to fp32 where the oracle keeps fp64, and
sums in another order (fp32 inside a lane's chunk, compensated across
chunks and lanes; fp64 in the oracle). Each moves a term by a few 1e-7 of
its size at most, so the two sums differ by less than 1e-5 of the sum of
the terms' sizes, which the test takes as m E S (m E A) for the unweighted
controls and m E S T_bar (m E A T_bar) for the weighted ones, T_bar the
mean time in system over the same customers. A control near zero by
cancellation is held to the size of its terms, not to its own value."""
import numpy as np
import pytest

from gpu_util import LANE0, SIMT, WAVE, announce
from oracle import core
from paper_1501_01405_amd import inputs, mrip

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _scales(N, K, lam, mu, out, feat):
    """Per control the size of its terms' sum (see the module docstring)."""
    es, ea = core.variate_mean(mu), core.variate_mean(lam)
    t_pre = float(feat[5]) if K > 0 else 0.0
    t_all = float(out[1])
    t_post = (N * t_all - K * t_pre) / (N - K) if N > K else 0.0
    post = (N - K) * np.array([es, ea, es * t_post, ea * t_post])
    pre = K * np.array([es, ea, es * t_pre, ea * t_pre])
    return np.concatenate([post, pre]) + 1e-6


def _check(ctl, ref_out, ref_feat, ref_ctl, N, K, lam, mu=1.0):
    assert ctl.shape == ref_ctl.shape
    for r in range(ctl.shape[0]):
        sc = _scales(N, K, lam, mu, ref_out[r], ref_feat[r])
        err = np.abs(ctl[r].astype(np.float64) - ref_ctl[r]) / sc
        assert err.max() <= TOL, (r, err, ctl[r], ref_ctl[r])


def _uniform(mapping, lam, N, K, R, rpw=1, split=1, rng=None, seed=42):
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(lam, 1.0, N, K), mapping)
    if rng is not None:
        ctx.set_rng(rng)
    if mapping == WAVE:
        ctx.set_shape(rpw, 256)
        if split > 1:
            ctx.set_split(split)
    ctx.run(R, seed=seed)
    return ctx.output(4).cpu().numpy()


CASES = [(5000, 1000, 0.9), (40000, 1000, 0.9), (777, 512, 0.8), (2048, 1, 0.9),
         (1, 1, 0.9), (1000, 1000, 0.7), (20000, 1000, 1.3), (3000, 100, 0.5)]


@pytest.mark.parametrize("N,K,lam", CASES)
@pytest.mark.parametrize("mapping,rpw,split", [(WAVE, 1, 1), (WAVE, 2, 1), (WAVE, 4, 1),
                                               (WAVE, 1, 2), (WAVE, 1, 4), (WAVE, 1, 8),
                                               (SIMT, 1, 1), (LANE0, 1, 1)])
def test_controls_match_oracle(gpu, mapping, rpw, split, N, K, lam):
    announce("controls", mapping, rpw, split, N, K, lam)
    R = 13
    ctl = _uniform(mapping, lam, N, K, R, rpw, split)
    ref, feat, rctl = core.mm1_many(42, R, N, lam, 1.0, features=K, ctl=True,
                                    threads=core.default_threads())
    _check(ctl, ref, feat, rctl, N, K, lam)


@pytest.mark.parametrize("rpw,split", [(1, 1), (4, 1), (1, 2), (1, 4)])
@pytest.mark.parametrize("N,K,lam", [(5000, 1000, 0.9), (3001, 777, 1.2)])
def test_controls_on_taus88_streams(gpu, rpw, split, N, K, lam):
    announce("controls taus88", rpw, split, N, K, lam)
    R = 9
    ctl = _uniform(WAVE, lam, N, K, R, rpw, split, rng=mrip.MRIP_RNG_TAUS88)
    ref, feat, rctl = core.mm1_many(42, R, N, lam, 1.0, features=K, ctl=True, rng="taus88",
                                    threads=core.default_threads())
    _check(ctl, ref, feat, rctl, N, K, lam)
    ctl = _uniform(SIMT, lam, N, K, R, rng=mrip.MRIP_RNG_TAUS88)
    _check(ctl, ref, feat, rctl, N, K, lam)


@pytest.mark.parametrize("plan_split,long_min", [(1, 0), (8, 20000), (2, 1)])
def test_controls_in_plans(gpu, plan_split, long_min):
    # uneven run lengths, both persistent kernels (items split over
    # wavefronts above long_min), one launch
    announce("controls plan", plan_split, long_min)
    K = 1000
    items = inputs.plan_table(n_dp=6, reps=5, n_lo=1000, n_hi=60000, seed=3)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000, K), WAVE)
    ctx.set_plan_split(plan_split, long_min)
    ctx.plan_set(items)
    ctx.run_plan(seed=42)
    ctl = ctx.output(4).cpu().numpy()
    tup = [(int(i["dp"]), int(i["rep"]), int(i["customers"]), float(i["lambda_"]),
            float(i["mu"])) for i in items]
    ref, feat, rctl = core.mm1_items(42, tup, features=K, ctl=True,
                                     threads=core.default_threads())
    for r, it in enumerate(items):
        sc = _scales(int(it["customers"]), K, float(it["lambda_"]), float(it["mu"]), ref[r],
                     feat[r])
        err = np.abs(ctl[r].astype(np.float64) - rctl[r]) / sc
        assert err.max() <= TOL, (r, err)


def test_controls_have_mean_zero_given_the_prefix(gpu):
    # a property at any size: over 8192 replications every post-prefix
    # control times a function of the prefix features, and every prefix
    # control, averages to zero within 4 standard errors
    announce("controls mean zero")
    R, N, K = 8192, 20000, 1000
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.95, 1.0, N, K), WAVE)
    ctx.set_split(4)
    ctx.run(R, seed=99)
    ctl = ctx.output(4).cpu().numpy().astype(np.float64)
    feat = ctx.output(3).cpu().numpy().astype(np.float64)
    fs = [np.ones(R), np.tanh(feat[:, 9] / 10.0 - 1.0), feat[:, 6] - 0.3, feat[:, 4]]
    for k in range(4):
        for f in fs:
            h = f * ctl[:, k]
            assert abs(h.mean()) < 4 * h.std(ddof=1) / np.sqrt(R), k
    for k in range(4, 8):
        h = ctl[:, k]
        assert abs(h.mean()) < 4 * h.std(ddof=1) / np.sqrt(R), k


def test_no_controls_without_a_prefix(gpu):
    announce("controls absent at K = 0")
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 1000, 0), WAVE)
    ctx.run(4, seed=1)
    with pytest.raises(mrip.MripError):
        ctx.output(4)
