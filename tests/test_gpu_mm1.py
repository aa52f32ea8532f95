"""GPU parity of the M/M/1 engines against the oracle: fp32 per-replication
means within 1e-5 relative (abs floor 1e-6), both mappings and every WAVE
launch shape, ragged run lengths, features, and the full 1024 x 1e5
configuration on sampled replications."""
import numpy as np
import pytest

from gpu_util import LANE0, SIMT, WAVE, announce, rel_err
from oracle import core
from oracle import stats as ostats
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu

TOL = 1e-5
SHAPES = [(SIMT, 1, 64), (WAVE, 1, 256), (WAVE, 2, 64), (WAVE, 4, 1024), (WAVE, 1, 1024),
          (LANE0, 1, 64)]
RUNS = [(1, 3, 0.9), (2, 5, 0.9), (31, 7, 0.5), (33, 9, 0.9), (129, 5, 0.7), (1000, 40, 0.95),
        (12345, 16, 0.9)]


def _run(mapping, rpw, wg, lam, N, R, seed=42, K=0):
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(lam, 1.0, N, K), mapping)
    if mapping == WAVE:
        ctx.set_shape(rpw, wg)
    ctx.run(R, seed=seed)
    outs = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    feat = ctx.output(3).cpu().numpy() if K else None
    return ctx, outs, feat


@pytest.mark.parametrize("mapping,rpw,wg", SHAPES)
@pytest.mark.parametrize("N,R,lam", RUNS)
def test_mm1_matches_oracle(gpu, mapping, rpw, wg, N, R, lam):
    announce("mm1", mapping, rpw, wg, N, R, lam)
    _, outs, _ = _run(mapping, rpw, wg, lam, N, R)
    ref = core.mm1_many(42, R, N, lam, 1.0, threads=core.default_threads())
    assert rel_err(outs, ref).max() <= TOL


@pytest.mark.parametrize("mapping,rpw,wg", [(SIMT, 1, 64), (WAVE, 1, 256), (WAVE, 4, 256)])
def test_mm1_features(gpu, mapping, rpw, wg):
    announce("mm1 features", mapping, rpw)
    K, N, R = 1000, 5000, 24
    _, outs, feat = _run(mapping, rpw, wg, 0.9, N, R, K=K)
    ref, rfeat = core.mm1_many(42, R, N, 0.9, 1.0, features=K, threads=core.default_threads())
    assert rel_err(outs, ref).max() <= TOL
    cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
    assert rel_err(feat[:, cont], rfeat[:, cont]).max() <= TOL
    # the fraction of zero waits counts exact zeros: a wait within rounding
    # of zero may flip, one customer at most here
    assert np.abs(feat[:, 6] - rfeat[:, 6]).max() <= 2.0 / K


@pytest.mark.parametrize("split", [1, 4])
def test_mm1_full_config_sampled(gpu, split):
    # 1024 replications x 1e5 customers, lambda 0.9, mu 1: WAVE in the
    # default shape, and split over 4 wavefronts per replication (the launch
    # bench.py times: the split kernel's feature-free form)
    announce("mm1 full config", split)
    if split == 1:
        ctx, outs, _ = _run(WAVE, 1, 256, 0.9, 100000, 1024)
    else:
        ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
        ctx.set_split(split)
        ctx.run(1024, seed=42)
        outs = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    rng = np.random.default_rng(5)
    ids = sorted(set([0, 1, 511, 1023] + list(rng.integers(0, 1024, 28))))
    ref = core.mm1_many(42, ids, 100000, 0.9, 1.0, threads=core.default_threads())
    assert rel_err(outs[ids], ref).max() <= TOL
    s = ctx.stats(0)
    e = ostats.summarize(outs[:, 0])
    assert abs(s["mean"] - e["mean"]) <= 1e-12 * e["mean"]
    assert abs(s["var"] - e["var"]) <= 1e-10 * e["var"]
    # the closed form Wq = 9 (start-empty transient ~ -0.01)
    assert abs(s["mean"] - 9.0) < 4 * s["half_width"] / 1.96 + 0.03


def test_mm1_simt_full_config_sampled(gpu):
    announce("mm1 simt full config")
    _, outs, _ = _run(SIMT, 1, 64, 0.9, 100000, 1024)
    ids = [0, 63, 64, 700, 1023]
    ref = core.mm1_many(42, ids, 100000, 0.9, 1.0, threads=core.default_threads())
    assert rel_err(outs[ids], ref).max() <= TOL


def test_mm1_shape_invariance(gpu):
    announce("mm1 shape invariance")
    base = _run(WAVE, 1, 64, 0.9, 4321, 37)[1]
    for rpw, wg in ((1, 256), (1, 1024)):
        assert np.array_equal(_run(WAVE, rpw, wg, 0.9, 4321, 37)[1], base)
    for rpw in (2, 4):
        for wg in (64, 256, 1024):
            got = _run(WAVE, rpw, wg, 0.9, 4321, 37)[1]
            # same per-customer values; only the summation order differs
            assert rel_err(got, base).max() <= 1e-6


def test_mm1_lane0_equals_simt(gpu):
    # the paper's one-working-lane form runs the SIMT code on one lane per wave
    announce("mm1 lane0 vs simt")
    a = _run(SIMT, 1, 64, 0.9, 2345, 70)[1]
    b = _run(LANE0, 1, 64, 0.9, 2345, 70)[1]
    assert np.array_equal(a, b)


def test_mm1_prefix_and_repeat(gpu):
    announce("mm1 prefix/repeat")
    a = _run(WAVE, 1, 256, 0.9, 3000, 100)[1]
    b = _run(WAVE, 1, 256, 0.9, 3000, 100)[1]
    c = _run(WAVE, 1, 256, 0.9, 3000, 13)[1]
    assert np.array_equal(a, b)
    assert np.array_equal(a[:13], c)


@pytest.mark.parametrize("split", [2, 4, 8])
@pytest.mark.parametrize("N,R,lam", [(100000, 40, 0.9), (20000, 33, 0.95), (3000, 9, 0.5),
                                     (1500, 5, 0.9), (50000, 6, 1.3), (40000, 17, 1.0)])
def test_mm1_split_matches_unsplit_and_oracle(gpu, split, N, R, lam):
    # lambda = 1.3: an unstable queue never empties, so every part's assumed
    # start is wrong and the in-order correction re-runs whole parts;
    # lambda = 1: some parts meet their trajectory and some do not; short
    # runs fall back to one part
    announce("mm1 split", split, N, R, lam)
    base = _run(WAVE, 1, 256, lam, N, R)[1]
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(lam, 1.0, N), WAVE)
    ctx.set_split(split)
    ctx.run(R, seed=42)
    got = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    assert rel_err(got, base).max() <= 1e-6
    ref = core.mm1_many(42, R, N, lam, 1.0, threads=core.default_threads())
    assert rel_err(got[:, :2], ref[:, :2]).max() <= TOL
    # idle time I = max(0, A - T): the scan rounds T differently from the
    # sequential recursion by a few ulp(T), and each idle customer carries
    # that into I (about E[A] = 1/lambda), so the relative error of mean I
    # is bounded by a few ulp(T) * lambda, above 1e-5 once T ~ 100 (rho = 1)
    tol_i = np.maximum(TOL, 4 * 2.0**-23 * ref[:, 1] * lam)
    assert np.all(rel_err(got[:, 2], ref[:, 2]) <= tol_i)


def test_mm1_split_features(gpu):
    announce("mm1 split features")
    K, N, R = 1000, 40000, 12
    base = _run(WAVE, 1, 256, 0.9, N, R, K=K)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, N, K), WAVE)
    ctx.set_split(2)
    ctx.run(R, seed=42)
    assert np.array_equal(ctx.output(3).cpu().numpy(), base[2])
    assert rel_err(ctx.output(0).cpu().numpy(), base[1][:, 0]).max() <= 1e-6


@pytest.mark.parametrize("split", [2, 4, 8])
@pytest.mark.parametrize("N,lam", [(100000, 0.9), (20000, 1.3), (3000, 0.5)])
def test_mm1_split_feature_free_form(gpu, split, N, lam):
    # a run without a feature prefix takes the split kernel's feature-free
    # form; with a short prefix (one chunk, so the parts are the same) the
    # feature form runs the same customers in the same order: the means
    # must agree bit for bit
    announce("mm1 split feature-free form", split, N, lam)
    R = 24
    outs = []
    for K in (0, 100):
        ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(lam, 1.0, N, K), WAVE)
        ctx.set_split(split)
        ctx.run(R, seed=7)
        outs.append(np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1))
    assert np.array_equal(outs[0], outs[1])


@pytest.mark.parametrize("mapping,rpw", [(WAVE, 1), (WAVE, 4), (SIMT, 1)])
@pytest.mark.parametrize("N,K", [(1, 1), (5000, 5000), (777, 512), (2048, 1)])
def test_mm1_feature_edges(gpu, mapping, rpw, N, K):
    # prefix = whole run, a one-customer run, prefixes ending inside a chunk
    announce("mm1 feature edges", mapping, rpw, N, K)
    R = 9
    _, outs, feat = _run(mapping, rpw, 256, 0.8, N, R, K=K)
    ref, rfeat = core.mm1_many(42, R, N, 0.8, 1.0, features=K, threads=core.default_threads())
    assert rel_err(outs, ref).max() <= TOL
    cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
    assert rel_err(feat[:, cont], rfeat[:, cont]).max() <= TOL
    assert np.abs(feat[:, 6] - rfeat[:, 6]).max() <= 2.0 / K


@pytest.mark.parametrize("split", [2, 8])
def test_split_statistics_across_runs(gpu, split):
    # statistics written straight to pinned host memory: consecutive runs of
    # different sizes on one context each report their own replications
    announce("mm1 split stats across runs", split)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.8, 1.0, 20000), WAVE)
    ctx.set_split(split)
    for R in (1024, 37, 2, 1024):
        ctx.run(R, seed=R)
        for o in range(3):
            x = ctx.output(o).cpu().numpy().astype(np.float64)
            st = ctx.stats(o)
            assert st["n"] == R
            assert abs(st["mean"] - x.mean()) <= 1e-12 * abs(x.mean())
            assert abs(st["var"] - x.var(ddof=1)) <= 1e-9 * x.var(ddof=1)
