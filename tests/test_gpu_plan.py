"""The persistent plan kernels against the oracle: every item within 1e-5 of
its standalone oracle run, per-design-point statistics, item == standalone
GPU run, invariance over the autotuner's shapes, and the thread-per-
replication forms (SIMT, one working lane) of the same plans."""
import numpy as np
import pytest

from gpu_util import LANE0, SIMT, WAVE, announce, rel_err
from oracle import core
from oracle import stats as ostats
from paper_1501_01405_amd import inputs, mrip

pytestmark = pytest.mark.gpu


def _items_tuple(items):
    return [(int(i["dp"]), int(i["rep"]), int(i["customers"]), float(i["lambda_"]),
             float(i["mu"])) for i in items]


def _plan_ctx(items, rpw=1, wg=256, split=1, long_min=0):
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), WAVE)
    ctx.set_shape(rpw, wg)
    ctx.set_plan_split(split, long_min)
    ctx.plan_set(items)
    return ctx


def test_plan_matches_oracle(gpu):
    items = inputs.plan_table(n_dp=16, reps=8, n_lo=100, n_hi=20000, seed=1)
    announce("plan", len(items))
    ctx = _plan_ctx(items)
    ctx.run_plan(42)
    got = ctx.output(0, n=len(items)).cpu().numpy()
    ref = core.mm1_items(42, _items_tuple(items), threads=core.default_threads())[:, 0]
    assert rel_err(got, ref).max() <= 1e-5
    for dp in range(16):
        s = ctx.plan_stats(dp)
        e = ostats.summarize(got[items["dp"] == dp])
        assert s["n"] == 8
        assert abs(s["mean"] - e["mean"]) <= 1e-12 * e["mean"]
        assert abs(s["var"] - e["var"]) <= 1e-10 * e["var"]


@pytest.mark.parametrize("split", [1, 4, 8])
def test_plan_full_config_sampled(gpu, split):
    items = inputs.plan_table()  # 64 dp x 32 reps, N log-uniform in [1e4, 1e6]
    announce("plan full", len(items), split)
    ctx = _plan_ctx(items, split=split)
    ctx.run_plan(42)
    got = ctx.output(0, n=len(items)).cpu().numpy()
    rng = np.random.default_rng(3)
    longest = int(np.argmax(items["customers"]))
    ids = sorted(set([0, len(items) - 1, longest] + list(rng.integers(0, len(items), 13))))
    ref = core.mm1_items(42, _items_tuple(items[ids]), threads=core.default_threads())[:, 0]
    assert rel_err(got[ids], ref).max() <= 1e-5


def test_plan_split_long_items_match_oracle(gpu):
    # unstable and near-critical factor levels: long correction runs
    items = inputs.plan_table(n_dp=6, reps=4, rho_lo=0.9, rho_hi=1.2, n_lo=4000, n_hi=40000,
                              seed=9)
    announce("plan split oracle", len(items))
    ctx = _plan_ctx(items, rpw=2, wg=256, split=4, long_min=8000)
    ctx.run_plan(42)
    got = ctx.output(0, n=len(items)).cpu().numpy()
    ref = core.mm1_items(42, _items_tuple(items), threads=core.default_threads())[:, 0]
    assert rel_err(got, ref).max() <= 1e-5


@pytest.mark.parametrize("split", [2, 4, 8])
def test_plan_split_features_match_unsplit(gpu, split):
    # a plan with prefix features: the split kernel's feature form keeps the
    # prefix on the item's first part, so features match the unsplit plan's
    # bit for bit and the means to the summation order
    items = inputs.plan_table(n_dp=4, reps=8, n_lo=2000, n_hi=40000, seed=5)
    announce("plan split features", split, len(items))
    K = 1000
    outs = []
    for x, long_min in ((1, 0), (split, 1000)):
        ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 1000, K), WAVE)
        ctx.set_plan_split(x, long_min)
        ctx.plan_set(items)
        ctx.run_plan(42)
        outs.append((ctx.output(0, n=len(items)).cpu().numpy(),
                     ctx.output(3, n=len(items)).cpu().numpy()))
    assert np.array_equal(outs[0][1], outs[1][1])
    assert rel_err(outs[1][0], outs[0][0]).max() <= 1e-6


def test_plan_item_equals_standalone_run(gpu):
    announce("plan item == standalone")
    items = inputs.uniform_items(1, 40, 5000, [0.9])
    ctx = _plan_ctx(items)
    ctx.run_plan(42)
    got = ctx.output(0, n=40).cpu().numpy()
    solo = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 5000), WAVE)
    solo.run(40, seed=42)
    assert np.array_equal(got, solo.output(0).cpu().numpy())


def test_plan_shape_invariance_and_autotune(gpu):
    items = inputs.plan_table(n_dp=8, reps=8, n_lo=50, n_hi=5000, seed=2)
    announce("plan shapes")
    base = None
    for rpw in (1, 2, 4):
        for wg in (64, 256, 1024):
            ctx = _plan_ctx(items, rpw, wg)
            ctx.run_plan(42)
            got = ctx.output(0, n=len(items)).cpu().numpy()
            if base is None:
                base = got
            tol = 0.0 if rpw == 1 else 1e-6
            assert rel_err(got, base).max() <= tol
    for rpw in (1, 2, 4):
        for split in (2, 4, 8):
            # long_min 1000: most items take the split path here
            ctx = _plan_ctx(items, rpw, 256, split, long_min=1000)
            ctx.run_plan(42)
            got = ctx.output(0, n=len(items)).cpu().numpy()
            assert rel_err(got, base).max() <= 1e-6, (rpw, split)
    ctx = _plan_ctx(items, long_min=1000)
    rpw, wg, ms = ctx.autotune(42)
    assert rpw in (1, 2, 4) and wg in (64, 256, 1024) and ms > 0
    assert ctx.shape()["plan_split"] in (1, 2, 4, 8)
    ctx.run_plan(42)
    assert rel_err(ctx.output(0, n=len(items)).cpu().numpy(), base).max() <= 1e-6


@pytest.mark.parametrize("mapping", [SIMT, LANE0])
def test_plan_thread_forms_match_oracle(gpu, mapping):
    # every working lane pops its own items; K > 0 also checks the features
    items = inputs.plan_table(n_dp=8, reps=8, n_lo=1000, n_hi=20000, seed=3)
    announce("plan thread form", mapping, len(items))
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000, 500), mapping)
    ctx.plan_set(items)
    ctx.run_plan(42)
    got = np.stack([ctx.output(o, n=len(items)).cpu().numpy() for o in range(3)], axis=1)
    ref, rfeat = core.mm1_items(42, _items_tuple(items), features=500,
                                threads=core.default_threads())
    assert rel_err(got, ref).max() <= 1e-5
    feat = ctx.output(3, n=len(items)).cpu().numpy()
    cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
    assert rel_err(feat[:, cont], rfeat[:, cont]).max() <= 1e-5
    assert np.abs(feat[:, 6] - rfeat[:, 6]).max() <= 2.0 / 500
    for dp in range(8):
        st = ctx.plan_stats(dp)
        e = ostats.summarize(got[items["dp"] == dp, 0])
        assert st["n"] == 8 and abs(st["mean"] - e["mean"]) <= 1e-12 * e["mean"]


@pytest.mark.parametrize("mapping", [SIMT, LANE0])
def test_plan_thread_form_item_equals_standalone_run(gpu, mapping):
    announce("plan thread form item == standalone", mapping)
    items = inputs.uniform_items(1, 40, 5000, [0.9])
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), mapping)
    ctx.plan_set(items)
    ctx.run_plan(42)
    got = ctx.output(0, n=40).cpu().numpy()
    solo = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 5000), mapping)
    solo.run(40, seed=42)
    assert np.array_equal(got, solo.output(0).cpu().numpy())


def test_autotune_cache_round_trip(gpu, tmp_path, monkeypatch):
    # with MRIP_TUNE_CACHE set, the first tuning stores its winner and a
    # second context with a plan of the same kind installs it untimed
    items = inputs.plan_table(n_dp=8, reps=8, n_lo=1000, n_hi=50000, seed=6)
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("MRIP_TUNE_CACHE", str(path))
    announce("autotune cache")
    a = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
    a.plan_set(items)
    a.set_plan_split(8, 20000)
    first = a.autotune(42)
    lines = path.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("m2/map2/")
    b = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
    b.plan_set(items)
    b.set_plan_split(8, 20000)
    second = b.autotune(42)
    assert second[0] == first[0] and second[1] == first[1]
    assert abs(second[2] - first[2]) <= 1e-6 * first[2]  # the stored time, not a new one
    assert b.shape()["plan_split"] == a.shape()["plan_split"]
    b.run_plan(42)
    a.run_plan(42)
    assert np.array_equal(a.output(0, n=len(items)).cpu().numpy(),
                          b.output(0, n=len(items)).cpu().numpy())
