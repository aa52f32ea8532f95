"""GPU tests of the boundary's caller-owned outputs and plan resume: a bound
torch buffer receives exactly the outputs (and statistics) of an unbound
run, and a plan resumed from saved outputs of its finished items gives the
outputs and per-design-point statistics of an uninterrupted run; a plan
stopped by its item limit has run exactly the items the oracle's plan runner
runs, flags them done on the device, and resumes from those flags to the
uninterrupted run; runs of one context on two streams are ordered on the
device."""
import numpy as np
import pytest
import torch

from gpu_util import SIMT, WAVE, announce
from oracle import core
from oracle import plan as oplan
from paper_1501_01405_amd import inputs, mrip

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("split", [1, 2])
def test_bound_outputs_receive_the_run(gpu, split):
    announce("bind output mm1", split)
    N, R = 20000, 300
    ref = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, N, 100), WAVE)
    ref.set_split(split)
    ref.run(R, seed=4)
    want = [ref.output(o).cpu().numpy() for o in range(4)]
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, N, 100), WAVE)
    ctx.set_split(split)
    bufs = [torch.full((R + 5,), -1.0, device="cuda") for _ in range(3)]
    feat = torch.zeros((R, 10), device="cuda")
    for o in range(3):
        ctx.bind_output(o, bufs[o])
    ctx.bind_output(3, feat)
    ctx.run(R, seed=4)
    for o in range(3):
        got = bufs[o].cpu().numpy()
        assert np.array_equal(got[:R], want[o])
        assert np.all(got[R:] == -1.0)  # nothing written past the run
        assert ctx.stats(o) == ref.stats(o)
    assert np.array_equal(feat.cpu().numpy(), want[3])
    small = torch.zeros(R - 1, device="cuda")
    ctx.bind_output(0, small)
    with pytest.raises(mrip.MripError):
        ctx.run(R, seed=4)
    ctx.bind_output(0, None)  # back to the context's own buffer
    ctx.run(R, seed=4)
    assert np.array_equal(ctx.output(0).cpu().numpy(), want[0])


def test_bound_outputs_other_models(gpu):
    announce("bind output rw / pi")
    for model, params, mapping in ((mrip.MRIP_RW, mrip.rw_params(64, 64, 200), SIMT),
                                   (mrip.MRIP_PI, mrip.pi_params(5000), WAVE)):
        ref = mrip.Context(model, params, mapping)
        ref.run(70, seed=2)
        ctx = mrip.Context(model, params, mapping)
        b = torch.zeros(70, dtype=torch.int32, device="cuda")
        ctx.bind_output(0, b)
        ctx.run(70, seed=2)
        assert np.array_equal(b.cpu().numpy(), ref.output(0).cpu().numpy())
        assert ctx.stats(0) == ref.stats(0)


def _plan():
    items = inputs.plan_table()
    keep = np.concatenate([np.arange(0, 2048, 7), [0, 1, 2]])  # a smaller plan, longest kept
    order = np.argsort(-items["customers"], kind="stable")[:8]
    sel = np.unique(np.concatenate([keep, order]))
    return items[sel]


def test_resumed_plan_equals_uninterrupted_plan(gpu):
    announce("plan resume")
    items = _plan()
    n = len(items)
    full = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), WAVE)
    full.plan_set(items)
    full.run_plan(seed=9)
    want = [full.output(o).cpu().numpy() for o in range(3)]
    dps = sorted(set(items["dp"].tolist()))
    want_stats = {dp: full.plan_stats(dp) for dp in dps}

    rng = np.random.default_rng(1)
    done = (rng.random(n) < 0.5).astype(np.uint8)
    done[np.argmax(items["customers"])] = 1  # the longest item finished before the stop
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), WAVE)
    ctx.plan_set(items)
    bufs = []
    for o in range(3):
        t = torch.full((n,), float("nan"), device="cuda")
        t[torch.from_numpy(done.astype(bool)).cuda()] = torch.from_numpy(want[o][done == 1]).cuda()
        ctx.bind_output(o, t)
        bufs.append(t)
    ctx.run_plan_resume(done, seed=9)
    for o in range(3):
        assert np.array_equal(bufs[o].cpu().numpy(), want[o])
    for dp in dps:
        assert ctx.plan_stats(dp) == want_stats[dp]
    # everything already done: only the reductions run
    ctx.run_plan_resume(np.ones(n, np.uint8), seed=9)
    for dp in dps:
        assert ctx.plan_stats(dp) == want_stats[dp]
    # nothing done: the whole plan
    ctx.run_plan_resume(np.zeros(n, np.uint8), seed=9)
    assert np.array_equal(bufs[0].cpu().numpy(), want[0])


def test_resumed_plan_splits_long_items_as_the_whole_plan_does(gpu):
    # 8192 equal long items: the whole plan holds enough work per wavefront
    # slot that its long items run unsplit by default; the 5 % left to a
    # resumed run alone would be split eight ways. The split is the plan's,
    # so the resumed items come out with the uninterrupted run's bits.
    announce("plan resume, default split of many long items")
    items = inputs.uniform_items(64, 128, 70000, np.linspace(0.5, 0.95, 64))
    n = len(items)
    full = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), WAVE)
    full.plan_set(items)
    full.run_plan(seed=4)
    want = full.output(0, n=n).cpu().numpy()
    done = (np.arange(n) % 20 != 7).astype(np.uint8)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), WAVE)
    ctx.plan_set(items)
    t = torch.full((n,), float("nan"), device="cuda")
    ctx.bind_output(0, t)
    ctx.run_plan_resume(done, seed=4)
    got = t.cpu().numpy()
    assert np.array_equal(got[done == 0], want[done == 0])


def _tuples(items):
    return [(int(r["dp"]), int(r["rep"]), int(r["customers"]), float(r["lambda_"]),
             float(r["mu"])) for r in items]


@pytest.mark.parametrize("mapping,limit,split", [(WAVE, 5, 8), (WAVE, 40, 8), (WAVE, 40, 1),
                                                 (SIMT, 7, 8)])
def test_plan_stopped_at_its_item_limit_resumes_to_the_uninterrupted_plan(gpu, mapping, limit,
                                                                          split):
    announce("plan item limit", mapping, limit, split)
    items = _plan()
    n = len(items)
    full = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), mapping)
    full.set_plan_split(split)
    full.plan_set(items)
    full.run_plan(seed=9)
    assert np.all(full.plan_done() == 1)
    want = [full.output(o).cpu().numpy() for o in range(3)]
    dps = sorted(set(items["dp"].tolist()))
    want_stats = {dp: full.plan_stats(dp) for dp in dps}

    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(), mapping)
    ctx.set_plan_split(split)
    ctx.plan_set(items)
    ctx.set_plan_limit(limit)
    ctx.run_plan(seed=9)
    done = ctx.plan_done()
    ref_out, ref_done = oplan.plan_run(9, _tuples(items), max_items=limit, threads=8)
    assert np.array_equal(done, ref_done)  # the `limit` longest items, nothing else
    run = done == 1
    got = ctx.output(0).cpu().numpy()
    assert np.array_equal(got[run], want[0][run])
    assert np.max(np.abs(got[run] - ref_out[run, 0]) / np.abs(ref_out[run, 0])) <= 1e-5
    with pytest.raises(mrip.MripError):  # a stopped run has no statistics
        ctx.plan_stats(dps[0])
    # resumed under the same limit: stops again after `limit` more items
    ctx.run_plan_resume(done, seed=9)
    done2 = ctx.plan_done()
    _, ref_done2 = oplan.plan_run(9, _tuples(items), max_items=limit, skip_done=ref_done,
                                  prev=ref_out)
    assert np.array_equal(done2, ref_done2)
    # then finished without the limit
    ctx.set_plan_limit(0)
    ctx.run_plan_resume(done2, seed=9)
    assert np.all(ctx.plan_done() == 1)
    for o in range(3):
        assert np.array_equal(ctx.output(o).cpu().numpy(), want[o])
    for dp in dps:
        assert ctx.plan_stats(dp) == want_stats[dp]
    assert n > 2 * limit


def test_runs_on_two_streams_share_scratch_in_order(gpu):
    # SIMT walk bitmaps live in the context's scratch buffer: a run enqueued
    # on a second stream waits for the first run's launch
    announce("rw simt on two streams")
    W, G, T, R = 64, 64, 1000, 4096
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T), SIMT)
    ctx.run(R, seed=1, stream=s1.cuda_stream)
    ctx.run(R, seed=2, stream=s2.cuda_stream)
    got = [ctx.output(o).cpu().numpy() for o in range(2)]
    ref = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T), SIMT)
    ref.run(R, seed=2)
    for o in range(2):
        assert np.array_equal(got[o], ref.output(o).cpu().numpy())
    ids = [0, 4095]
    ssd, distinct = core.rw_many(2, ids, W, G, T, threads=2)
    assert np.array_equal(got[0][ids], ssd)
    assert np.array_equal(got[1][ids], distinct)


def test_plans_on_two_streams_run_in_order(gpu):
    # the persistent plan kernel pops from the context's device queue: a
    # plan enqueued on a second stream, with no host synchronisation, must
    # not reset the queue under the first; and a run after a plan on a third
    # stream waits for it too
    announce("plans on two streams")
    items = inputs.plan_table(n_dp=16, reps=16, n_lo=2000, n_hi=200000, seed=8)
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
    ctx.plan_set(items)
    ref = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
    ref.plan_set(items)
    ref.run_plan(seed=2)
    want = [ref.output(o, n=len(items)).cpu().numpy() for o in range(3)]
    want_stats = {int(d): ref.plan_stats(int(d)) for d in np.unique(items["dp"])}
    for _ in range(3):
        ctx.run_plan(seed=1, stream=s1.cuda_stream)
        ctx.run_plan(seed=2, stream=s2.cuda_stream)
        got = [ctx.output(o, n=len(items)).cpu().numpy() for o in range(3)]
        for o in range(3):
            assert np.array_equal(got[o], want[o]), o
        for d, st in want_stats.items():
            assert ctx.plan_stats(d) == st
    # a plain run on a third stream right after a plan on the second
    ctx.run_plan(seed=1, stream=s2.cuda_stream)
    ctx.run(64, seed=5, stream=s3.cuda_stream)
    ref1 = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
    ref1.run(64, seed=5)
    assert np.array_equal(ctx.output(0).cpu().numpy(), ref1.output(0).cpu().numpy())


def test_autotune_leaves_the_run_shape_alone(gpu):
    # the tuner sets the plans' shape only: a split run context stays valid
    announce("autotune and the run shape")
    items = inputs.plan_table(n_dp=4, reps=8, n_lo=1000, n_hi=100000, seed=4)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 20000), WAVE)
    ctx.set_split(4)
    ctx.plan_set(items)
    ctx.set_plan_split(8, 50000)
    rpw, wg, ms = ctx.autotune(42)
    sh = ctx.shape()
    assert sh["reps_per_wave"] == 1 and sh["split"] == 4
    if sh["plan_split"] == 8:
        assert wg == 512
    elif sh["plan_split"] in (2, 4):
        assert wg == 256
    ctx.set_split(2)  # still accepted: reps_per_wave stayed 1
    ctx.run(8, seed=1)
    assert ctx.stats(0)["n"] == 8


def test_kernel_times_of_self_timed_and_marked_launches(gpu):
    # the split M/M/1 launch records its timing events from its own
    # dispatch, the other launches between stream markers; a context that
    # alternates them keeps one history, oldest first, and its statistics
    announce("kernel timing history")
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 50000), WAVE)
    expect = []
    for k, split in enumerate((4, 1, 4, 2, 1)):
        ctx.set_split(split)
        ctx.run(64 + k, seed=k)
        ms = ctx.last_ms()
        assert 0.0 < ms < 1000.0
        expect.append(ms)
        assert ctx.stats(0)["n"] == 64 + k
    hist = ctx.history_ms(16)
    assert len(hist) == 5
    assert np.allclose(hist, expect)
