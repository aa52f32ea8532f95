"""GPU tests of the deferred statistics of split M/M/1 runs: a run's
reduction computed in the next run's kernel (one extra workgroup) gives the
same bits as the reduction launched on its own, and the fp64 statistics of
the outputs; runs pipelined several deep, switches of stream, other calls in
between, and the timing sample all keep every run's statistics right."""
import numpy as np
import pytest
import torch

from gpu_util import WAVE, announce
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu

N = 20000


def _ctx(split=4):
    c = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, N), WAVE)
    c.set_split(split)
    return c


def _reference(split, R, seed):
    """Statistics and outputs of one run reduced at once."""
    c = _ctx(split)
    c.run(R, seed=seed)
    return [c.stats(o) for o in range(3)], [c.output(o).cpu().numpy() for o in range(3)]


def _numpy_stats(x):
    x = x.astype(np.float64)
    return x.mean(), x.var(ddof=1)


@pytest.mark.parametrize("split,R", [(4, 1024), (2, 333), (4, 2)])
def test_pipelined_runs_match_runs_reduced_at_once(gpu, split, R):
    announce("deferred stats", split, R)
    seeds = [11, 12, 13, 14, 15, 16]
    refs = [_reference(split, R, sd) for sd in seeds]
    ctx = _ctx(split)
    stream = torch.cuda.current_stream().cuda_stream
    got = {}
    for i, sd in enumerate(seeds):
        ctx.run(R, seed=sd, stream=stream)
        if i >= 2:  # two runs in flight behind the newest
            got[i - 2] = [ctx.stats_back(2, o) for o in range(3)]
    for back in (1, 0):
        got[len(seeds) - 1 - back] = [ctx.stats_back(back, o) for o in range(3)]
    for i in range(len(seeds)):
        want, outs = refs[i]
        assert got[i] == want, i
        if R > 1:
            m, v = _numpy_stats(outs[0])
            assert abs(got[i][0]["mean"] - m) <= 1e-12 * abs(m)
            assert abs(got[i][0]["var"] - v) <= 1e-10 * v
    # the last run's outputs are there without asking for its statistics
    assert np.array_equal(ctx.output(0).cpu().numpy(), refs[-1][1][0])


def test_stream_switch_and_other_calls_flush_the_pending_reduction(gpu):
    announce("deferred stats, stream switch")
    R = 512
    refs = [_reference(4, R, sd) for sd in (21, 22, 23, 24)]
    ctx = _ctx(4)
    s1 = torch.cuda.Stream()
    s2 = torch.cuda.Stream()
    ctx.run(R, seed=21, stream=s1.cuda_stream)
    ctx.run(R, seed=22, stream=s2.cuda_stream)  # the first run's reduction launches on s1
    ctx.run(R, seed=23, stream=s2.cuda_stream)  # fuses the second's
    assert [ctx.stats_back(2, o) for o in range(3)] == refs[0][0]
    assert [ctx.stats_back(1, o) for o in range(3)] == refs[1][0]
    # a run of another form in between reduces the pending one first
    ctx.set_split(8)
    ctx.run(R, seed=24, stream=s2.cuda_stream)
    assert [ctx.stats_back(1, o) for o in range(3)] == refs[2][0]
    stats8 = [ctx.stats_back(0, o) for o in range(3)]
    want8 = refs[3][0]
    for o in range(3):  # eight parts instead of four: the means differ by summation order
        assert abs(stats8[o]["mean"] - want8[o]["mean"]) <= 1e-6 * abs(want8[o]["mean"])


def test_plan_after_pending_run(gpu):
    announce("deferred stats, then a plan")
    from paper_1501_01405_amd import inputs
    R = 256
    want, _ = _reference(4, R, 31)
    ctx = _ctx(4)
    ctx.run(R, seed=31)
    items = inputs.uniform_items(4, 8, 3000, [0.5, 0.6, 0.7, 0.8])
    ctx.plan_set(items)
    ctx.run_plan(seed=5)
    ps = ctx.plan_stats(0)
    assert ps["n"] == 8
    # the uniform run's statistics were computed before the plan reused its buffers
    assert [ctx.stats_back(1, o) for o in range(3)] == want


def test_timing_sample(gpu):
    announce("deferred stats, timing sample")
    ctx = _ctx(4)
    ctx.set_timing(0)
    ctx.run(64, seed=1)
    with pytest.raises(mrip.MripError):  # no timed launch yet
        ctx.last_ms()
    ctx.set_timing(3)
    for i in range(7):
        ctx.run(64, seed=2 + i)
    ms = ctx.history_ms(256)
    assert len(ms) == 3 and all(0.0 < t < 1000.0 for t in ms)  # launches 0, 3 and 6
    ctx.set_timing(1)
    ctx.run(64, seed=20)
    assert ctx.last_ms() > 0.0
    assert ctx.stats(0)["n"] == 64
