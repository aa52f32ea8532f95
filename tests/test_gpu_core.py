"""GPU parity of Philox, the random walk and the statistics reduction against
the CPU oracle (integer outputs bit-exact; fp64 statistics to 1e-12 of the
oracle's reduction of the GPU's own per-replication values)."""
import numpy as np
import pytest
import torch

from gpu_util import LANE0, SIMT, WAVE, announce
from oracle import core
from oracle import stats as ostats
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu


def test_philox_blocks_bit_exact(gpu):
    rng = np.random.default_rng(0)
    n = 200000
    ctr = rng.integers(0, 2**32, (n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1000, 0] = 0xFFFFFFFF
    ctr[1000:2000] = 0
    for seed in (42, 0, 0x123456789ABCDEF0):
        announce("philox", seed, n)
        d_ctr = torch.from_numpy(ctr.view(np.int32)).cuda()
        out = torch.empty((n, 4), dtype=torch.int32, device="cuda")
        mrip.mrip_philox(seed, d_ctr, n, out, mrip.current_stream())
        torch.cuda.synchronize()
        got = out.cpu().numpy().view(np.uint32)
        assert np.array_equal(got, core.philox(ctr, core.seed_key(seed)))


RW_CASES = [(64, 64, 1000, 32), (1, 16, 7, 5), (37, 128, 130, 9), (64, 32, 64, 70),
            (8, 64, 1, 3)]


@pytest.mark.parametrize("mapping", [SIMT, WAVE, LANE0])
@pytest.mark.parametrize("walkers,grid,steps,reps", RW_CASES)
def test_rw_bit_exact(gpu, mapping, walkers, grid, steps, reps):
    announce("rw", mapping, walkers, grid, steps, reps)
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(walkers, grid, steps), mapping)
    ctx.run(reps, seed=42)
    ssd = ctx.output(0).cpu().numpy()
    dist = ctx.output(1).cpu().numpy()
    essd, edist = core.rw_many(42, reps, walkers, grid, steps, threads=core.default_threads())
    assert np.array_equal(ssd, essd)
    assert np.array_equal(dist, edist)
    for o, vals in ((0, ssd), (1, dist)):
        s = ctx.stats(o)
        e = ostats.summarize(vals)
        assert s["n"] == reps
        assert abs(s["mean"] - e["mean"]) <= 1e-12 * abs(e["mean"])
        assert abs(s["var"] - e["var"]) <= 1e-12 * max(abs(e["var"]), 1e-300)
        assert abs(s["half_width"] - e["half_width"]) <= 1e-9 * max(e["half_width"], 1e-300)


def test_rw_wave_workgroup_and_prefix_invariance(gpu):
    announce("rw invariance")
    ref = None
    for wg in (64, 256, 1024):
        ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(), WAVE)
        ctx.set_shape(1, wg)
        ctx.run(100, seed=9)
        got = ctx.output(0).cpu().numpy()
        if ref is None:
            ref = got
        assert np.array_equal(got, ref)
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(), WAVE)
    ctx.run(17, seed=9)
    assert np.array_equal(ctx.output(0).cpu().numpy(), ref[:17])


def test_stats_too_few(gpu):
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(steps=10), WAVE)
    ctx.run(1, seed=1)
    with pytest.raises(mrip.MripError) as e:
        ctx.stats(0)
    assert e.value.status == mrip.MRIP_E_TOO_FEW


def test_rw_many_replications_sampled(gpu):
    # 16384 replications (the top of the replication sweep), sampled ids
    announce("rw 16384")
    for mapping in (WAVE, SIMT):
        ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), mapping)
        ctx.run(16384, seed=5)
        ssd = ctx.output(0).cpu().numpy()
        dist = ctx.output(1).cpu().numpy()
        ids = [0, 1, 8191, 16383]
        essd, edist = core.rw_many(5, ids, 64, 64, 1000)
        assert np.array_equal(ssd[ids], essd) and np.array_equal(dist[ids], edist)


def test_statistics_of_earlier_runs_are_kept(gpu):
    # a pipelined loop enqueues run k + 1 before reading run k's interval
    announce("stats ring")
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 5000), WAVE)
    seeds = [5, 6, 7, 8, 9]
    for s in seeds:
        ctx.run(64, seed=s)
    for back in range(4):
        one = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 5000), WAVE)
        one.run(64, seed=seeds[-1 - back])
        for o in range(3):
            assert ctx.stats_back(back, o) == one.stats(o)
    assert ctx.stats_back(0, 1) == ctx.stats(1)
    with pytest.raises(mrip.MripError):
        ctx.stats_back(4, 0)  # only the last four runs are kept


@pytest.mark.parametrize("rng", [mrip.MRIP_RNG_PHILOX, mrip.MRIP_RNG_TAUS88])
def test_rw_segmented_and_sequential_forms_agree(gpu, rng):
    # up to 2048 replications the walk runs as a segmented scan, beyond it
    # one wave per replication walks its steps in order: same outputs
    announce("rw forms", rng)
    for W, G, T in ((64, 64, 1000), (7, 32, 77), (64, 128, 3000)):
        small = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T), WAVE)
        small.set_rng(rng)
        small.run(2048, seed=9)
        big = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T), WAVE)
        big.set_rng(rng)
        big.run(2049, seed=9)
        for o in range(2):
            assert np.array_equal(small.output(o).cpu().numpy(),
                                  big.output(o).cpu().numpy()[:2048])
