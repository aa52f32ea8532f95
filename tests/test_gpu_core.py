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


@pytest.mark.parametrize("rng", ["philox", "taus88"])
@pytest.mark.parametrize("mapping", [SIMT, WAVE, LANE0])
@pytest.mark.parametrize("W,G,T,R", [(64, 64, 1000, 12), (5, 16, 37, 9), (33, 128, 300, 5)])
def test_rw_walker_sites_bit_exact(gpu, rng, mapping, W, G, T, R):
    announce("rw walker sites", rng, mapping, W, G, T, R)
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T, walker_sites=True), mapping)
    ctx.set_rng(mrip.MRIP_RNG_PHILOX if rng == "philox" else mrip.MRIP_RNG_TAUS88)
    ctx.run(R, seed=13)
    ref = core.rw_many(13, R, W, G, T, threads=core.default_threads(), rng=rng,
                       walker_sites=True)
    for o in range(3):
        assert np.array_equal(ctx.output(o).cpu().numpy(), ref[o])
    s = ctx.stats(2)
    assert abs(s["mean"] - ref[2].mean()) <= 1e-12 * ref[2].mean()


@pytest.mark.parametrize("rng", ["philox", "taus88"])
def test_rw_walker_sites_one_wave_per_replication(gpu, rng):
    # beyond 2048 replications each walker is one lane that owns its bitmap
    announce("rw walker sites, sequential form", rng)
    R, W, G, T = 2100, 64, 64, 200
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T, walker_sites=True), WAVE)
    ctx.set_rng(mrip.MRIP_RNG_PHILOX if rng == "philox" else mrip.MRIP_RNG_TAUS88)
    ctx.run(R, seed=14)
    ids = [0, 1, 1050, R - 1]
    ref = core.rw_many(14, ids, W, G, T, threads=4, rng=rng, walker_sites=True)
    got = [ctx.output(o).cpu().numpy()[ids] for o in range(3)]
    for o in range(3):
        assert np.array_equal(got[o], ref[o])


def test_rw_walker_sites_in_several_launches(gpu):
    # 64 walkers on a 128 x 128 torus keep 128 KiB of walker bitmaps per
    # replication: 9000 replications go in two launches (8192, then 808)
    announce("rw walker sites, two launches")
    R, W, G, T = 9000, 64, 128, 64
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T, walker_sites=True), WAVE)
    ctx.run(R, seed=15)
    plain = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T), WAVE)
    plain.run(R, seed=15)
    for o in range(2):
        assert np.array_equal(ctx.output(o).cpu().numpy(), plain.output(o).cpu().numpy())
    ids = [0, 8191, 8192, 8193, R - 1]
    ref = core.rw_many(15, ids, W, G, T, threads=4, walker_sites=True)
    assert np.array_equal(ctx.output(2).cpu().numpy()[ids], ref[2])


@pytest.mark.parametrize("rng", ["philox", "taus88"])
def test_rw_consecutive_runs_of_different_sizes(gpu, rng):
    # one context, runs alternating between the segmented (<= 2048
    # replications) and sequential forms, with per-walker counts
    announce("rw consecutive runs", rng)
    W, G, T = 64, 64, 300
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, G, T, walker_sites=True), WAVE)
    ctx.set_rng(mrip.MRIP_RNG_PHILOX if rng == "philox" else mrip.MRIP_RNG_TAUS88)
    for R, seed in ((1, 3), (32, 4), (2100, 5), (7, 6), (32, 7)):
        ctx.run(R, seed=seed)
        ids = sorted({0, R // 2, R - 1})
        ref = core.rw_many(seed, ids, W, G, T, threads=4, rng=rng, walker_sites=True)
        for o in range(3):
            assert np.array_equal(ctx.output(o).cpu().numpy()[ids], ref[o]), (R, o)
