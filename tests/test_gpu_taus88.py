"""GPU parity of the second generator, taus88 with Random Spacing, against the
oracle: raw outputs bit-exact at any jump distance, pi hit counts and
random-walk outputs bit-exact, M/M/1 means within 1e-5 relative, in every
mapping and WAVE shape; and the check the generator exists for: replications
on taus88 and on Philox estimate the same quantities."""
import math

import numpy as np
import pytest
import torch

from gpu_util import LANE0, SIMT, WAVE, announce, rel_err
from oracle import core
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu

TAUS = mrip.MRIP_RNG_TAUS88
TOL = 1e-5


def _dump(seed, model, dp, rep, skip, n):
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    mrip.mrip_taus88(seed, model, dp, rep, skip, n, out)
    return out.cpu().numpy().view(np.uint32)


@pytest.mark.parametrize("model,dp,rep", [(4, 0, 0), (2, 7, 123456), (1, 0, 2**31 + 5)])
@pytest.mark.parametrize("skip", [0, 1, 17, 1008, 65535, 3_000_001])
def test_outputs_bit_exact_after_jumps(gpu, model, dp, rep, skip):
    announce("taus88 dump", model, dp, rep, skip)
    seed = 0xDEADBEEF12345
    n = 300
    got = _dump(seed, model, dp, rep, skip, n)
    st = core.taus88_seed(seed, model, rep, dp)
    ref, _ = core.taus88_outputs(st, skip + n)
    assert np.array_equal(got, ref[skip:])


def test_long_jumps_compose(gpu):
    # beyond what the oracle walks in seconds: jumps of 2^40 + k agree with
    # each other (every output is reached by its own combination of tables)
    announce("taus88 long jumps")
    base = 2**40 + 12345
    a = _dump(9, 2, 0, 3, base, 512)
    b = _dump(9, 2, 0, 3, base + 200, 312)
    assert np.array_equal(a[200:], b)
    c = _dump(9, 2, 0, 3, 2**63 - 10, 10)
    assert len(set(c.tolist())) == 10


def _ctx(model, params, mapping, rpw=1, wg=256):
    ctx = mrip.Context(model, params, mapping)
    if mapping == WAVE:
        ctx.set_shape(rpw, wg)
    ctx.set_rng(TAUS)
    return ctx


@pytest.mark.parametrize("mapping", [WAVE, SIMT, LANE0])
@pytest.mark.parametrize("points,R", [(1, 3), (2, 5), (63, 9), (64, 4), (65, 70), (1000, 33),
                                      (100001, 12)])
def test_pi_bit_exact(gpu, mapping, points, R):
    announce("pi taus88", mapping, points, R)
    ctx = _ctx(mrip.MRIP_PI, mrip.pi_params(points), mapping)
    ctx.run(R, seed=11)
    ref = core.pi_many(11, R, points, threads=core.default_threads(), rng="taus88")
    assert np.array_equal(ctx.output(0).cpu().numpy(), ref)
    assert np.array_equal(ctx.output(1).cpu().numpy(), (4.0 * ref / points).astype(np.float32))


@pytest.mark.parametrize("mapping", [WAVE, SIMT, LANE0])
@pytest.mark.parametrize("walkers,grid,steps,R", [(64, 64, 1000, 20), (5, 16, 37, 9),
                                                  (1, 128, 16, 3), (33, 32, 250, 70)])
def test_rw_bit_exact(gpu, mapping, walkers, grid, steps, R):
    announce("rw taus88", mapping, walkers, grid, steps, R)
    ctx = _ctx(mrip.MRIP_RW, mrip.rw_params(walkers, grid, steps), mapping)
    ctx.run(R, seed=5)
    ssd, distinct = core.rw_many(5, R, walkers, grid, steps, threads=core.default_threads(),
                                 rng="taus88")
    assert np.array_equal(ctx.output(0).cpu().numpy(), ssd)
    assert np.array_equal(ctx.output(1).cpu().numpy(), distinct)


@pytest.mark.parametrize("mapping,rpw,wg,split", [(SIMT, 1, 64, 1), (LANE0, 1, 64, 1),
                                                  (WAVE, 1, 256, 1), (WAVE, 2, 64, 1),
                                                  (WAVE, 4, 1024, 1), (WAVE, 1, 256, 2),
                                                  (WAVE, 1, 256, 4)])
@pytest.mark.parametrize("N,R,lam,K", [(1, 3, 0.9, 0), (100, 5, 0.5, 0), (513, 33, 0.9, 0),
                                       (5000, 24, 0.9, 1000), (20000, 9, 0.95, 0),
                                       (777, 7, 0.8, 300)])
def test_mm1_matches_oracle(gpu, mapping, rpw, wg, split, N, R, lam, K):
    # the lanes of a replication take contiguous runs: N below, at and past
    # one customer per lane, and feature prefixes that end inside a run
    announce("mm1 taus88", mapping, rpw, wg, split, N, R, lam, K)
    ctx = _ctx(mrip.MRIP_MM1, mrip.mm1_params(lam, 1.0, N, K), mapping, rpw, wg)
    if split > 1:
        ctx.set_split(split)
    ctx.run(R, seed=3)
    outs = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    res = core.mm1_many(3, R, N, lam, 1.0, features=K, threads=core.default_threads(),
                        rng="taus88")
    ref = res[0] if K else res
    assert rel_err(outs, ref).max() <= TOL
    if K:
        feat = ctx.output(3).cpu().numpy()
        cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
        assert rel_err(feat[:, cont], res[1][:, cont]).max() <= TOL
        assert np.abs(feat[:, 6] - res[1][:, 6]).max() <= 2.0 / K


@pytest.mark.parametrize("split", [1, 4])
def test_mm1_wave_sampled_at_full_size(gpu, split):
    # 1024 x 1e5 (lambda 0.9) on taus88, WAVE: sampled replications
    announce("mm1 taus88 1024 x 1e5", split)
    ctx = _ctx(mrip.MRIP_MM1, mrip.mm1_params(0.9, 1.0, 100000), WAVE)
    ctx.set_split(split)
    ctx.run(1024, seed=8)
    outs = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    ids = [0, 1, 517, 1023]
    ref = core.mm1_many(8, ids, 100000, 0.9, 1.0, threads=core.default_threads(), rng="taus88")
    assert rel_err(outs[ids], ref).max() <= TOL


def _z(a, b):
    return abs(a["mean"] - b["mean"]) / math.sqrt(a["var"] / a["n"] + b["var"] / b["n"])


def test_both_generators_estimate_the_same_quantities(gpu):
    """Section 5.3's use of a second generator: a set of replications on
    another high-quality generator must agree with the first (and with the
    models' laws) within sampling error."""
    announce("taus88 vs philox")
    res = {}
    for rng in (mrip.MRIP_RNG_PHILOX, TAUS):
        out = {}
        c = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.5, 1.0, 20000), WAVE)
        c.set_rng(rng)
        c.run(1024, seed=21)
        out["wq"] = c.stats(0)
        c = mrip.Context(mrip.MRIP_PI, mrip.pi_params(1_000_000), WAVE)
        c.set_rng(rng)
        c.run(1024, seed=21)
        out["pi"] = c.stats(1)
        c = mrip.Context(mrip.MRIP_RW, mrip.rw_params(64, 64, 1000), WAVE)
        c.set_rng(rng)
        c.run(1024, seed=21)
        out["ssd"] = c.stats(0)
        res[rng] = out
    for k in ("wq", "pi", "ssd"):
        assert _z(res[mrip.MRIP_RNG_PHILOX][k], res[TAUS][k]) < 4.5, k
    for rng in res:
        pi = res[rng]["pi"]
        assert abs(pi["mean"] - math.pi) < 4.5 * math.sqrt(pi["var"] / pi["n"])
        ssd = res[rng]["ssd"]
        assert abs(ssd["mean"] - 64000) < 4.5 * math.sqrt(ssd["var"] / ssd["n"])


def test_philox_only_paths_refuse_taus88(gpu):
    announce("taus88 refusals")
    ctx = _ctx(mrip.MRIP_MM1, mrip.mm1_params(), WAVE)
    items = np.zeros(4, dtype=mrip.PLAN_ITEM_DTYPE)
    items["customers"] = 100
    items["lambda_"] = 0.5
    items["mu"] = 1.0
    with pytest.raises(mrip.MripError):
        ctx.plan_set(items)
    with pytest.raises(mrip.MripError):
        ctx.set_split(8)
    ctx.set_rng(mrip.MRIP_RNG_PHILOX)
    ctx.set_split(8)  # back on Philox, splitting over 8 is allowed again


@pytest.mark.parametrize("steps", [1024, 1025, 2000])
@pytest.mark.parametrize("R", [7, 512, 513, 2100])
def test_rw_long_walks_in_both_wave_forms(gpu, steps, R):
    # segments of 128 moves (steps > 1024), trailing segments that start at
    # or past the last move, and the one-lane-per-walker form above 512
    # replications on taus88 streams: each lane reaches its place with one
    # jump per level
    announce("rw taus88 long walks", steps, R)
    ctx = _ctx(mrip.MRIP_RW, mrip.rw_params(64, 64, steps), WAVE)
    ctx.run(R, seed=9)
    ids = sorted({0, R // 2, R - 1})
    ref = core.rw_many(9, ids, 64, 64, steps, threads=core.default_threads(), rng="taus88")
    assert np.array_equal(ctx.output(0).cpu().numpy()[ids], ref[0])
    assert np.array_equal(ctx.output(1).cpu().numpy()[ids], ref[1])
