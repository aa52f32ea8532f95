"""GPU parity of the Monte Carlo pi engines against the oracle: hit counts
bit-exact in the three mappings (ragged point counts, several waves), the
estimate output, and the paper's 1e7-draw configuration on sampled
replications."""
import math

import numpy as np
import pytest

from gpu_util import LANE0, SIMT, WAVE, announce
from oracle import core
from oracle import stats as ostats
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu


def _run(mapping, points, R, seed=42, wg=256):
    ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(points), mapping)
    if mapping == WAVE:
        ctx.set_shape(1, wg)
    ctx.run(R, seed=seed)
    return ctx, ctx.output(0).cpu().numpy(), ctx.output(1).cpu().numpy()


@pytest.mark.parametrize("mapping", [WAVE, SIMT, LANE0])
@pytest.mark.parametrize("points,R", [(1, 3), (2, 5), (3, 70), (255, 9), (1000, 33),
                                      (100001, 12)])
def test_pi_bit_exact(gpu, mapping, points, R):
    announce("pi", mapping, points, R)
    _, hits, est = _run(mapping, points, R)
    ref = core.pi_many(42, R, points, threads=core.default_threads())
    assert np.array_equal(hits, ref)
    assert np.array_equal(est, (4.0 * ref / points).astype(np.float32))


def test_pi_paper_configuration(gpu):
    # 1e7 draws per replication (the paper's figure), 64 replications
    announce("pi 1e7")
    ctx, hits, est = _run(WAVE, 10_000_000, 64)
    ref = core.pi_many(42, [0, 63], 10_000_000, threads=2)
    assert np.array_equal(hits[[0, 63]], ref)
    s = ctx.stats(1)
    e = ostats.summarize(est)
    assert abs(s["mean"] - e["mean"]) <= 1e-12 * e["mean"]
    assert abs(s["mean"] - math.pi) < 5 * s["half_width"]


def test_pi_bench_configuration_sampled(gpu):
    # 1024 replications x 1e7 draws, the launch bench.py times (four
    # wavefronts per replication): sampled replications bit-exact
    announce("pi 1024 x 1e7")
    _, hits, _ = _run(WAVE, 10_000_000, 1024)
    ids = [0, 511, 1023]
    ref = core.pi_many(42, ids, 10_000_000, threads=3)
    assert np.array_equal(hits[ids], ref)


@pytest.mark.parametrize("R", [2049, 1500, 700, 300, 100])
@pytest.mark.parametrize("rng", ["philox", "taus88"])
def test_pi_shared_out_over_wavefronts(gpu, R, rng):
    # fewer than 4096 long replications get 2, 4, 8 or 16 wavefronts each
    # (R = 1500, 700, 300, 100); the counts are the same integer sums
    announce("pi wide", R, rng)
    N = 65537
    ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(N), WAVE)
    ctx.set_rng(mrip.MRIP_RNG_PHILOX if rng == "philox" else mrip.MRIP_RNG_TAUS88)
    ctx.run(R, seed=31)
    ref = core.pi_many(31, R, N, threads=core.default_threads(), rng=rng)
    assert np.array_equal(ctx.output(0).cpu().numpy(), ref)
