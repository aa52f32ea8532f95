"""GPU tests at the edges of the documented sizes: the walk at the largest
walkers * steps^2 the int32 outputs allow (bit-exact against the oracle),
four million replications (sampled ids bit-exact, statistics against numpy),
and pi at the largest point count per replication (laws that hold at any
size: the oracle would need minutes there)."""
import math

import numpy as np
import pytest

from gpu_util import SIMT, WAVE, announce
from oracle import core
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("mapping", [WAVE, SIMT])
def test_rw_at_the_int32_limit(gpu, mapping):
    # 64 * 5792^2 = 2,147,024,896 < 2^31: the largest walk the outputs allow
    announce("rw limit", mapping)
    W, T, R = 64, 5792, 6
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(W, 64, T), mapping)
    ctx.run(R, seed=3)
    ssd, distinct = core.rw_many(3, R, W, 64, T, threads=core.default_threads())
    assert np.array_equal(ctx.output(0).cpu().numpy(), ssd)
    assert np.array_equal(ctx.output(1).cpu().numpy(), distinct)
    bad = mrip.rw_params(W, 64, T + 1)
    with pytest.raises(mrip.MripError):
        mrip.Context(mrip.MRIP_RW, bad, mapping)


def test_four_million_replications(gpu):
    announce("pi 2^22 replications")
    R, N = 1 << 22, 64
    ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(N), WAVE)
    ctx.run(R, seed=17)
    hits = ctx.output(0).cpu().numpy()
    ids = [0, 1, (1 << 21) + 7, R - 2, R - 1]
    assert np.array_equal(hits[ids], core.pi_many(17, ids, N))
    x = hits.astype(np.float64)
    s = ctx.stats(0)
    assert s["n"] == R
    assert abs(s["mean"] - x.mean()) <= 1e-12 * x.mean()
    assert abs(s["var"] - x.var(ddof=1)) <= 1e-9 * x.var(ddof=1)
    p = math.pi / 4
    assert abs(x.mean() - N * p) < 5 * math.sqrt(N * p * (1 - p) / R)


def test_pi_at_the_largest_point_count(gpu):
    announce("pi 2^31 - 1 points")
    N, R = (1 << 31) - 1, 4
    ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(N), WAVE)
    ctx.run(R, seed=23)
    hits = ctx.output(0).cpu().numpy().astype(np.int64)
    assert np.all((hits > 0) & (hits <= N))
    p = math.pi / 4
    sd = math.sqrt(N * p * (1 - p))
    assert np.all(np.abs(hits - N * p) < 6 * sd)
    est = ctx.output(1).cpu().numpy()
    assert np.array_equal(est, (4.0 * hits / N).astype(np.float32))
    with pytest.raises(mrip.MripError):
        mrip.Context(mrip.MRIP_PI, mrip.pi_params(N + 1), WAVE)
