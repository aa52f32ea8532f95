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


def test_mm1_beyond_2_32_customers(gpu):
    # the largest runs the parameters allow are < 2^33 customers: here
    # 2^32 + 4097 (customer indices past 32 bits, draw blocks up to 2^31),
    # two replications split over 8 and over 4 wavefronts. The oracle would
    # need minutes, so: the two splits agree (same per-customer values) and
    # the means match the closed forms at rho = 0.5 (Wq = 1, idle per
    # arrival (1 - rho) / lambda = 1), far inside the sampling error at
    # this length
    announce("mm1 2^32 + 4097 customers")
    N = (1 << 32) + 4097
    outs = {}
    for split in (8, 4):
        ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(0.5, 1.0, N), WAVE)
        ctx.set_split(split)
        ctx.run(2, seed=31)
        outs[split] = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    assert np.all(np.abs(outs[8] - outs[4]) <= 1e-6 * np.abs(outs[4]))
    wq, t, idle = outs[8][:, 0], outs[8][:, 1], outs[8][:, 2]
    assert np.all(np.abs(wq - 1.0) < 0.01)
    assert np.all(np.abs(t - 2.0) < 0.01)
    assert np.all(np.abs(idle - 1.0) < 0.01)
