"""A seeded sweep of parameter combinations across every model, mapping,
generator and launch shape, each run against the oracle to the usual bar
(integers bit-exact; M/M/1 means within 1e-5 relative, idle time within the
scan's rounding bound; features as in the M/M/1 tests). The cases are drawn
from fixed seeds, so the sweep is the same on every run."""
import math

import numpy as np
import pytest

from gpu_util import LANE0, SIMT, WAVE, announce, rel_err
from oracle import core
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu

MAPS = (WAVE, SIMT, LANE0)
RNGS = ("philox", "taus88")


def _rng_id(name):
    return mrip.MRIP_RNG_PHILOX if name == "philox" else mrip.MRIP_RNG_TAUS88


def _rw_cases(n=24):
    g = np.random.default_rng(101)
    out = []
    for _ in range(n):
        walkers = int(g.integers(1, 65))
        steps = int(g.integers(1, 401))
        out.append((walkers, int(g.choice([16, 32, 64, 128])), steps, int(g.integers(1, 41)),
                    MAPS[int(g.integers(0, 3))], RNGS[int(g.integers(0, 2))],
                    bool(g.integers(0, 2)), int(g.integers(0, 2**40))))
    return out


@pytest.mark.parametrize("walkers,grid,steps,R,mapping,rng,sites,seed", _rw_cases())
def test_rw_sweep(gpu, walkers, grid, steps, R, mapping, rng, sites, seed):
    announce("sweep rw", walkers, grid, steps, R, mapping, rng, sites, seed)
    ctx = mrip.Context(mrip.MRIP_RW, mrip.rw_params(walkers, grid, steps, sites), mapping)
    ctx.set_rng(_rng_id(rng))
    ctx.run(R, seed=seed)
    ref = core.rw_many(seed, R, walkers, grid, steps, threads=core.default_threads(), rng=rng,
                       walker_sites=True)
    for o in range(3 if sites else 2):
        assert np.array_equal(ctx.output(o).cpu().numpy(), ref[o]), o


def _mm1_cases(n=30):
    g = np.random.default_rng(202)
    out = []
    for _ in range(n):
        mapping = MAPS[int(g.integers(0, 3))]
        rng = RNGS[int(g.integers(0, 2))]
        N = int(g.integers(1, 6001))
        lam = float(np.float32(g.uniform(0.1, 1.5)))
        mu = float(np.float32(g.uniform(0.5, 2.0)))
        K = int(g.integers(1, N + 1)) if g.integers(0, 3) == 0 else 0
        rpw, wg, split = 1, 256, 1
        if mapping == WAVE:
            kind = int(g.integers(0, 3))
            if kind == 1:
                rpw, wg = int(g.choice([1, 2, 4])), int(g.choice([64, 256, 1024]))
            elif kind == 2:
                split = int(g.choice([2, 4] if rng == "taus88" else [2, 4, 8]))
        out.append((mapping, rng, N, lam, mu, K, rpw, wg, split, int(g.integers(1, 41)),
                    int(g.integers(0, 2**40))))
    return out


@pytest.mark.parametrize("mapping,rng,N,lam,mu,K,rpw,wg,split,R,seed", _mm1_cases())
def test_mm1_sweep(gpu, mapping, rng, N, lam, mu, K, rpw, wg, split, R, seed):
    announce("sweep mm1", mapping, rng, N, lam, mu, K, rpw, wg, split, R, seed)
    ctx = mrip.Context(mrip.MRIP_MM1, mrip.mm1_params(lam, mu, N, K), mapping)
    ctx.set_rng(_rng_id(rng))
    if mapping == WAVE:
        ctx.set_shape(rpw, wg)
        if split > 1:
            ctx.set_split(split)
    ctx.run(R, seed=seed)
    got = np.stack([ctx.output(o).cpu().numpy() for o in range(3)], axis=1)
    res = core.mm1_many(seed, R, N, lam, mu, features=K, threads=core.default_threads(), rng=rng)
    ref = res[0] if K else res
    assert rel_err(got[:, :2], ref[:, :2]).max() <= 1e-5
    # idle time I = W - (T - A): where the engine composes maps its T
    # rounds differently by a few ulp(T), and each idle customer carries
    # that into I (about 1/lambda apart), so the bound is a few ulp(T) lambda
    tol_i = np.maximum(1e-5, 4 * 2.0**-23 * ref[:, 1] * lam)
    assert np.all(rel_err(got[:, 2], ref[:, 2]) <= tol_i)
    if K:
        feat = ctx.output(3).cpu().numpy()
        cont = [0, 1, 2, 3, 4, 5, 7, 8, 9]
        tol_f = np.maximum(1e-5, 4 * 2.0**-23 * ref[:, 1:2] * lam)
        assert np.all(rel_err(feat[:, cont], res[1][:, cont]) <= tol_f)
        assert np.abs(feat[:, 6] - res[1][:, 6]).max() <= 2.0 / K


def _pi_cases(n=18):
    g = np.random.default_rng(303)
    out = []
    for _ in range(n):
        points = int(math.exp(g.uniform(0, math.log(300_000))))
        out.append((points, int(g.integers(1, 41)), MAPS[int(g.integers(0, 3))],
                    RNGS[int(g.integers(0, 2))], int(g.integers(0, 2**40))))
    return out


@pytest.mark.parametrize("points,R,mapping,rng,seed", _pi_cases())
def test_pi_sweep(gpu, points, R, mapping, rng, seed):
    announce("sweep pi", points, R, mapping, rng, seed)
    ctx = mrip.Context(mrip.MRIP_PI, mrip.pi_params(points), mapping)
    ctx.set_rng(_rng_id(rng))
    ctx.run(R, seed=seed)
    ref = core.pi_many(seed, R, points, threads=core.default_threads(), rng=rng)
    assert np.array_equal(ctx.output(0).cpu().numpy(), ref)


def _ff_cases(n=14):
    g = np.random.default_rng(404)
    out = []
    for _ in range(n):
        mapping = (WAVE, SIMT)[int(g.integers(0, 2))]
        grid = int(g.choice([64, 128])) if mapping == WAVE else int(g.choice([32, 64, 96, 160]))
        out.append((mapping, grid, int(g.integers(1, 61)), float(g.uniform(0.0, 0.2)),
                    float(10 ** g.uniform(-6, -1)), int(g.integers(1, 13)),
                    int(g.integers(0, 2**40))))
    return out


@pytest.mark.parametrize("mapping,grid,steps,p,f,R,seed", _ff_cases())
def test_ff_sweep(gpu, mapping, grid, steps, p, f, R, seed):
    announce("sweep ff", mapping, grid, steps, p, f, R, seed)
    ctx = mrip.Context(mrip.MRIP_FF, mrip.ff_params(grid, steps, p, f), mapping)
    ctx.run(R, seed=seed)
    ref = core.ff_many(seed, R, grid, steps, p, f, threads=core.default_threads())
    assert np.array_equal(ctx.output(0).cpu().numpy(), ref)
