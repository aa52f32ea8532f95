"""GPU parity of the forest-fire engines against the oracle: burnt counts
bit-exact, both mappings, several grid sizes, and the full 4096-replication
128x128x2000 configuration on sampled replications."""
import numpy as np
import pytest

from gpu_util import LANE0, SIMT, WAVE, announce
from oracle import core
from paper_1501_01405_amd import mrip

pytestmark = pytest.mark.gpu


def _run(mapping, grid, steps, R, p, f, seed=42, wg=256):
    ctx = mrip.Context(mrip.MRIP_FF, mrip.ff_params(grid, steps, p, f), mapping)
    if mapping == WAVE:
        ctx.set_shape(1, wg)
    ctx.run(R, seed=seed)
    return ctx, ctx.output(0).cpu().numpy()


@pytest.mark.parametrize("mapping,grid", [(WAVE, 128), (WAVE, 64), (SIMT, 128), (SIMT, 96),
                                          (SIMT, 32), (LANE0, 128)])
def test_ff_bit_exact_busy_fire(gpu, mapping, grid):
    # high growth and lightning so that every rule fires within a few steps
    announce("ff", mapping, grid)
    R, T, p, f = 10, 120, 0.05, 1e-3
    _, got = _run(mapping, grid, T, R, p, f)
    ref = core.ff_many(42, R, grid, T, p, f, threads=core.default_threads())
    assert np.all(ref > 0)
    assert np.array_equal(got, ref)


def test_ff_configuration_parameters(gpu):
    announce("ff config params short")
    R, T = 70, 400
    _, got = _run(WAVE, 128, T, R, 0.01, 1e-5, wg=1024)
    ref = core.ff_many(42, R, 128, T, 0.01, 1e-5, threads=core.default_threads())
    assert np.array_equal(got, ref)


def test_ff_full_config_sampled(gpu):
    # 4096 replications x 128^2 x 2000 steps, p = 0.01, f = 1e-5
    announce("ff full config")
    ctx, got = _run(WAVE, 128, 2000, 4096, 0.01, 1e-5)
    ids = [0, 1777, 4095]
    ref = core.ff_many(42, ids, 128, 2000, 0.01, 1e-5, threads=core.default_threads())
    assert np.array_equal(got[ids], ref)
    assert np.all((got > 1.0e5) & (got < 3.0e5))


def test_ff_simt_matches_wave(gpu):
    announce("ff simt vs wave")
    _, a = _run(WAVE, 128, 300, 200, 0.01, 1e-4)
    _, b = _run(SIMT, 128, 300, 200, 0.01, 1e-4)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("grid,p,f", [(256, 0.05, 1e-3), (224, 1.0, 0.0), (32, 0.0, 1.0),
                                      (64, 1.0, 1.0)])
def test_ff_edges(gpu, grid, p, f):
    # the largest SIMT grid, and probabilities at their ends: p = 1 grows a
    # full forest every other step, f = 1 lights every tree, p = 0 never
    # grows (burnt = 0); both mappings where the grid allows
    announce("ff edges", grid, p, f)
    R, T = 6, 40
    ref = core.ff_many(7, R, grid, T, p, f, threads=core.default_threads())
    for mapping in ((SIMT, WAVE) if grid in (64, 128) else (SIMT,)):
        _, got = _run(mapping, grid, T, R, p, f, seed=7)
        assert np.array_equal(got, ref), mapping
    if p == 0.0:
        assert np.all(ref == 0)
