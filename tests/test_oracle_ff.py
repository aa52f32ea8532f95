"""Pins for the oracle's forest-fire cellular automaton (Drossel-Schwabl).

The model is not in the paper (its conclusion asks for bigger models); the
rule is the standard synchronous Drossel-Schwabl one on a torus with the
4-neighbourhood. Independent facts used: injected uniforms with closed-form
outcomes (period-3 cycle, no growth, no ignition, a diamond fire front), and
an independent whole-array implementation (numpy roll) on tiny grids.
"""
import numpy as np

from oracle import core

P, F = 0.01, 1e-5
TP, TF = core.ff_threshold(P), core.ff_threshold(F)


def test_thresholds():
    assert TP == 42949672 and TF == 42949
    assert core.ff_threshold(0.0) == 0 and core.ff_threshold(1.0) == 0xFFFFFFFF


def test_all_zero_uniforms_cycle_with_period_three():
    L, T = 8, 20
    u = np.zeros((T, L, L), np.uint32)
    final, burnt = core.ff_injected(u, P, F)
    assert burnt == L * L * ((T + 1) // 3)
    # T = 20: ignitions at steps 1, 4, ..., 19 -> burning after the last step
    assert np.all(final == 2)


def test_no_growth_when_uniforms_are_large():
    u = np.full((30, 8, 8), 0xFFFFFFFF, np.uint32)
    final, burnt = core.ff_injected(u, P, F)
    assert burnt == 0 and np.all(final == 0)


def test_growth_without_ignition():
    u = np.full((5, 8, 8), TF, np.uint32)  # TF <= u < TP
    final, burnt = core.ff_injected(u, P, F)
    assert burnt == 0 and np.all(final == 1)


def test_diamond_front_from_one_seed():
    L = 32
    init = np.ones((L, L), np.uint8)
    init[10, 12] = 2
    for k in (1, 2, 5, 9):
        u = np.full((k, L, L), TP, np.uint32)  # no growth, no lightning
        final, burnt = core.ff_injected(u, P, F, init=init)
        assert burnt == 2 * k * (k + 1)
        ys, xs = np.nonzero(final == 2)
        assert len(ys) == 4 * k
        assert np.all(np.abs(ys - 10) + np.abs(xs - 12) == k)
    u = np.full((L + 2, L, L), TP, np.uint32)
    final, burnt = core.ff_injected(u, P, F, init=init)
    assert burnt == L * L - 1 and np.all(final == 0)


def _roll_model(u, init, tp, tf):
    """Whole-array synchronous update with periodic shifts."""
    s = init.copy()
    burnt = 0
    for t in range(u.shape[0]):
        b = s == 2
        nb = np.roll(b, 1, 0) | np.roll(b, -1, 0) | np.roll(b, 1, 1) | np.roll(b, -1, 1)
        tree = s == 1
        ignite = tree & (nb | (u[t] < tf))
        grow = (s == 0) & (u[t] < tp)
        new = np.zeros_like(s)
        new[tree & ~ignite] = 1
        new[ignite] = 2
        new[grow] = 1
        burnt += int(ignite.sum())
        s = new
    return s, burnt


def test_brute_force_tiny_grids():
    rng = np.random.default_rng(0)
    for L in (4, 5, 6):
        for trial in range(20):
            T = int(rng.integers(1, 11))
            # thresholds chosen so every branch fires on a tiny grid
            p, f = 0.4, 0.1
            tp, tf = core.ff_threshold(p), core.ff_threshold(f)
            u = rng.integers(0, 2**32, size=(T, L, L), dtype=np.uint64).astype(np.uint32)
            init = rng.integers(0, 3, size=(L, L)).astype(np.uint8)
            final, burnt = core.ff_injected(u, p, f, init=init)
            ef, eb = _roll_model(u, init, tp, tf)
            assert burnt == eb
            assert np.array_equal(final, ef)


def test_stream_convention(philox_ref):
    # cell c = y*L + x at step t reads word c&3 of block (t, c>>2, rep, 3)
    seed, rep, L, T = 42, 5, 8, 6
    ctr = np.array([[t, q, rep, 3] for t in range(T) for q in range(L * L // 4)], np.uint32)
    key = np.tile(np.array([[seed, 0]], np.uint32), (ctr.shape[0], 1))
    blk = np.empty_like(ctr)
    philox_ref.torch_philox_batch(ctr.shape[0], ctr, key, blk)
    u = blk.reshape(T, L, L)
    p, f = 0.3, 0.05
    fa, ba = core.ff_injected(u, p, f)
    fb, bb = core.ff_state(seed, rep, L, T, p, f)
    assert ba == bb and np.array_equal(fa, fb)


def test_long_run_burnt_range():
    b = core.ff(42, 0, 128, 300)
    assert 0 < b < 128 * 128 * 300
