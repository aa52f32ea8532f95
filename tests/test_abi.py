"""The C-ABI library loads, exports every symbol include/mrip.h declares,
and its host-side logic (argument checks, Student-t quantile) behaves; no
GPU needed (no compute calls)."""
import ctypes as C
import os
import re

import pytest
import scipy.stats

from paper_1501_01405_amd import mrip

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mrip.h")).read()
    return sorted(set(re.findall(r"^MRIP_API [^;]*?\b(mrip_\w+)\s*\(", src, flags=re.M)))


def test_library_loads_and_exports_every_declared_symbol():
    L = mrip.load()
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(mrip.EXPORTED) == names


def test_version_and_status_strings():
    L = mrip.load()
    assert b"gfx950" in L.mrip_version()
    assert L.mrip_status_string(mrip.MRIP_E_TOO_FEW) == b"fewer than two replications"


@pytest.mark.parametrize("dof", [1, 2, 5, 31, 1023, 2047, 100000])
@pytest.mark.parametrize("p", [0.95, 0.975, 0.995])
def test_t_quantile_matches_scipy(dof, p):
    # scipy's own ppf is accurate to ~1e-10 relative (it is off by 2e-11 at
    # dof 1, where the closed form is known); the closed forms are pinned below
    q = mrip.mrip_t_quantile(p, dof)
    assert abs(q - scipy.stats.t.ppf(p, dof)) <= 1e-9 * max(1.0, q)


def test_t_quantile_closed_forms():
    import math
    for p in (0.8, 0.95, 0.975, 0.995):
        assert abs(mrip.mrip_t_quantile(p, 1) - math.tan(math.pi * (p - 0.5))) < 1e-13 * 100
        a = 4 * p * (1 - p)
        assert abs(mrip.mrip_t_quantile(p, 2) - (2 * p - 1) * math.sqrt(2 / a)) < 1e-13 * 10
    assert mrip.mrip_t_quantile(0.5, 7) == 0.0
    assert math.isnan(mrip.mrip_t_quantile(0.4, 7))


def _create(model, params, mapping=mrip.MRIP_MAP_AUTO):
    ctx = mrip.ctx_t()
    rc = mrip.load().mrip_create(C.byref(ctx), model, C.byref(params), mapping)
    if rc == mrip.MRIP_OK:
        mrip.load().mrip_destroy(ctx)
    return rc


def test_parameter_validation():
    ok = mrip.MRIP_OK
    bad = mrip.MRIP_E_INVAL
    assert _create(mrip.MRIP_RW, mrip.rw_params()) == ok
    assert _create(mrip.MRIP_RW, mrip.rw_params(walkers=65)) == bad
    assert _create(mrip.MRIP_RW, mrip.rw_params(grid=48)) == bad
    assert _create(mrip.MRIP_RW, mrip.rw_params(steps=10**5)) == bad
    assert _create(mrip.MRIP_RW, mrip.rw_params(walker_sites=True)) == ok
    p = mrip.rw_params()
    p.walker_sites = 2
    assert _create(mrip.MRIP_RW, p) == bad
    assert _create(mrip.MRIP_MM1, mrip.mm1_params()) == ok
    assert _create(mrip.MRIP_MM1, mrip.mm1_params(lam=0.0)) == bad
    assert _create(mrip.MRIP_MM1, mrip.mm1_params(customers=0)) == bad
    assert _create(mrip.MRIP_MM1, mrip.mm1_params(customers=10, feature_prefix=11)) == bad
    assert _create(mrip.MRIP_FF, mrip.ff_params()) == ok
    assert _create(mrip.MRIP_FF, mrip.ff_params(grid=96), mrip.MRIP_MAP_WAVE) == bad
    assert _create(mrip.MRIP_FF, mrip.ff_params(grid=96), mrip.MRIP_MAP_SIMT) == ok
    assert _create(mrip.MRIP_FF, mrip.ff_params(p_grow=1.5)) == bad
    p = mrip.rw_params()
    p.size = 4
    assert _create(mrip.MRIP_RW, p) == bad
    assert _create(7, mrip.rw_params()) == bad
    assert _create(mrip.MRIP_RW, mrip.rw_params(), mrip.MRIP_MAP_LANE0) == ok
    assert _create(mrip.MRIP_RW, mrip.rw_params(), 9) == bad
    assert _create(mrip.MRIP_PI, mrip.pi_params(1000)) == ok
    assert _create(mrip.MRIP_PI, mrip.pi_params(0)) == bad
    assert _create(mrip.MRIP_PI, mrip.pi_params(2**31)) == bad


def test_calls_out_of_order_and_bad_shapes():
    L = mrip.load()
    ctx = mrip.ctx_t()
    assert L.mrip_create(C.byref(ctx), mrip.MRIP_MM1, C.byref(mrip.mm1_params()), 0) == 0
    s = mrip.mrip_stats_t()
    assert L.mrip_stats(ctx, 0, 0.95, C.byref(s)) == mrip.MRIP_E_STATE
    assert L.mrip_run(ctx, 0, 42, None) == mrip.MRIP_E_INVAL
    assert L.mrip_set_shape(ctx, 3, 256) == mrip.MRIP_E_INVAL
    assert L.mrip_set_shape(ctx, 2, 128) == mrip.MRIP_E_INVAL
    assert L.mrip_set_shape(ctx, 4, 1024) == mrip.MRIP_OK
    assert L.mrip_set_split(ctx, 2) == mrip.MRIP_E_INVAL  # needs reps_per_wave = 1
    assert L.mrip_set_shape(ctx, 1, 256) == mrip.MRIP_OK
    assert L.mrip_set_split(ctx, 3) == mrip.MRIP_E_INVAL
    assert L.mrip_set_split(ctx, 8) == mrip.MRIP_OK
    assert L.mrip_set_split(ctx, 16) == mrip.MRIP_E_INVAL
    assert L.mrip_set_split(ctx, 4) == mrip.MRIP_OK
    for x, want in ((1, 0), (2, 0), (3, mrip.MRIP_E_INVAL), (8, 0), (16, mrip.MRIP_E_INVAL),
                    (4, 0)):
        assert L.mrip_set_plan_split(ctx, x, 0) == want, x
    # a launch holds < 2^32 lanes: 2^24 replications x 256 lanes is refused
    # before any device call
    assert L.mrip_run(ctx, 1 << 24, 42, None) == mrip.MRIP_E_INVAL
    assert b"lanes" in L.mrip_last_error(ctx)
    assert L.mrip_run(ctx, 1 << 32, 42, None) == mrip.MRIP_E_INVAL
    assert L.mrip_set_shape(ctx, 2, 256) == mrip.MRIP_E_INVAL
    assert L.mrip_run_plan(ctx, 42, None) == mrip.MRIP_E_STATE
    assert L.mrip_plan_stats(ctx, 0, 0.95, C.byref(s)) == mrip.MRIP_E_STATE
    assert b"no" in L.mrip_last_error(ctx)
    L.mrip_destroy(ctx)


def test_generator_choice_checks():
    # error paths only: choosing taus88 successfully uploads jump tables
    L = mrip.load()
    ctx = mrip.ctx_t()
    assert L.mrip_create(C.byref(ctx), mrip.MRIP_FF, C.byref(mrip.ff_params()), 0) == 0
    assert L.mrip_set_rng(ctx, mrip.MRIP_RNG_TAUS88) == mrip.MRIP_E_UNSUPPORTED
    assert L.mrip_set_rng(ctx, 7) == mrip.MRIP_E_INVAL
    assert L.mrip_set_rng(ctx, mrip.MRIP_RNG_PHILOX) == mrip.MRIP_OK
    L.mrip_destroy(ctx)
    ctx = mrip.ctx_t()
    assert L.mrip_create(C.byref(ctx), mrip.MRIP_MM1, C.byref(mrip.mm1_params()), 0) == 0
    assert L.mrip_set_split(ctx, 8) == mrip.MRIP_OK
    assert L.mrip_set_rng(ctx, mrip.MRIP_RNG_TAUS88) == mrip.MRIP_E_UNSUPPORTED
    assert b"4 wavefronts" in L.mrip_last_error(ctx)
    L.mrip_destroy(ctx)
    assert L.mrip_taus88(1, 4, 0, 0, 0, 0, None, None) == mrip.MRIP_OK  # n = 0: nothing to do
    assert L.mrip_taus88(1, 4, 0, 0, 0, 5, None, None) == mrip.MRIP_E_INVAL
    # one lane per value: 2^32 - 255 values would not fit one launch
    fake = C.cast(C.c_void_p(256), C.POINTER(C.c_uint32))
    assert L.mrip_taus88(1, 4, 0, 0, 0, 2**32 - 255, fake, None) == mrip.MRIP_E_INVAL
    assert L.mrip_philox(1, fake, 2**32 - 255, fake, None) == mrip.MRIP_E_INVAL
    assert L.mrip_mlp_forward(fake, fake, 2**30, fake, None) == mrip.MRIP_E_INVAL
    assert L.mrip_adam_step(fake, fake, fake, fake, 2**32, 1, 1e-3, 0.9, 0.999, 1e-8,
                            None) == mrip.MRIP_E_INVAL


def test_bind_output_and_resume_checks():
    L = mrip.load()
    ctx = mrip.ctx_t()
    assert L.mrip_create(C.byref(ctx), mrip.MRIP_RW, C.byref(mrip.rw_params()), 0) == 0
    assert L.mrip_bind_output(ctx, 2, None, 0) == mrip.MRIP_E_INVAL  # the walk has 2 outputs
    assert L.mrip_bind_output(ctx, 0, 0x1002, 64) == mrip.MRIP_E_INVAL  # misaligned
    assert L.mrip_bind_output(ctx, 0, 0x1000, 0) == mrip.MRIP_E_INVAL  # empty
    assert L.mrip_bind_output(ctx, 1, None, 0) == mrip.MRIP_OK  # unbind
    L.mrip_destroy(ctx)
    ctx = mrip.ctx_t()
    assert L.mrip_create(C.byref(ctx), mrip.MRIP_MM1, C.byref(mrip.mm1_params()), 0) == 0
    assert L.mrip_bind_output(ctx, 3, None, 0) == mrip.MRIP_OK  # features are output 3
    assert L.mrip_run_plan_resume(ctx, 42, None, None) == mrip.MRIP_E_STATE  # no plan
    flags = (C.c_uint8 * 4)()
    assert L.mrip_plan_done(ctx, flags, 4) == mrip.MRIP_E_STATE  # no plan run
    assert L.mrip_plan_done(ctx, None, 4) == mrip.MRIP_E_INVAL
    assert L.mrip_set_plan_limit(ctx, 3) == mrip.MRIP_OK
    assert L.mrip_set_plan_limit(ctx, 0) == mrip.MRIP_OK
    L.mrip_destroy(ctx)


def test_c_example_is_built_and_checks_its_arguments():
    # the plain-C client of the library (built by build()); these calls
    # return before any HIP call
    import subprocess
    exe = os.path.join(ROOT, "paper_1501_01405_amd", "examples", "mrip_from_c")
    assert os.access(exe, os.X_OK), "the C example is not built"
    assert subprocess.run([exe], capture_output=True, timeout=60).returncode == 2
    r = subprocess.run([exe, "pi", "100", "4", "42", "warp"], capture_output=True, timeout=60)
    assert r.returncode == 2 and b"unknown mapping" in r.stderr


def test_tune_cache_key_and_file_round_trip(tmp_path):
    # the autotuner's cache on the host: keys bucket the plan by powers of
    # two, entries survive a write and a read, the last put for a key wins,
    # other keys are kept, and an absent file or key reads as absent
    key = mrip.mrip_tune_key(mrip.MRIP_MM1, mrip.MRIP_MAP_WAVE, 2048, 70, 997000, "gfx950:sramecc+",
                             256)
    assert key == "m2/map2/n2^11/long2^6/max2^19/gfx950:sramecc+/256cu"
    # same buckets, same key; another bucket, another key; the arch is one token
    assert mrip.mrip_tune_key(2, 2, 3000, 100, 600000, "gfx950:sramecc+", 256) == key
    assert mrip.mrip_tune_key(2, 2, 4096, 70, 997000, "gfx950:sramecc+", 256) != key
    assert " " not in mrip.mrip_tune_key(2, 2, 1, 0, 1, "gfx 950/x", 8)
    with pytest.raises(mrip.MripError):
        mrip.mrip_tune_key(2, 2, 0, 0, 1, "gfx950", 256)
    path = tmp_path / "tune.txt"
    assert mrip.mrip_tune_cache_get(path, key) is None
    mrip.mrip_tune_cache_put(path, key, 2, 256, 8, 0.612)
    mrip.mrip_tune_cache_put(path, "other", 1, 64, 1, 1.5)
    got = mrip.mrip_tune_cache_get(path, key)
    assert got["reps_per_wave"] == 2 and got["workgroup"] == 256 and got["plan_split"] == 8
    assert abs(got["ms"] - 0.612) < 1e-6
    mrip.mrip_tune_cache_put(path, key, 4, 1024, 1, 0.5)
    assert mrip.mrip_tune_cache_get(path, key)["reps_per_wave"] == 4
    assert mrip.mrip_tune_cache_get(path, "other")["workgroup"] == 64
    assert len(path.read_text().splitlines()) == 2
    assert mrip.mrip_tune_cache_get(path, "absent") is None
    with pytest.raises(mrip.MripError):
        mrip.mrip_tune_cache_put(path, "has space", 1, 64, 1, 1.0)
