"""ctypes view of the C oracle (oracle.c) -- TEST INFRASTRUCTURE ONLY.

Every function here is a thin call into the sequential C oracle, one
replication per call. Only tests, the smoke check and the benchmark's
CPU-baseline leg use this module.
"""
import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

_lib = None

u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")


def lib():
    """Load liboracle.so, compiling it first if it is missing or stale
    (MRIP_ORACLE_LIB names another build of it, loaded as it is)."""
    global _lib
    if _lib is None:
        path = os.environ.get("MRIP_ORACLE_LIB") or _build.build(force=False)
        L = C.CDLL(path)
        L.oracle_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.oracle_philox_batch.argtypes = [C.c_uint64, u32p, u32p, u32p]
        L.oracle_u01.argtypes = [C.c_uint32]
        L.oracle_u01.restype = C.c_float
        L.oracle_exp_variate.argtypes = [C.c_uint32, C.c_float]
        L.oracle_exp_variate.restype = C.c_float
        L.oracle_rw_direction.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32]
        L.oracle_rw_direction.restype = C.c_int
        L.oracle_rw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32,
                                C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                C.POINTER(C.c_int64)]
        L.oracle_rw_injected.argtypes = [u8p, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.POINTER(C.c_int64), C.POINTER(C.c_int64),
                                         C.POINTER(C.c_int64)]
        L.oracle_mm1.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_float,
                                 C.c_float, C.c_uint64, f32p, C.c_void_p, C.c_void_p]
        L.oracle_mm1_injected.argtypes = [f32p, f32p, C.c_uint64, C.c_uint64, C.c_double,
                                          C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, f32p,
                                          C.c_void_p]
        L.oracle_variate_mean.argtypes = [C.c_float]
        L.oracle_variate_mean.restype = C.c_double
        L.oracle_pi_inside.argtypes = [C.c_uint32, C.c_uint32]
        L.oracle_pi_inside.restype = C.c_int
        L.oracle_pi.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.oracle_pi.restype = C.c_int64
        L.oracle_ff_threshold.argtypes = [C.c_double]
        L.oracle_ff_threshold.restype = C.c_uint32
        L.oracle_ff.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_double,
                                C.c_double, C.POINTER(C.c_int64)]
        L.oracle_ff_injected.argtypes = [C.c_uint32, C.c_uint32, C.c_double, C.c_double, u32p,
                                         C.c_void_p, u8p, C.POINTER(C.c_int64)]
        L.oracle_ff_state.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32,
                                      C.c_double, C.c_double, u8p, C.POINTER(C.c_int64)]
        L.oracle_taus88_next.argtypes = [u32p]
        L.oracle_taus88_next.restype = C.c_uint32
        L.oracle_taus88_seed.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, u32p]
        L.oracle_taus88_seed.restype = None
        L.oracle_taus88_outputs.argtypes = [u32p, C.c_uint64, u32p]
        L.oracle_taus88_outputs.restype = None
        L.oracle_pi_taus.argtypes = [C.c_uint64, C.c_uint32, C.c_uint64]
        L.oracle_pi_taus.restype = C.c_int64
        L.oracle_rw_taus.argtypes = L.oracle_rw.argtypes
        L.oracle_mm1_taus.argtypes = L.oracle_mm1.argtypes
        for name in ("oracle_rw_taus", "oracle_mm1_taus", "oracle_rw", "oracle_mm1", "oracle_mm1_injected", "oracle_ff",
                     "oracle_ff_injected", "oracle_ff_state", "oracle_rw_injected"):
            getattr(L, name).restype = C.c_int
        L.oracle_philox4x32_10.restype = None
        L.oracle_philox_batch.restype = None
        _lib = L
    return _lib


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s rejected its arguments (rc=%d)" % (what, rc))


# ---------------------------------------------------------------- Philox
def philox(ctr, key):
    """Philox4x32-10 blocks for ctr (n,4) and key (n,2) uint32 arrays."""
    ctr = np.ascontiguousarray(ctr, dtype=np.uint32).reshape(-1, 4)
    key = np.ascontiguousarray(key, dtype=np.uint32).reshape(-1, 2)
    if key.shape[0] == 1 and ctr.shape[0] > 1:
        key = np.ascontiguousarray(np.repeat(key, ctr.shape[0], axis=0))
    out = np.empty_like(ctr)
    lib().oracle_philox_batch(ctr.shape[0], ctr, key, out)
    return out


def seed_key(seed):
    return np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint32)


def u01(x):
    return np.float32(lib().oracle_u01(int(x)))


def exp_variate(x, rate):
    return np.float32(lib().oracle_exp_variate(int(x), float(rate)))


# ---------------------------------------------------------------- random walk
def rw_direction(seed, rep, walker, t):
    return lib().oracle_rw_direction(seed, rep, walker, t)


def rw(seed, rep, walkers=64, grid=64, steps=1000, walker_sites=False):
    """(ssd, distinct) of one random-walk replication, and the per-walker
    site count sum when walker_sites."""
    s, d, v = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().oracle_rw(seed, rep, walkers, grid, steps, C.byref(s), C.byref(d),
                           C.byref(v)), "rw")
    return (s.value, d.value, v.value) if walker_sites else (s.value, d.value)


def rw_injected(dirs, walker_sites=False):
    """dirs: (walkers, steps) array of moves 0..3 on a 64x64 torus."""
    dirs = np.ascontiguousarray(dirs, dtype=np.uint8)
    w, t = dirs.shape
    s, d, v = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().oracle_rw_injected(dirs.reshape(-1), w, 64, t, C.byref(s), C.byref(d),
                                    C.byref(v)), "rw_injected")
    return (s.value, d.value, v.value) if walker_sites else (s.value, d.value)


def rw_taus(seed, rep, walkers=64, grid=64, steps=1000, walker_sites=False):
    """rw() on the replication's taus88 stream."""
    s, d, v = C.c_int64(), C.c_int64(), C.c_int64()
    _check(lib().oracle_rw_taus(seed, rep, walkers, grid, steps, C.byref(s), C.byref(d),
                                C.byref(v)), "rw_taus")
    return (s.value, d.value, v.value) if walker_sites else (s.value, d.value)


def rw_many(seed, reps, walkers=64, grid=64, steps=1000, threads=1, rng="philox",
            walker_sites=False):
    """Outputs (ssd[R], distinct[R]) for replications 0..reps-1 (or an id
    list), and walker_sites[R] when requested."""
    ids = list(range(reps)) if isinstance(reps, int) else list(reps)
    one = rw if rng == "philox" else rw_taus
    res = _map(lambda r: one(seed, r, walkers, grid, steps, True), ids, threads)
    out = tuple(np.array([x[i] for x in res], dtype=np.int64) for i in range(3))
    return out if walker_sites else out[:2]


# ---------------------------------------------------------------- M/M/1
def _mm1_call(fn, name, seed, rep, customers, lam, mu, dp, features, ctl):
    out = np.zeros(3, dtype=np.float32)
    feat = np.zeros(10, dtype=np.float32)
    c8 = np.zeros(8, dtype=np.float64)
    _check(fn(seed, dp, rep, customers, lam, mu, features, out,
              feat.ctypes.data if features else None, c8.ctypes.data if ctl else None), name)
    res = (out,) + ((feat,) if features else ()) + ((c8,) if ctl else ())
    return res if len(res) > 1 else out


def variate_mean(rate):
    """Exact mean of the exponential variate of `rate` as drawn (fp64)."""
    return lib().oracle_variate_mean(rate)


def mm1(seed, rep, customers, lam, mu, dp=0, features=0, ctl=False):
    """(mean_wq, mean_T, mean_idle); when features > 0 also the 10 features;
    with ctl, also the eight controls: over customers n >= features
    sum (S - E S), sum (A - E A), sum T_{n-1} (S - E S), sum T_{n-1} (A - E A),
    then the same four over customers n < features."""
    return _mm1_call(lib().oracle_mm1, "mm1", seed, rep, customers, lam, mu, dp, features, ctl)


def mm1_injected(A, S, ctl_after=None, es=1.0, ea=1.0):
    """Per-customer W, I, T and the means on explicit arrays; with
    ctl_after = K, also the eight controls (n >= K, then n < K) with means
    es, ea."""
    A = np.ascontiguousarray(A, dtype=np.float32)
    S = np.ascontiguousarray(S, dtype=np.float32)
    n = A.shape[0]
    W = np.zeros(n, np.float32)
    I = np.zeros(n, np.float32)
    T = np.zeros(n, np.float32)
    out = np.zeros(3, np.float32)
    c8 = np.zeros(8, np.float64)
    K = 0 if ctl_after is None else int(ctl_after)
    _check(lib().oracle_mm1_injected(A, S, n, K, es, ea, W.ctypes.data, I.ctypes.data,
                                     T.ctypes.data, out, c8.ctypes.data), "mm1_injected")
    return (W, I, T, out) if ctl_after is None else (W, I, T, out, c8)


def mm1_taus(seed, rep, customers, lam, mu, dp=0, features=0, ctl=False):
    """mm1() on the replication's taus88 stream."""
    return _mm1_call(lib().oracle_mm1_taus, "mm1_taus", seed, rep, customers, lam, mu, dp,
                     features, ctl)


def _stack(res, features, ctl):
    if not (features or ctl):
        return np.stack(res)
    cols = list(zip(*res))
    out = [np.stack(cols[0])]
    if features:
        out.append(np.stack(cols[1]))
    if ctl:
        out.append(np.stack(cols[-1]))
    return tuple(out)


def mm1_many(seed, reps, customers, lam, mu, dp=0, features=0, threads=1, rng="philox",
             ctl=False):
    """Outputs (R,3) float32, (R,10) features when requested, and the (R,8)
    fp64 controls with ctl."""
    ids = list(range(reps)) if isinstance(reps, int) else list(reps)
    one = mm1 if rng == "philox" else mm1_taus
    res = _map(lambda r: one(seed, r, customers, lam, mu, dp, features, ctl), ids, threads)
    return _stack(res, features, ctl)


def mm1_items(seed, items, features=0, threads=1, ctl=False):
    """Run plan items: an iterable of (dp, rep, customers, lambda, mu)."""
    items = list(items)
    res = _map(lambda it: mm1(seed, int(it[1]), int(it[2]), float(it[3]), float(it[4]),
                              int(it[0]), features, ctl), items, threads)
    return _stack(res, features, ctl)


# ---------------------------------------------------------------- forest fire
def ff_threshold(prob):
    return lib().oracle_ff_threshold(prob)


def ff(seed, rep, grid=128, steps=2000, p=0.01, f=1e-5):
    b = C.c_int64()
    _check(lib().oracle_ff(seed, rep, grid, steps, p, f, C.byref(b)), "ff")
    return b.value


def ff_state(seed, rep, grid, steps, p=0.01, f=1e-5):
    final = np.zeros(grid * grid, np.uint8)
    b = C.c_int64()
    _check(lib().oracle_ff_state(seed, rep, grid, steps, p, f, final, C.byref(b)), "ff_state")
    return final.reshape(grid, grid), b.value


def ff_injected(u, p, f, init=None):
    """u: (steps, L, L) uint32 uniforms; init: (L, L) states or None (empty)."""
    u = np.ascontiguousarray(u, dtype=np.uint32)
    steps, L, L2 = u.shape
    assert L == L2
    final = np.zeros(L * L, np.uint8)
    b = C.c_int64()
    init_arr = None if init is None else np.ascontiguousarray(init, dtype=np.uint8).reshape(-1)
    _check(lib().oracle_ff_injected(L, steps, p, f, u.reshape(-1),
                                    None if init_arr is None else init_arr.ctypes.data,
                                    final, C.byref(b)), "ff_injected")
    return final.reshape(L, L), b.value


def ff_many(seed, reps, grid=128, steps=2000, p=0.01, f=1e-5, threads=1):
    ids = list(range(reps)) if isinstance(reps, int) else list(reps)
    return np.array(_map(lambda r: ff(seed, r, grid, steps, p, f), ids, threads), np.int64)


# ---------------------------------------------------------------- Monte Carlo pi
def pi_inside(wx, wy):
    return bool(lib().oracle_pi_inside(int(wx), int(wy)))


def pi_hits(seed, rep, points):
    return int(lib().oracle_pi(seed, rep, points))


def pi_taus(seed, rep, points):
    return int(lib().oracle_pi_taus(seed, rep, points))


def pi_many(seed, reps, points, threads=1, rng="philox"):
    ids = list(range(reps)) if isinstance(reps, int) else list(reps)
    one = pi_hits if rng == "philox" else pi_taus
    return np.array(_map(lambda r: one(seed, r, points), ids, threads), np.int64)


# ---------------------------------------------------------------- taus88
MODEL_TAG = {"rw": 1, "mm1": 2, "ff": 3, "pi": 4}


def taus88_seed(seed, model, rep, dp=0):
    """Random Spacing start state (3 words) of the stream of (model, dp, rep)."""
    st = np.zeros(3, np.uint32)
    lib().oracle_taus88_seed(seed, MODEL_TAG.get(model, model), dp, rep, st)
    return st


def taus88_outputs(state, n):
    """n outputs from a start state; returns (outputs, state after)."""
    st = np.ascontiguousarray(state, dtype=np.uint32).copy()
    out = np.zeros(max(n, 1), np.uint32)
    lib().oracle_taus88_outputs(st, n, out)
    return out[:n], st


# ---------------------------------------------------------------- helpers
def _map(fn, xs, threads):
    if threads <= 1:
        return [fn(x) for x in xs]
    # ctypes drops the GIL during each call, so replications run in parallel.
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(fn, xs))


def default_threads():
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1
