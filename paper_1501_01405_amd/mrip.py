"""ctypes binding of libmrip.so (include/mrip.h), same names as the C ABI.

Argument marshalling only: every step of the computation runs in the HIP
library. Device buffers passed in or out are torch CUDA tensors (PyTorch
provides device memory and streams, nothing else). There is no fallback:
if the library is missing, `load()` raises.
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# MRIP_LIB names another build of the library (for example one with the
# host code under sanitizers); the default is the in-tree build
LIB_PATH = os.environ.get("MRIP_LIB") or os.path.join(_HERE, "libmrip.so")

MRIP_OK, MRIP_E_INVAL, MRIP_E_NOMEM, MRIP_E_HIP, MRIP_E_STATE, MRIP_E_TOO_FEW, \
    MRIP_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MRIP_RW, MRIP_MM1, MRIP_FF, MRIP_PI = 1, 2, 3, 4
MRIP_MAP_AUTO, MRIP_MAP_SIMT, MRIP_MAP_WAVE, MRIP_MAP_LANE0 = 0, 1, 2, 3
MRIP_RNG_PHILOX, MRIP_RNG_TAUS88 = 0, 1
MRIP_MLP_OUT = 4
MRIP_MLP_GRAD_NOALLOC_MAX = 4096
MRIP_MLP_PARAMS = 18436
MRIP_CV_BETA_BINS = 16
MRIP_CV_COEFS = 5


class mrip_rw_params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("walkers", C.c_uint32), ("grid", C.c_uint32),
                ("steps", C.c_uint32), ("walker_sites", C.c_uint32)]


class mrip_mm1_params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("lambda_", C.c_float), ("mu", C.c_float),
                ("customers", C.c_uint64), ("feature_prefix", C.c_uint64)]


class mrip_ff_params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("grid", C.c_uint32), ("steps", C.c_uint32),
                ("p_grow", C.c_double), ("f_light", C.c_double)]


class mrip_pi_params(C.Structure):
    _fields_ = [("size", C.c_uint32), ("points", C.c_uint64)]


class mrip_stats_t(C.Structure):
    _fields_ = [("n", C.c_uint64), ("mean", C.c_double), ("var", C.c_double),
                ("half_width", C.c_double), ("t_quantile", C.c_double),
                ("confidence", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class mrip_plan_item(C.Structure):
    _fields_ = [("dp", C.c_uint32), ("rep", C.c_uint32), ("customers", C.c_uint64),
                ("lambda_", C.c_float), ("mu", C.c_float)]


class mrip_tune_entry(C.Structure):
    _fields_ = [("reps_per_wave", C.c_uint32), ("workgroup", C.c_uint32),
                ("plan_split", C.c_uint32), ("ms", C.c_float)]


class mrip_cv_hparams(C.Structure):
    _fields_ = [("size", C.c_uint32), ("epochs", C.c_uint32), ("batch", C.c_uint32),
                ("lr", C.c_float), ("beta1", C.c_float), ("beta2", C.c_float),
                ("eps", C.c_float)]


PLAN_ITEM_DTYPE = np.dtype([("dp", "<u4"), ("rep", "<u4"), ("customers", "<u8"),
                            ("lambda_", "<f4"), ("mu", "<f4")])
assert PLAN_ITEM_DTYPE.itemsize == C.sizeof(mrip_plan_item)

ctx_t = C.c_void_p
vp = C.c_void_p
u32, u64, f32, f64 = C.c_uint32, C.c_uint64, C.c_float, C.c_double
st = C.c_int

# name -> (restype, argtypes)
_SIGS = {
    "mrip_create": (st, [C.POINTER(ctx_t), C.c_int, vp, C.c_int]),
    "mrip_destroy": (None, [ctx_t]),
    "mrip_set_shape": (st, [ctx_t, u32, u32]),
    "mrip_set_split": (st, [ctx_t, u32]),
    "mrip_set_plan_split": (st, [ctx_t, u32, u64]),
    "mrip_set_rng": (st, [ctx_t, C.c_int]),
    "mrip_get_shape": (st, [ctx_t, C.POINTER(u32), C.POINTER(u32), C.POINTER(u32),
                            C.POINTER(u32)]),
    "mrip_run": (st, [ctx_t, u64, u64, vp]),
    "mrip_stats": (st, [ctx_t, u32, f64, C.POINTER(mrip_stats_t)]),
    "mrip_stats_back": (st, [ctx_t, u32, u32, f64, C.POINTER(mrip_stats_t)]),
    "mrip_outputs": (st, [ctx_t, u32, vp, u64, C.c_int]),
    "mrip_output_ptr": (st, [ctx_t, u32, C.POINTER(vp)]),
    "mrip_bind_output": (st, [ctx_t, u32, vp, u64]),
    "mrip_run_plan_resume": (st, [ctx_t, u64, vp, vp]),
    "mrip_last_run_ms": (st, [ctx_t, C.POINTER(f32)]),
    "mrip_set_timing": (st, [ctx_t, u32]),
    "mrip_run_history_ms": (st, [ctx_t, C.POINTER(f32), u32, C.POINTER(u32)]),
    "mrip_plan_set": (st, [ctx_t, vp, u64]),
    "mrip_run_plan": (st, [ctx_t, u64, vp]),
    "mrip_plan_stats": (st, [ctx_t, u32, f64, C.POINTER(mrip_stats_t)]),
    "mrip_set_plan_limit": (st, [ctx_t, u64]),
    "mrip_plan_done": (st, [ctx_t, vp, u64]),
    "mrip_autotune": (st, [ctx_t, u64, u64, vp, C.POINTER(u32), C.POINTER(u32),
                           C.POINTER(f32)]),
    "mrip_tune_key": (st, [C.c_int, C.c_int, u64, u64, u64, C.c_char_p, u32, C.c_char_p, u64]),
    "mrip_tune_cache_get": (st, [C.c_char_p, C.c_char_p, C.POINTER(mrip_tune_entry)]),
    "mrip_tune_cache_put": (st, [C.c_char_p, C.c_char_p, C.POINTER(mrip_tune_entry)]),
    "mrip_mlp_forward": (st, [vp, vp, u64, vp, vp]),
    "mrip_mlp_grad": (st, [vp, vp, vp, vp, u64, vp, vp, vp]),
    "mrip_mlp_grad_noalloc": (st, [vp, vp, vp, vp, u64, vp, vp, vp]),
    "mrip_adam_step": (st, [vp, vp, vp, vp, u64, u64, f32, f32, f32, f32, vp]),
    "mrip_cv_train": (st, [ctx_t, vp, u64, vp, C.POINTER(mrip_cv_hparams), u64, vp]),
    "mrip_cv_model": (st, [ctx_t, vp, vp, vp, vp, vp, vp]),
    "mrip_cv_set_model": (st, [ctx_t, vp, vp, vp, vp, f32, f32]),
    "mrip_cv_outputs": (st, [ctx_t, u32, vp, u64]),
    "mrip_cv_apply": (st, [ctx_t, vp, u64, u64, vp]),
    "mrip_cv_stats": (st, [ctx_t, u32, f64, C.POINTER(mrip_stats_t),
                           C.POINTER(mrip_stats_t)]),
    "mrip_cv_times": (st, [ctx_t, C.POINTER(f32), C.POINTER(f32)]),
    "mrip_philox": (st, [u64, vp, u64, vp, vp]),
    "mrip_taus88": (st, [u64, u32, u32, u32, u64, u64, vp, vp]),
    "mrip_t_quantile": (f64, [f64, f64]),
    "mrip_status_string": (C.c_char_p, [C.c_int]),
    "mrip_last_error": (C.c_char_p, [ctx_t]),
    "mrip_version": (C.c_char_p, []),
}

EXPORTED = tuple(_SIGS)

_lib = None


class MripError(RuntimeError):
    def __init__(self, status, msg=""):
        self.status = status
        super().__init__("%s (%d)%s" % (_status_name(status), status, ": " + msg if msg else ""))


def _status_name(s):
    try:
        return load().mrip_status_string(s).decode()
    except Exception:  # noqa: BLE001 - only used to format an error
        return "status"


def load():
    """Load libmrip.so (built by __graft_entry__.build()); raises if absent.

    PyTorch is imported first so that the library binds to the HIP runtime
    PyTorch already loaded (both carry the soname libamdhip64.so.7): one
    runtime per process, so torch's streams and buffers are valid handles
    for the library."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (see docstring)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmrip.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status, ctx=None):
    if status != MRIP_OK:
        msg = load().mrip_last_error(ctx).decode() if ctx else ""
        raise MripError(status, msg)
    return status


def _ptr(t):
    """Device (or host) address of a torch tensor or numpy array, or None."""
    if t is None:
        return None
    if hasattr(t, "data_ptr"):
        return t.data_ptr()
    return t.ctypes.data


def current_stream():
    import torch
    return torch.cuda.current_stream().cuda_stream


# ----------------------------------------------------------- raw C-ABI calls
def mrip_create(model, params, mapping=MRIP_MAP_AUTO):
    ctx = ctx_t()
    check(load().mrip_create(C.byref(ctx), model, C.byref(params), mapping))
    return ctx


def mrip_destroy(ctx):
    load().mrip_destroy(ctx)


def mrip_set_shape(ctx, reps_per_wave, workgroup):
    check(load().mrip_set_shape(ctx, reps_per_wave, workgroup), ctx)


def mrip_set_split(ctx, waves_per_rep):
    check(load().mrip_set_split(ctx, waves_per_rep), ctx)


def mrip_set_plan_split(ctx, waves_per_item, long_min=0):
    check(load().mrip_set_plan_split(ctx, waves_per_item, long_min), ctx)


def mrip_set_rng(ctx, rng):
    check(load().mrip_set_rng(ctx, rng), ctx)


def mrip_get_shape(ctx):
    """dict(reps_per_wave, workgroup, split, plan_split)."""
    v = [u32() for _ in range(4)]
    check(load().mrip_get_shape(ctx, *[C.byref(x) for x in v]), ctx)
    return dict(zip(("reps_per_wave", "workgroup", "split", "plan_split"),
                    (x.value for x in v)))


def mrip_run(ctx, n_reps, seed, stream=None):
    check(load().mrip_run(ctx, n_reps, seed, stream), ctx)


def mrip_stats(ctx, output=0, confidence=0.95):
    s = mrip_stats_t()
    check(load().mrip_stats(ctx, output, confidence, C.byref(s)), ctx)
    return s.as_dict()


def mrip_stats_back(ctx, back, output=0, confidence=0.95):
    s = mrip_stats_t()
    check(load().mrip_stats_back(ctx, back, output, confidence, C.byref(s)), ctx)
    return s.as_dict()


def mrip_outputs(ctx, output, dst, dst_is_device):
    nbytes = dst.numel() * dst.element_size() if hasattr(dst, "numel") else dst.nbytes
    check(load().mrip_outputs(ctx, output, _ptr(dst), nbytes, int(dst_is_device)), ctx)
    return dst


def mrip_set_timing(ctx, every):
    check(load().mrip_set_timing(ctx, every), ctx)


def mrip_last_run_ms(ctx):
    ms = f32()
    check(load().mrip_last_run_ms(ctx, C.byref(ms)), ctx)
    return ms.value


def mrip_run_history_ms(ctx, max_n=256):
    buf = (f32 * max_n)()
    n = u32()
    check(load().mrip_run_history_ms(ctx, buf, max_n, C.byref(n)), ctx)
    return [buf[i] for i in range(n.value)]


def mrip_plan_set(ctx, items):
    items = np.ascontiguousarray(items, dtype=PLAN_ITEM_DTYPE)
    check(load().mrip_plan_set(ctx, items.ctypes.data, items.shape[0]), ctx)


def mrip_run_plan(ctx, seed, stream=None):
    check(load().mrip_run_plan(ctx, seed, stream), ctx)


def mrip_bind_output(ctx, output, tensor):
    """Bind a torch device tensor as output `output` (None unbinds)."""
    if tensor is None:
        check(load().mrip_bind_output(ctx, output, None, 0), ctx)
    else:
        nbytes = tensor.numel() * tensor.element_size()
        check(load().mrip_bind_output(ctx, output, tensor.data_ptr(), nbytes), ctx)


def mrip_run_plan_resume(ctx, seed, skip_done, stream=None):
    skip = None
    if skip_done is not None:
        skip = np.ascontiguousarray(skip_done, dtype=np.uint8)
    check(load().mrip_run_plan_resume(ctx, seed, _ptr(skip), stream), ctx)


def mrip_set_plan_limit(ctx, max_items):
    check(load().mrip_set_plan_limit(ctx, max_items), ctx)


def mrip_plan_done(ctx, n):
    out = np.zeros(n, np.uint8)
    check(load().mrip_plan_done(ctx, out.ctypes.data, n), ctx)
    return out


def mrip_plan_stats(ctx, dp, confidence=0.95):
    s = mrip_stats_t()
    check(load().mrip_plan_stats(ctx, dp, confidence, C.byref(s)), ctx)
    return s.as_dict()


def mrip_autotune(ctx, seed, calib_items=0, stream=None):
    r, w, ms = u32(), u32(), f32()
    check(load().mrip_autotune(ctx, seed, calib_items, stream, C.byref(r), C.byref(w),
                               C.byref(ms)), ctx)
    return r.value, w.value, ms.value


def mrip_tune_key(model, mapping, n_items, n_long, max_customers, arch, cus):
    buf = C.create_string_buffer(256)
    check(load().mrip_tune_key(model, mapping, n_items, n_long, max_customers, arch.encode(), cus,
                               buf, len(buf)))
    return buf.value.decode()


def mrip_tune_cache_get(path, key):
    """dict(reps_per_wave, workgroup, plan_split, ms), or None when absent."""
    e = mrip_tune_entry()
    s = load().mrip_tune_cache_get(str(path).encode(), key.encode(), C.byref(e))
    if s == MRIP_E_STATE:
        return None
    check(s)
    return {k: getattr(e, k) for k, _ in e._fields_}


def mrip_tune_cache_put(path, key, reps_per_wave, workgroup, plan_split, ms):
    e = mrip_tune_entry(reps_per_wave, workgroup, plan_split, ms)
    check(load().mrip_tune_cache_put(str(path).encode(), key.encode(), C.byref(e)))


def mrip_mlp_forward(theta, x, n, y, stream=None):
    check(load().mrip_mlp_forward(_ptr(theta), _ptr(x), n, _ptr(y), stream))


def mrip_mlp_grad(theta, x, z, y, n, grad, loss=None, stream=None):
    check(load().mrip_mlp_grad(_ptr(theta), _ptr(x), _ptr(z), _ptr(y), n, _ptr(grad),
                               _ptr(loss), stream))


def mrip_mlp_grad_noalloc(theta, x, z, y, n, grad, loss=None, stream=None):
    check(load().mrip_mlp_grad_noalloc(_ptr(theta), _ptr(x), _ptr(z), _ptr(y), n, _ptr(grad),
                                       _ptr(loss), stream))


def mrip_adam_step(theta, m, v, grad, n_params, step, lr=1e-3, beta1=0.9, beta2=0.999,
                   eps=1e-8, stream=None):
    check(load().mrip_adam_step(_ptr(theta), _ptr(m), _ptr(v), _ptr(grad), n_params, step, lr,
                                beta1, beta2, eps, stream))


def mrip_cv_train(ctx, items, theta0, hparams=None, seed=42, stream=None):
    items = np.ascontiguousarray(items, dtype=PLAN_ITEM_DTYPE)
    theta0 = np.ascontiguousarray(theta0, dtype=np.float32)
    assert theta0.shape == (MRIP_MLP_PARAMS,)
    hp = C.byref(hparams) if hparams is not None else None
    check(load().mrip_cv_train(ctx, items.ctypes.data, items.shape[0], theta0.ctypes.data, hp,
                               seed, stream), ctx)


def mrip_cv_model(ctx):
    """dict(theta, feat_mean, feat_std, coef (bins x coefs), rho_range, final_loss)."""
    theta = np.zeros(MRIP_MLP_PARAMS, np.float32)
    mean = np.zeros(10, np.float32)
    std = np.zeros(10, np.float32)
    coef = np.zeros((MRIP_CV_BETA_BINS, MRIP_CV_COEFS), np.float32)
    rr = np.zeros(2, np.float32)
    loss = f32()
    check(load().mrip_cv_model(ctx, theta.ctypes.data, mean.ctypes.data, std.ctypes.data,
                               coef.ctypes.data, rr.ctypes.data, C.byref(loss)), ctx)
    return dict(theta=theta, feat_mean=mean, feat_std=std, coef=coef,
                rho_range=(float(rr[0]), float(rr[1])), final_loss=loss.value)


def mrip_cv_set_model(ctx, theta, feat_mean, feat_std, coef_table, rho_lo, rho_hi):
    """coef_table: (MRIP_CV_BETA_BINS, MRIP_CV_COEFS), or one row for every bin."""
    theta = np.ascontiguousarray(theta, dtype=np.float32)
    feat_mean = np.ascontiguousarray(feat_mean, dtype=np.float32)
    feat_std = np.ascontiguousarray(feat_std, dtype=np.float32)
    coef = np.ascontiguousarray(np.broadcast_to(np.asarray(coef_table, np.float32),
                                                (MRIP_CV_BETA_BINS, MRIP_CV_COEFS)))
    check(load().mrip_cv_set_model(ctx, theta.ctypes.data, feat_mean.ctypes.data,
                                   feat_std.ctypes.data, coef.ctypes.data, rho_lo, rho_hi), ctx)


# columns per replication of each mrip_cv_outputs `which`
CV_OUTPUT_COLS = {0: 1, 1: 1, 2: 4, 3: 10, 4: 8, 5: 1, 6: 10, 7: 8, 8: 4}


def mrip_cv_outputs(ctx, which, n):
    cols = CV_OUTPUT_COLS.get(which, 1)
    out = np.zeros((n, cols) if cols > 1 else n, np.float32)
    check(load().mrip_cv_outputs(ctx, which, out.ctypes.data, out.nbytes), ctx)
    return out


def mrip_cv_apply(ctx, items, seed=42, stream=None):
    items = np.ascontiguousarray(items, dtype=PLAN_ITEM_DTYPE)
    check(load().mrip_cv_apply(ctx, items.ctypes.data, items.shape[0], seed, stream), ctx)


def mrip_cv_stats(ctx, dp, confidence=0.95):
    a, b = mrip_stats_t(), mrip_stats_t()
    check(load().mrip_cv_stats(ctx, dp, confidence, C.byref(a), C.byref(b)), ctx)
    return a.as_dict(), b.as_dict()


def mrip_cv_times(ctx):
    """(simulation kernel ms, inference and estimator ms) of the last apply."""
    a, b = f32(), f32()
    check(load().mrip_cv_times(ctx, C.byref(a), C.byref(b)), ctx)
    return a.value, b.value


def mrip_philox(seed, ctr, n, out, stream=None):
    check(load().mrip_philox(seed, _ptr(ctr), n, _ptr(out), stream))


def mrip_taus88(seed, model, dp, rep, skip, n, out, stream=None):
    check(load().mrip_taus88(seed, model, dp, rep, skip, n, _ptr(out), stream))


def mrip_t_quantile(p, dof):
    return load().mrip_t_quantile(p, dof)


# ------------------------------------------------------------ convenience
def rw_params(walkers=64, grid=64, steps=1000, walker_sites=False):
    return mrip_rw_params(C.sizeof(mrip_rw_params), walkers, grid, steps, int(walker_sites))


def mm1_params(lam=0.9, mu=1.0, customers=100000, feature_prefix=0):
    return mrip_mm1_params(C.sizeof(mrip_mm1_params), lam, mu, customers, feature_prefix)


def ff_params(grid=128, steps=2000, p_grow=0.01, f_light=1e-5):
    return mrip_ff_params(C.sizeof(mrip_ff_params), grid, steps, p_grow, f_light)


def pi_params(points=10_000_000):
    return mrip_pi_params(C.sizeof(mrip_pi_params), points)


def cv_hparams(epochs=20, batch=1024, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    return mrip_cv_hparams(C.sizeof(mrip_cv_hparams), epochs, batch, lr, beta1, beta2, eps)


_OUT_DTYPES = {MRIP_RW: ("int32", "int32", "int32"), MRIP_MM1: ("float32",) * 3,
               MRIP_FF: ("int32",), MRIP_PI: ("int32", "float32")}


class Context:
    """An owned mrip_ctx; outputs come back as torch tensors on the device."""

    def __init__(self, model, params, mapping=MRIP_MAP_AUTO):
        self.model = model
        self.params = params
        self.ctx = mrip_create(model, params, mapping)
        self.n = 0

    def close(self):
        if self.ctx:
            mrip_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass

    def set_shape(self, reps_per_wave, workgroup):
        mrip_set_shape(self.ctx, reps_per_wave, workgroup)

    def set_split(self, waves_per_rep):
        mrip_set_split(self.ctx, waves_per_rep)

    def set_plan_split(self, waves_per_item, long_min=0):
        mrip_set_plan_split(self.ctx, waves_per_item, long_min)

    def shape(self):
        return mrip_get_shape(self.ctx)

    def set_rng(self, rng):
        mrip_set_rng(self.ctx, rng)

    def run(self, n_reps, seed=42, stream=None):
        mrip_run(self.ctx, n_reps, seed, current_stream() if stream is None else stream)
        self.n = n_reps

    def stats(self, output=0, confidence=0.95):
        return mrip_stats(self.ctx, output, confidence)

    def stats_back(self, back, output=0, confidence=0.95):
        return mrip_stats_back(self.ctx, back, output, confidence)

    def output(self, output=0, n=None):
        import torch
        n = self.n if n is None else n
        if self.model == MRIP_MM1 and output in (3, 4):
            t = torch.empty((n, 10 if output == 3 else 8), dtype=torch.float32, device="cuda")
        else:
            dt = getattr(torch, _OUT_DTYPES[self.model][output])
            t = torch.empty(n, dtype=dt, device="cuda")
        return mrip_outputs(self.ctx, output, t, True)

    def set_timing(self, every):
        mrip_set_timing(self.ctx, every)

    def last_ms(self):
        return mrip_last_run_ms(self.ctx)

    def history_ms(self, max_n=256):
        return mrip_run_history_ms(self.ctx, max_n)

    def plan_set(self, items):
        mrip_plan_set(self.ctx, items)
        self.n = len(items)

    def run_plan(self, seed=42, stream=None):
        mrip_run_plan(self.ctx, seed, current_stream() if stream is None else stream)

    def bind_output(self, output, tensor):
        mrip_bind_output(self.ctx, output, tensor)
        self._bound = getattr(self, "_bound", {})
        self._bound[output] = tensor  # keep the buffer alive while bound

    def run_plan_resume(self, skip_done, seed=42, stream=None):
        mrip_run_plan_resume(self.ctx, seed, skip_done,
                             current_stream() if stream is None else stream)

    def plan_stats(self, dp, confidence=0.95):
        return mrip_plan_stats(self.ctx, dp, confidence)

    def set_plan_limit(self, max_items):
        mrip_set_plan_limit(self.ctx, max_items)

    def plan_done(self):
        return mrip_plan_done(self.ctx, self.n)

    def autotune(self, seed=42, calib_items=0):
        return mrip_autotune(self.ctx, seed, calib_items, current_stream())
