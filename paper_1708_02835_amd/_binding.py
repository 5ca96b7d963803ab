"""ctypes binding of libgeolik.so (include/geolik.h), same names as the C ABI.

Argument marshalling only: torch tensors provide device memory and streams,
every computation runs in the HIP library.  A missing library raises
``GeolikError``; there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libgeolik.so")

GL_OK = 0
GL_NOT_SPD = 1
GL_EINVAL = -1
GL_ENOMEM = -2
GL_EHIP = -3
GL_EBUSY = -4
GL_ECANCELED = -5
GL_ETIMEDOUT = -6
GL_ENODEV = -7
GL_EVICTED = -9
GL_E2BIG = -10
GL_SCRATCH_BYTES = 96 << 20

GL_FP64 = 0
GL_MIXED_FP32 = 1
GL_MIXED_BF16 = 2
GL_MIXED_FP16 = 3

GL_EUCLIDEAN = 0
GL_GREAT_CIRCLE = 1

GL_LAYOUT_DENSE = 0
GL_LAYOUT_LOWER_TILES = 1


class GeolikError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__(f"{what}: {gl_status_string(status)} ({status})" if what else gl_status_string(status))


class gl_theta(ctypes.Structure):
    _fields_ = [("theta1", ctypes.c_double), ("theta2", ctypes.c_double), ("theta3", ctypes.c_double)]


class gl_opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("tile", ctypes.c_int32), ("keep_factor", ctypes.c_int32),
                ("band", ctypes.c_int32), ("reorder", ctypes.c_int32), ("metric", ctypes.c_int32),
                ("tol_hi", ctypes.c_double), ("tol_lo", ctypes.c_double), ("radius", ctypes.c_double),
                ("tol_64", ctypes.c_double), ("accuracy", ctypes.c_double), ("ind_tiles", ctypes.c_int32),
                ("graph", ctypes.c_int32), ("near_tiles", ctypes.c_int32), ("layout", ctypes.c_int32)]


class gl_result(ctypes.Structure):
    _fields_ = [("loglik", ctypes.c_double), ("logdet", ctypes.c_double), ("quad", ctypes.c_double),
                ("info", ctypes.c_int64), ("status", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("factor", ctypes.c_void_p)]

    def as_dict(self) -> dict:
        return {"loglik": self.loglik, "logdet": self.logdet, "quad": self.quad, "info": int(self.info),
                "status": int(self.status), "tile": int(self.tile), "factor": self.factor}


class lq_config(ctypes.Structure):
    _fields_ = [("max_inflight", ctypes.c_int32), ("streams", ctypes.c_int32), ("batch_small", ctypes.c_int32),
                ("small_n", ctypes.c_int32), ("hbm_budget_bytes", ctypes.c_size_t)]


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_U64 = ctypes.c_uint64
_SZ = ctypes.c_size_t
_D = ctypes.c_double

_SIGNATURES = {
    "gl_context_create": (_I32, [ctypes.c_int, _SZ, ctypes.POINTER(_P)]),
    "gl_context_destroy": (None, [_P]),
    "gl_opts_default": (None, [ctypes.POINTER(gl_opts)]),
    "gl_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "gl_footprint_bytes": (_SZ, [_I64, _I32, _I32]),
    "gl_pick_tile": (_I32, [_I64, _I32]),
    "gl_workspace_layout": (_I32, [_I64, _I32, _I32, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ),
                                   ctypes.POINTER(_SZ)]),
    "matern_generate": (_I32, [_P, _P, _P, _I64, _P, _P, _I64, gl_theta, _P, _P, _I64, _P]),
    "loglik_eval": (_I32, [_P, _P, _P, _P, _I64, gl_theta, ctypes.POINTER(gl_opts), ctypes.POINTER(gl_result), _P]),
    "loglik_eval_noalloc": (_I32, [_P, _P, _P, _P, _I64, gl_theta, ctypes.POINTER(gl_opts), ctypes.POINTER(gl_result),
                                   _P]),
    "krige_predict": (_I32, [_P, _P, _P, _P, _I64, _P, _P, _P]),
    "krige_cv": (_I32, [_P, _P, _P, _P, _I64, gl_theta, _P, _P, _I32, _P, _P, _P]),
    "gl_factor_release": (_I32, [_P, _P]),
    "gl_factor_to_dense": (_I32, [_P, _P, _P, _I64, _P]),
    "gl_factor_shape": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I32)]),
    "synth_generate": (_I32, [_P, _P, _P, _P, _I64, gl_theta, _P, _P, ctypes.POINTER(_I64), _P]),
    "gl_dataset_register": (_I32, [_P, _P, _P, _P, _I64, ctypes.POINTER(_U64)]),
    "gl_dataset_release": (_I32, [_P, _U64]),
    "lq_config_default": (None, [ctypes.POINTER(lq_config)]),
    "lq_create": (_I32, [_P, ctypes.POINTER(lq_config), ctypes.POINTER(_P)]),
    "lq_submit": (_I32, [_P, _U64, gl_theta, ctypes.POINTER(gl_opts), ctypes.POINTER(_U64)]),
    "lq_poll": (_I32, [_P, _U64, ctypes.POINTER(gl_result)]),
    "lq_wait": (_I32, [_P, _U64, ctypes.POINTER(gl_result), _I64]),
    "lq_cancel": (_I32, [_P, _U64]),
    "lq_tick_stats": (_I32, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "lq_stats": (_I32, [_P, ctypes.POINTER(_U64), ctypes.POINTER(_SZ), ctypes.POINTER(_I32), ctypes.POINTER(_U64)]),
    "lq_destroy": (_I32, [_P]),
    "gl_selftest": (_I32, [_P, _I32, ctypes.POINTER(_D), _I64]),
    "gl_profile_enable": (_I32, [_P, _I32]),
    "gl_morton_order": (_I32, [_P, _P, _P, _I64, _P, _P]),
    "gl_precision_stats": (_I32, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    "gl_profile_read": (_I32, [_P, ctypes.POINTER(_D), ctypes.POINTER(_D), ctypes.POINTER(_I64)]),
    "gl_profile_phases": (_I32, [_P, _P, _P, _P]),
}


def lib() -> ctypes.CDLL:
    """Load libgeolik.so; raises GeolikError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise GeolikError(GL_ENODEV, f"{LIB_PATH} is missing; run python -m paper_1708_02835_amd.build")
    l = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGNATURES.items():
        f = getattr(l, name)
        f.restype = res
        f.argtypes = args
    _lib = l
    return l


def gl_status_string(status: int) -> str:
    try:
        return lib().gl_status_string(int(status)).decode()
    except GeolikError:
        return f"status {status}"


def _check(status: int, what: str) -> int:
    if status < 0:
        raise GeolikError(status, what)
    return status


def _ptr(t) -> int:
    """Device pointer of a contiguous float64 CUDA tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise TypeError("expected a contiguous float64 CUDA tensor")
    return t.data_ptr()


def _stream(stream) -> int:
    import torch
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return getattr(stream, "cuda_stream", stream)


def _theta(theta) -> gl_theta:
    t1, t2, t3 = (float(v) for v in theta)
    return gl_theta(t1, t2, t3)


def _set_fields(obj, kw, what):
    names = {f for f, _ in type(obj)._fields_}
    for k, v in kw.items():
        if k not in names:
            raise TypeError(f"{what} has no field {k!r}")
        setattr(obj, k, v)


def _same_len(*ts):
    n = ts[0].numel()
    if any(t.numel() != n for t in ts[1:]):
        raise ValueError("coordinate and value vectors must have the same length")
    return n


def gl_opts_default(**kw) -> gl_opts:
    o = gl_opts()
    lib().gl_opts_default(ctypes.byref(o))
    _set_fields(o, kw, "gl_opts")
    return o


def gl_footprint_bytes(n: int, tile: int = 0, precision: int = GL_FP64) -> int:
    return int(lib().gl_footprint_bytes(int(n), int(tile), int(precision)))


def gl_workspace_layout(n: int, tile: int = 0, precision: int = GL_FP64) -> tuple[int, int, int]:
    t, v, m = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(lib().gl_workspace_layout(int(n), int(tile), int(precision), ctypes.byref(t), ctypes.byref(v),
                                     ctypes.byref(m)), "gl_workspace_layout")
    return t.value, v.value, m.value


class Context:
    """Owns a gl_context; use as a context manager or call close()."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = _P()
        _check(lib().gl_context_create(int(device), int(hbm_budget_bytes), ctypes.byref(h)), "gl_context_create")
        self.handle = h.value

    def close(self):
        if self.handle:
            lib().gl_context_destroy(self.handle)
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gl_context_create(device: int = 0, hbm_budget_bytes: int = 0) -> Context:
    return Context(device, hbm_budget_bytes)


def gl_context_destroy(ctx: Context) -> None:
    ctx.close()


def matern_generate(ctx: Context, x1, y1, x2, y2, theta, opts: gl_opts | None = None, out=None, stream=None):
    """Dense column-major n1×n2 Matérn covariance (distance from opts.metric);
    returns a torch tensor of shape (n2, n1) whose transpose is Σ12
    (out.T[i, j] = C(d(s1_i, s2_j)))."""
    import torch
    n1, n2 = _same_len(x1, y1), _same_len(x2, y2)
    if out is None:
        out = torch.empty((n2, n1), dtype=torch.float64, device=x1.device)
    if out.numel() != n1 * n2:
        raise ValueError("out must hold n1 * n2 values")
    _check(lib().matern_generate(ctx.handle, _ptr(x1), _ptr(y1), n1, _ptr(x2), _ptr(y2), n2, _theta(theta),
                                 ctypes.byref(opts) if opts is not None else None, _ptr(out), n1,
                                 _stream(stream)), "matern_generate")
    return out


def matern_generate_tiles(ctx: Context, x, y, theta, opts: gl_opts | None = None, out=None, stream=None):
    """Σ(θ) of one point set in the packed lower-tile storage (layout
    GL_LAYOUT_LOWER_TILES of matern_generate); returns (tiles, b) with tiles a
    flat float64 tensor of NT(NT+1)/2·b² values."""
    import torch
    n = _same_len(x, y)
    o = gl_opts()
    if opts is not None:
        ctypes.memmove(ctypes.byref(o), ctypes.byref(opts), ctypes.sizeof(gl_opts))
    else:
        o = gl_opts_default()
    o.layout = GL_LAYOUT_LOWER_TILES
    t_bytes, _, _ = gl_workspace_layout(n, o.tile, GL_FP64)
    if out is None:
        out = torch.empty(t_bytes // 8, dtype=torch.float64, device=x.device)
    if out.numel() * 8 < t_bytes:
        raise ValueError("out must hold the packed lower tiles")
    _check(lib().matern_generate(ctx.handle, _ptr(x), _ptr(y), n, None, None, 0, _theta(theta), ctypes.byref(o),
                                 _ptr(out), 0, _stream(stream)), "matern_generate")
    return out, gl_pick_tile(n, o.tile)


def gl_pick_tile(n: int, tile: int = 0) -> int:
    """The tile size loglik_eval uses for n locations (tile 0: automatic)."""
    b = lib().gl_pick_tile(int(n), int(tile))
    _check(b, "gl_pick_tile")
    return b


def loglik_eval(ctx: Context, x, y, z, theta, opts: gl_opts | None = None, stream=None) -> dict:
    """Alg. 2 on the device; returns the gl_result fields as a dict."""
    res = gl_result()
    o = opts if opts is not None else gl_opts_default()
    _same_len(x, y, z)
    st = lib().loglik_eval(ctx.handle, _ptr(x), _ptr(y), _ptr(z), x.numel(), _theta(theta), ctypes.byref(o),
                           ctypes.byref(res), _stream(stream))
    _check(st, "loglik_eval")
    return res.as_dict()


def loglik_eval_noalloc(ctx: Context, x, y, z, theta, opts: gl_opts | None = None, stream=None) -> dict:
    """loglik_eval with its workspace in the library's static device array
    (no allocation; binary64, n up to GL_SCRATCH_BYTES of workspace)."""
    res = gl_result()
    o = opts if opts is not None else gl_opts_default()
    _same_len(x, y, z)
    st = lib().loglik_eval_noalloc(ctx.handle, _ptr(x), _ptr(y), _ptr(z), x.numel(), _theta(theta),
                                   ctypes.byref(o), ctypes.byref(res), _stream(stream))
    _check(st, "loglik_eval_noalloc")
    return res.as_dict()


def krige_predict(ctx: Context, factor, xnew, ynew, out=None, return_variance: bool = False, var=None,
                  stream=None):
    """Eq. (5) predictions at the new locations; with return_variance, also
    the prediction variances of Eq. (4): returns (pred, var)."""
    import torch
    m = _same_len(xnew, ynew)
    if out is None:
        out = torch.empty(m, dtype=torch.float64, device=xnew.device)
    if out.numel() != m or (var is not None and var.numel() != m):
        raise ValueError("output vectors must have one entry per new location")
    if return_variance and var is None:
        var = torch.empty(m, dtype=torch.float64, device=xnew.device)
    _check(lib().krige_predict(ctx.handle, factor, _ptr(xnew), _ptr(ynew), m, _ptr(out),
                               _ptr(var) if return_variance else None, _stream(stream)), "krige_predict")
    return (out, var) if return_variance else out


def krige_cv(ctx: Context, x, y, z, theta, folds, opts: gl_opts | None = None, stream=None, pred=None):
    """k-fold cross-validation MSE of kriging; folds: n fold ids (0..k-1).
    pred: optional float64 CUDA tensor of n values that receives each
    location's prediction from the other folds.  Returns (mse per fold as a
    list, status)."""
    import numpy as np
    f = np.ascontiguousarray(np.asarray(folds, dtype=np.int32))
    n = _same_len(x, y, z)
    if f.size != n:
        raise ValueError("one fold id per location")
    if pred is not None and pred.numel() != n:
        raise ValueError("pred needs one value per location")
    k = int(f.max()) + 1 if f.size else 0
    mse = (ctypes.c_double * max(k, 1))()
    st = lib().krige_cv(ctx.handle, _ptr(x), _ptr(y), _ptr(z), x.numel(), _theta(theta),
                        ctypes.byref(opts) if opts is not None else None,
                        f.ctypes.data_as(ctypes.c_void_p), k, mse,
                        _ptr(pred) if pred is not None else None, _stream(stream))
    if st < 0:
        _check(st, "krige_cv")
    return [float(v) for v in mse[:k]], int(st)


def gl_factor_release(ctx: Context, factor) -> None:
    _check(lib().gl_factor_release(ctx.handle, factor), "gl_factor_release")


def gl_factor_shape(factor) -> tuple[int, int]:
    n, b = _I64(), _I32()
    _check(lib().gl_factor_shape(factor, ctypes.byref(n), ctypes.byref(b)), "gl_factor_shape")
    return int(n.value), int(b.value)


def gl_factor_to_dense(ctx: Context, factor, out=None, stream=None):
    """Dense lower factor; returns a (n, n) tensor holding Lᵀ in row-major order (L column-major)."""
    import torch
    n, _ = gl_factor_shape(factor)
    if out is None:
        out = torch.empty((n, n), dtype=torch.float64, device="cuda")
    _check(lib().gl_factor_to_dense(ctx.handle, factor, _ptr(out), n, _stream(stream)), "gl_factor_to_dense")
    return out


def synth_generate(ctx: Context, x, y, e, theta, tile: int = 0, opts: gl_opts | None = None, out=None,
                   stream=None):
    """Alg. 1: returns (z, info).  opts (tile, metric, radius) overrides tile."""
    import torch
    n = _same_len(x, y, e)
    if out is None:
        out = torch.empty(n, dtype=torch.float64, device=x.device)
    o = opts if opts is not None else gl_opts_default(tile=int(tile))
    info = _I64()
    _check(lib().synth_generate(ctx.handle, _ptr(x), _ptr(y), _ptr(e), n, _theta(theta), ctypes.byref(o),
                                _ptr(out), ctypes.byref(info), _stream(stream)), "synth_generate")
    return out, int(info.value)


def gl_dataset_register(ctx: Context, x, y, z) -> int:
    _same_len(x, y, z)
    ds = _U64()
    _check(lib().gl_dataset_register(ctx.handle, _ptr(x), _ptr(y), _ptr(z), x.numel(), ctypes.byref(ds)),
           "gl_dataset_register")
    return int(ds.value)


def gl_dataset_release(ctx: Context, ds: int) -> None:
    _check(lib().gl_dataset_release(ctx.handle, int(ds)), "gl_dataset_release")


def lq_config_default(**kw) -> lq_config:
    c = lq_config()
    lib().lq_config_default(ctypes.byref(c))
    _set_fields(c, kw, "lq_config")
    return c


def lq_create(ctx: Context, cfg: lq_config | None = None) -> int:
    q = _P()
    c = cfg if cfg is not None else lq_config_default()
    _check(lib().lq_create(ctx.handle, ctypes.byref(c), ctypes.byref(q)), "lq_create")
    return q.value


def lq_submit(q: int, ds: int, theta, opts: gl_opts | None = None) -> int:
    t = _U64()
    _check(lib().lq_submit(q, int(ds), _theta(theta), ctypes.byref(opts) if opts is not None else None,
                           ctypes.byref(t)), "lq_submit")
    return int(t.value)


def lq_poll(q: int, ticket: int):
    """None while pending, else the result dict; its "status" is the request's
    (GL_OK, GL_NOT_SPD, GL_ENOMEM, GL_ECANCELED, GL_EHIP).  An unknown ticket
    raises."""
    res = gl_result()
    st = lib().lq_poll(q, int(ticket), ctypes.byref(res))
    if st == GL_EBUSY:
        return None
    if st == GL_EINVAL:
        _check(st, "lq_poll")
    d = res.as_dict()
    d["status"] = st
    return d


def lq_wait(q: int, ticket: int, timeout_us: int = -1):
    """Result dict (status as for lq_poll), or None on timeout."""
    res = gl_result()
    st = lib().lq_wait(q, int(ticket), ctypes.byref(res), int(timeout_us))
    if st == GL_ETIMEDOUT:
        return None
    if st == GL_EINVAL:
        raise GeolikError(st, "lq_wait")
    d = res.as_dict()
    d["status"] = st
    return d


def lq_cancel(q: int, ticket: int) -> int:
    return int(lib().lq_cancel(q, int(ticket)))


def lq_stats(q: int) -> dict:
    c, pb, pi, fl = _U64(), _SZ(), _I32(), _U64()
    _check(lib().lq_stats(q, ctypes.byref(c), ctypes.byref(pb), ctypes.byref(pi), ctypes.byref(fl)), "lq_stats")
    return {"completed": int(c.value), "peak_bytes": int(pb.value), "peak_inflight": int(pi.value),
            "fused_launches": int(fl.value)}


def lq_tick_stats(q: int) -> dict:
    t, h, d, gp = _U64(), _D(), _D(), _D()
    _check(lib().lq_tick_stats(q, ctypes.byref(t), ctypes.byref(h), ctypes.byref(d), ctypes.byref(gp)),
           "lq_tick_stats")
    return {"ticks": int(t.value), "host_us": h.value, "device_ms": d.value, "gap_ms": gp.value}


def lq_destroy(q: int) -> None:
    _check(lib().lq_destroy(q), "lq_destroy")


def gl_selftest(ctx: Context, which: int):
    import numpy as np
    out = (ctypes.c_double * 256)()
    _check(lib().gl_selftest(ctx.handle, int(which), out, 256), "gl_selftest")
    return np.frombuffer(out, dtype=np.float64).copy()


PHASES = ("gen", "potrf", "trsm", "solve", "trail_crit", "trail_bulk", "reduce", "trail_pair",
          "mixed_fp64", "mixed_fp32", "mixed_bf16x6", "mixed_bf16x3", "mixed_bf16", "mixed_fp16x3",
          "mixed_fp16")  # GL_PHASE_* order


def gl_profile_enable(ctx: Context, on=True) -> None:
    """on: False/0 off, True/1 the trailing updates, 2 every phase."""
    _check(lib().gl_profile_enable(ctx.handle, int(on)), "gl_profile_enable")


def gl_profile_phases(ctx: Context) -> dict:
    """Per phase (PHASES): summed launch ms, algorithmic flops and launches since the last read."""
    k = len(PHASES)
    ms, fl, n = (_D * k)(), (_D * k)(), (_I64 * k)()
    _check(lib().gl_profile_phases(ctx.handle, ms, fl, n), "gl_profile_phases")
    return {p: {"ms": ms[i], "flops": fl[i], "launches": int(n[i])} for i, p in enumerate(PHASES)}


def gl_profile_read(ctx: Context) -> dict:
    ms, fl, n = _D(), _D(), _I64()
    _check(lib().gl_profile_read(ctx.handle, ctypes.byref(ms), ctypes.byref(fl), ctypes.byref(n)), "gl_profile_read")
    return {"ms": ms.value, "flops": fl.value, "launches": int(n.value)}


def gl_morton_order(ctx: Context, x, y, stream=None):
    """Morton permutation of the locations (int64 CUDA tensor, input index per position)."""
    import torch
    n = x.numel()
    perm = torch.empty(n, dtype=torch.int64, device=x.device)
    _check(lib().gl_morton_order(ctx.handle, _ptr(x), _ptr(y), n, perm.data_ptr(), _stream(stream)),
           "gl_morton_order")
    return perm


PRECISION_CLASSES = ("fp64", "fp32", "bf16x6", "bf16x3", "bf16", "fp16x3", "fp16")


def gl_precision_stats(ctx: Context) -> dict:
    """Tiles and trailing-update work per precision class of the last mixed evaluation."""
    tiles = (_I64 * len(PRECISION_CLASSES))()
    work = (_D * len(PRECISION_CLASSES))()
    thr = (_D * 4)()
    _check(lib().gl_precision_stats(ctx.handle, tiles, work, thr), "gl_precision_stats")
    tot = sum(work) or 1.0
    out = {c: {"tiles": int(tiles[i]), "work_frac": work[i] / tot} for i, c in enumerate(PRECISION_CLASSES)}
    out["thresholds"] = {"rho": thr[0], "tol_64": thr[1], "tol_hi": thr[2], "tol_lo": thr[3]}
    return out
