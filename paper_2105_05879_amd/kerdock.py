"""Python binding of the gfx950 Kerdock library (``libkerdock.so``).

Argument marshalling only: every step of the transform runs in the HIP
kernels behind the C ABI declared in ``include/kerdock.h``.  The functions
keep the C names.  Tensors must be contiguous CUDA (HIP) tensors of the
documented dtype on the current device; streams default to torch's current
stream.  There is no CPU fallback: without the built library every call
raises.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkerdock.so")

KERDOCK_F32, KERDOCK_BF16, KERDOCK_FP8E4M3 = 0, 1, 2
DTYPES = {"f32": KERDOCK_F32, "fp32": KERDOCK_F32, "bf16": KERDOCK_BF16,
          "fp8": KERDOCK_FP8E4M3, "fp8e4m3": KERDOCK_FP8E4M3}
STATUS = {0: "OK", -1: "INVALID_ARG", -2: "UNSUPPORTED_N", -3: "OOM", -4: "HIP", -5: "NOT_PREPARED"}


class KerdockError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (STATUS.get(code, "?"), code, msg))
        self.code = code


SHARED_TILE = 64      # KERDOCK_SHARED_TILE


class ApplyParams(ctypes.Structure):
    _fields_ = [("J", ctypes.c_int32), ("K", ctypes.c_int32), ("seed", ctypes.c_uint64),
                ("t0", ctypes.c_int64), ("tau", ctypes.c_float),
                ("dbg_samples", ctypes.c_void_p), ("dbg_coef", ctypes.c_void_p),
                ("dbg_mu", ctypes.c_void_p), ("dbg_survivors", ctypes.c_void_p),
                ("dbg_values", ctypes.c_void_p), ("kernel_ms", ctypes.POINTER(ctypes.c_float)),
                ("chunk", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int32), ("n", ctypes.c_int32), ("k", ctypes.c_int32),
                ("d", ctypes.c_int32), ("L", ctypes.c_int64), ("pitch", ctypes.c_int32),
                ("field_poly", ctypes.c_uint32), ("dtype", ctypes.c_int),
                ("table_bytes", ctypes.c_size_t), ("build_ms", ctypes.c_float)]


EXPORTS = {
    "kerdock_prepare": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "kerdock_sparse_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_float, ctypes.c_int,
                                            ctypes.POINTER(ApplyParams), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_sparse_apply_static": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                   ctypes.c_float, ctypes.c_int,
                                                   ctypes.POINTER(ApplyParams), ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_reserve": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_int]),
    "kerdock_query": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Info)]),
    "kerdock_read_columns": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                            ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_debug_signs": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    "kerdock_row_scales": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "kerdock_mlp_create": (ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                          ctypes.c_uint64, ctypes.POINTER(ctypes.c_void_p)]),
    "kerdock_mlp_param_count": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "kerdock_mlp_get_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_mlp_set_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_mlp_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                           ctypes.c_void_p]),
    "kerdock_mlp_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                              ctypes.c_float, ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p,
                                              ctypes.c_void_p]),
    "kerdock_mlp_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "kerdock_features": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p,
                                        ctypes.c_void_p]),
    "kerdock_learned_attach": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_learned_apply": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_float,
                                             ctypes.c_int, ctypes.POINTER(ApplyParams), ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_sparse_apply_shared": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                                   ctypes.c_float, ctypes.c_int,
                                                   ctypes.POINTER(ApplyParams), ctypes.c_void_p,
                                                   ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_theory_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                             ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                             ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "kerdock_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                        ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)]),
    "kerdock_multi_create": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ApplyParams), ctypes.c_float,
                                            ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                            ctypes.POINTER(ctypes.c_void_p)]),
    "kerdock_multi_run": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_multi_set_position": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    "kerdock_multi_graph_launch": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "kerdock_multi_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)]),
    "kerdock_multi_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "kerdock_sparse_apply_multi": (ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int),
                                                  ctypes.POINTER(ApplyParams), ctypes.c_float,
                                                  ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_void_p),
                                                  ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                                                  ctypes.c_void_p]),
    "kerdock_last_error": (ctypes.c_char_p, []),
}

_lib = None


def lib():
    """Load libkerdock.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkerdock.so is not built: run paper_2105_05879_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in EXPORTS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != 0:
        raise KerdockError(rc, lib().kerdock_last_error().decode())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t, dtype, name):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise TypeError("%s must be a contiguous CUDA tensor of dtype %s" % (name, dtype))
    return ctypes.c_void_p(t.data_ptr())


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _check_x(X, n, name="X"):
    """X must be a (B, n) FP32 CUDA tensor: the kernels read B n floats."""
    _dev(X, torch.float32, name)
    if X.dim() != 2 or X.shape[1] != n:
        raise ValueError("%s must have shape (batch, %d), got %s" % (name, n, tuple(X.shape)))


def _check_out(out, B, s_max, device):
    """Caller-supplied outputs: idx (B, s_max) int32, val (B, s_max) FP32,
    cnt (B,) int32, contiguous, on X's device."""
    if len(out) != 3:
        raise ValueError("out must be (idx, val, cnt)")
    for t, dt, shp, name in zip(out, (torch.int32, torch.float32, torch.int32),
                                ((B, s_max), (B, s_max), (B,)), ("idx", "val", "cnt")):
        _dev(t, dt, name)
        if tuple(t.shape) != shp or t.device != device:
            raise ValueError("%s must have shape %s on %s, got %s on %s" % (name, shp, device, tuple(t.shape),
                                                                           t.device))


class Handle:
    """A prepared matrix: owns the device tables until destroyed."""

    def __init__(self, ptr, info):
        self.ptr = ptr
        self.info = info

    @property
    def m(self):
        return self.info.m

    @property
    def n(self):
        return self.info.n

    @property
    def L(self):
        return self.info.L

    def destroy(self):
        if self.ptr:
            _check(lib().kerdock_destroy(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def kerdock_prepare(A, dtype="f32", stream=None):
    """Build the Kerdock sketch tables of A (m x n FP32 CUDA tensor)."""
    A = A if isinstance(A, torch.Tensor) else torch.as_tensor(A)
    m, n = A.shape
    out = ctypes.c_void_p()
    _check(lib().kerdock_prepare(_dev(A, torch.float32, "A"), m, n, DTYPES.get(dtype, dtype),
                                 _stream(stream), ctypes.byref(out)))
    return Handle(out, kerdock_query(out))


def kerdock_query(h):
    ptr = h.ptr if isinstance(h, Handle) else h
    info = Info()
    _check(lib().kerdock_query(ptr, ctypes.byref(info)))
    return info


def kerdock_reserve(h, batch, J, K, s_max):
    _check(lib().kerdock_reserve(h.ptr, batch, J, K, s_max))


def _sparse_apply(entry, h, X, eps, s_max, J, K, seed, t0, tau, out, debug, stream, kernel_ms, chunk):
    """Shared body of the two streaming entry points."""
    _check_x(X, h.n)
    B = X.shape[0]
    dev = X.device
    if out is None:
        out = (torch.empty((B, s_max), dtype=torch.int32, device=dev),
               torch.empty((B, s_max), dtype=torch.float32, device=dev),
               torch.empty((B,), dtype=torch.int32, device=dev))
    _check_out(out, B, s_max, dev)
    idx, val, cnt = out
    p = ApplyParams(J=J, K=K, seed=seed, t0=t0, tau=tau, chunk=chunk)
    if kernel_ms is not None:          # a ctypes c_float * 4 filled by the call
        p.kernel_ms = ctypes.cast(kernel_ms, ctypes.POINTER(ctypes.c_float))
    dbg = None
    if debug:
        N = J * K
        dbg = {"samples": torch.empty((B, N), dtype=torch.int32, device=dev),
               "coef": torch.empty((B, N), dtype=torch.float32, device=dev),
               "mu": torch.empty((B, h.m), dtype=torch.float32, device=dev),
               "survivors": torch.empty((B, s_max), dtype=torch.int32, device=dev),
               "values": torch.empty((B, s_max), dtype=torch.float32, device=dev)}
        p.dbg_samples = dbg["samples"].data_ptr()
        p.dbg_coef = dbg["coef"].data_ptr()
        p.dbg_mu = dbg["mu"].data_ptr()
        p.dbg_survivors = dbg["survivors"].data_ptr()
        p.dbg_values = dbg["values"].data_ptr()
    _check(getattr(lib(), entry)(h.ptr, _dev(X, torch.float32, "X"), B, float(eps), s_max,
                                 ctypes.byref(p), _dev(idx, torch.int32, "idx"),
                                 _dev(val, torch.float32, "val"), _dev(cnt, torch.int32, "cnt"),
                                 _stream(stream)))
    if debug:
        return idx, val, cnt, dbg
    return idx, val, cnt


def kerdock_sparse_apply(h, X, eps, s_max, J, K, seed, t0=0, tau=0.0, out=None, debug=False,
                         stream=None, kernel_ms=None, chunk=0):
    """h_eps(Ax) on the s_max rows of largest median-of-means estimate.

    Returns (idx [B, s_max] int32, val [B, s_max] f32, cnt [B] int32) and,
    with debug=True, a dict of samples, coef, mu, survivors, values.
    kernel_ms: optional (ctypes.c_float * 4)() that receives the durations
    of the four kernels, timed with HIP events on the call's stream."""
    return _sparse_apply("kerdock_sparse_apply", h, X, eps, s_max, J, K, seed, t0, tau, out, debug, stream,
                         kernel_ms, chunk)


def kerdock_sparse_apply_static(h, X, eps, s_max, J, K, seed, t0=0, tau=0.0, out=None, debug=False,
                                stream=None, chunk=0):
    """As kerdock_sparse_apply, with the workspace in the library's fixed
    device scratch (KERDOCK_STATIC_SCRATCH_BYTES per device): the call
    allocates nothing in the library (pass `out` to avoid torch allocating
    the outputs too); calls that overlap on one device race."""
    return _sparse_apply("kerdock_sparse_apply_static", h, X, eps, s_max, J, K, seed, t0, tau, out, debug, stream,
                         None, chunk)


def kerdock_sparse_apply_shared(h, X, eps, s_max, J, K, seed, t0=0, tau=0.0, out=None, debug=False,
                                stream=None, kernel_ms=None):
    """As kerdock_sparse_apply, with the draws shared by groups of
    SHARED_TILE consecutive rows of X (stream position t0 + group);
    kernel_ms: [coefficients, matrix product, select, survivors]."""
    return _sparse_apply("kerdock_sparse_apply_shared", h, X, eps, s_max, J, K, seed, t0, tau, out, debug,
                         stream, kernel_ms, 0)


def kerdock_read_columns(h, ells, stream=None):
    """Dequantised table columns T[l] (times the FP8 row scale), [count, m]."""
    if not (isinstance(ells, torch.Tensor) and ells.is_cuda):
        raise TypeError("ells must be a CUDA tensor")
    ells = ells.to(torch.int32).contiguous().view(-1)
    out = torch.empty((ells.numel(), h.m), dtype=torch.float32, device=ells.device)
    _check(lib().kerdock_read_columns(h.ptr, _ptr(ells), ells.numel(), _ptr(out), _stream(stream)))
    return out


def kerdock_debug_signs(h, b):
    words = max(1, h.info.d // 32)
    buf = (ctypes.c_uint32 * words)()
    _check(lib().kerdock_debug_signs(h.ptr, b, buf))
    return list(buf)


def kerdock_row_scales(h, stream=None):
    out = torch.empty((h.m,), dtype=torch.float32, device="cuda")
    _check(lib().kerdock_row_scales(h.ptr, _ptr(out), _stream(stream)))
    return out


def kerdock_autotune(h, X, J, K, stream=None):
    """Time the gather shapes on X and keep the fastest in the handle.
    Returns (chunk, unroll, ms)."""
    _check_x(X, h.n)
    c, u, ms = ctypes.c_int(), ctypes.c_int(), ctypes.c_float()
    _check(lib().kerdock_autotune(h.ptr, _dev(X, torch.float32, "X"), X.shape[0], J, K, _stream(stream),
                                  ctypes.byref(c), ctypes.byref(u), ctypes.byref(ms)))
    return c.value, u.value, ms.value


def _arr(ctype, vals):
    return (ctype * len(vals))(*vals)


class MultiPlan:
    """Batched form: several handles streamed in one persistent launch.
    Owns the output tensors it binds (idx, val, cnt per handle)."""

    def __init__(self, ptr, handles, Xs, outs):
        self.ptr = ptr
        self.handles = handles       # keep the handles and bound tensors alive
        self.Xs = Xs
        self.outs = outs

    def destroy(self):
        if self.ptr:
            _check(lib().kerdock_multi_destroy(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def _multi_args(handles, Xs, params, s_max, outs):
    nh = len(handles)
    if not (len(Xs) == nh and len(params) == nh and len(s_max) == nh and (outs is None or len(outs) == nh)):
        raise ValueError("handles, Xs, params, s_max (and outs) must have one entry per handle")
    for h, X in zip(handles, Xs):
        _check_x(X, h.n)
    if outs is not None:
        for X, sm, o in zip(Xs, s_max, outs):
            _check_out(o, X.shape[0], sm, X.device)
    if outs is None:
        outs = [(torch.empty((X.shape[0], sm), dtype=torch.int32, device=X.device),
                 torch.empty((X.shape[0], sm), dtype=torch.float32, device=X.device),
                 torch.empty((X.shape[0],), dtype=torch.int32, device=X.device))
                for X, sm in zip(Xs, s_max)]
    ps = (ApplyParams * nh)()
    for q, p in enumerate(params):
        ps[q] = ApplyParams(J=p["J"], K=p["K"], seed=p.get("seed", 0), t0=p.get("t0", 0),
                            tau=p.get("tau", 0.0), chunk=p.get("chunk", 0))
    hs = _arr(ctypes.c_void_p, [h.ptr.value if isinstance(h.ptr, ctypes.c_void_p) else h.ptr for h in handles])
    xp = _arr(ctypes.c_void_p, [_dev(X, torch.float32, "X").value for X in Xs])
    bt = _arr(ctypes.c_int, [X.shape[0] for X in Xs])
    sm = _arr(ctypes.c_int, list(s_max))
    oi = _arr(ctypes.c_void_p, [_dev(o[0], torch.int32, "idx").value for o in outs])
    ov = _arr(ctypes.c_void_p, [_dev(o[1], torch.float32, "val").value for o in outs])
    oc = _arr(ctypes.c_void_p, [_dev(o[2], torch.int32, "cnt").value for o in outs])
    return nh, hs, xp, bt, ps, sm, oi, ov, oc, outs


def kerdock_multi_create(handles, Xs, params, eps, s_max, outs=None):
    """Bind per-handle inputs X[q], parameters (dicts with J, K, seed, t0, tau)
    and outputs into a plan; returns a MultiPlan (outputs in plan.outs)."""
    nh, hs, xp, bt, ps, sm, oi, ov, oc, outs = _multi_args(handles, Xs, params, s_max, outs)
    out = ctypes.c_void_p()
    _check(lib().kerdock_multi_create(hs, nh, xp, bt, ps, float(eps), sm, oi, ov, oc, ctypes.byref(out)))
    return MultiPlan(out, list(handles), list(Xs), outs)


def kerdock_multi_run(plan, stream=None):
    _check(lib().kerdock_multi_run(plan.ptr, _stream(stream)))


def kerdock_multi_set_position(plan, t0s):
    _check(lib().kerdock_multi_set_position(plan.ptr, _arr(ctypes.c_int64, list(t0s))))


def kerdock_multi_graph_launch(plan, stream=None):
    _check(lib().kerdock_multi_graph_launch(plan.ptr, _stream(stream)))


def kerdock_multi_autotune(plan, stream=None):
    u = ctypes.c_int()
    _check(lib().kerdock_multi_autotune(plan.ptr, _stream(stream), ctypes.byref(u)))
    return u.value


def kerdock_multi_destroy(plan):
    plan.destroy()


def kerdock_sparse_apply_multi(handles, Xs, params, eps, s_max, outs=None, stream=None):
    """One-shot batched call; returns [(idx, val, cnt)] per handle."""
    nh, hs, xp, bt, ps, sm, oi, ov, oc, outs = _multi_args(handles, Xs, params, s_max, outs)
    _check(lib().kerdock_sparse_apply_multi(hs, nh, xp, bt, ps, float(eps), sm, oi, ov, oc, _stream(stream)))
    return outs


class MLP:
    """The learned-proposal network (device parameters, Adam state)."""

    def __init__(self, ptr, dims):
        self.ptr = ptr
        self.dims = dims

    @property
    def param_count(self):
        c = ctypes.c_size_t()
        _check(lib().kerdock_mlp_param_count(self.ptr, ctypes.byref(c)))
        return c.value

    def destroy(self):
        if self.ptr:
            _check(lib().kerdock_mlp_destroy(self.ptr))
            self.ptr = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def kerdock_mlp_create(d_in, h1, h2, d_out, seed=0):
    out = ctypes.c_void_p()
    _check(lib().kerdock_mlp_create(d_in, h1, h2, d_out, seed, ctypes.byref(out)))
    return MLP(out, (d_in, h1, h2, d_out))


def kerdock_mlp_get_params(net):
    import numpy as np
    buf = np.zeros(net.param_count, dtype=np.float32)
    _check(lib().kerdock_mlp_get_params(net.ptr, buf.ctypes.data_as(ctypes.c_void_p)))
    return buf


def kerdock_mlp_set_params(net, params):
    import numpy as np
    buf = np.ascontiguousarray(params, dtype=np.float32)
    assert buf.size == net.param_count
    _check(lib().kerdock_mlp_set_params(net.ptr, buf.ctypes.data_as(ctypes.c_void_p)))


def kerdock_mlp_forward(net, F, stream=None):
    _check_x(F, net.dims[0], "F")
    Z = torch.empty((F.shape[0], net.dims[3]), dtype=torch.float32, device=F.device)
    _check(lib().kerdock_mlp_forward(net.ptr, _dev(F, torch.float32, "F"), F.shape[0], _ptr(Z), _stream(stream)))
    return Z


def kerdock_mlp_train_step(net, F, Y, lr, pos_weight, want_grads=False, stream=None):
    """One training step; returns (loss tensor [1], grads or None)."""
    _check_x(F, net.dims[0], "F")
    if not (isinstance(Y, torch.Tensor) and Y.dim() == 2 and tuple(Y.shape) == (F.shape[0], net.dims[3])):
        raise ValueError("Y must have shape (batch, %d)" % net.dims[3])
    loss = torch.empty((1,), dtype=torch.float32, device=F.device)
    grads = torch.empty((net.param_count,), dtype=torch.float32, device=F.device) if want_grads else None
    _check(lib().kerdock_mlp_train_step(net.ptr, _dev(F, torch.float32, "F"), _dev(Y, torch.uint8, "Y"),
                                        F.shape[0], float(lr), float(pos_weight), _ptr(loss), _ptr(grads),
                                        _stream(stream)))
    return loss, grads


def kerdock_features(h, X, stream=None):
    _check_x(X, h.n)
    F = torch.empty((X.shape[0], h.info.d), dtype=torch.float32, device=X.device)
    _check(lib().kerdock_features(h.ptr, _dev(X, torch.float32, "X"), X.shape[0], _ptr(F), _stream(stream)))
    return F


def kerdock_learned_attach(h, net):
    _check(lib().kerdock_learned_attach(h.ptr, net.ptr))
    h._net = net                      # keep the network alive with the handle


def kerdock_learned_apply(h, X, eps, s_max, J, K, seed, t0=0, tau=0.0, out=None, stream=None, chunk=0,
                          candidates=False):
    """Returns (idx, val, cnt, fallback), and with candidates=True also the
    candidate set C of every row ([B, s_max] int32, ascending, -1 padded)."""
    _check_x(X, h.n)
    B = X.shape[0]
    dev = X.device
    if out is None:
        out = (torch.empty((B, s_max), dtype=torch.int32, device=dev),
               torch.empty((B, s_max), dtype=torch.float32, device=dev),
               torch.empty((B,), dtype=torch.int32, device=dev))
    _check_out(out, B, s_max, dev)
    fb = torch.empty((B,), dtype=torch.int32, device=dev)
    p = ApplyParams(J=J, K=K, seed=seed, t0=t0, tau=tau, chunk=chunk)
    cand = None
    if candidates:
        cand = torch.empty((B, s_max), dtype=torch.int32, device=dev)
        p.dbg_survivors = cand.data_ptr()
    _check(lib().kerdock_learned_apply(h.ptr, _dev(X, torch.float32, "X"), B, float(eps), s_max, ctypes.byref(p),
                                       _ptr(out[0]), _ptr(out[1]), _ptr(out[2]), _ptr(fb), _stream(stream)))
    if candidates:
        return out[0], out[1], out[2], fb, cand
    return out[0], out[1], out[2], fb


def kerdock_theory_params(h, eps, delta, eta):
    """Theorem 5's (J, K), tau = (eps + delta)/2 and |A|_{2->inf}^2."""
    J, K, tau, nrm = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_float(), ctypes.c_float()
    _check(lib().kerdock_theory_params(h.ptr, float(eps), float(delta), float(eta), ctypes.byref(J),
                                       ctypes.byref(K), ctypes.byref(tau), ctypes.byref(nrm)))
    return J.value, K.value, tau.value, nrm.value
