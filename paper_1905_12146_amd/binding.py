"""ctypes binding of libphylograd (argument marshalling only).

Each ``pg_*`` function of include/phylograd.h has a Python function of the
same name taking NumPy arrays (host memory) or integer device addresses
(device variants); ``Context`` is a small owner object over them.  There is
no fallback: if the shared library is missing or fails to load, every call
raises ``PhyloGradError``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
# PHYLOGRAD_LIB overrides the in-tree library (e.g. a build with other flags)
LIB_PATH = os.environ.get("PHYLOGRAD_LIB") or os.path.join(HERE, "libphylograd.so")

PG_OK = 0
PG_E_INVALID = -1
PG_E_TREE = -2
PG_E_MODEL = -3
PG_E_PATTERNS = -4
PG_E_STATE = -5
PG_E_OOM = -6
PG_E_DEVICE = -7
PG_E_ZERO_LIK = -8
PG_E_UNSUPPORTED = -9

PG_FP64 = 0
PG_FP32 = 1
PG_SPLIT_BF16 = 2

PG_K_PMAT, PG_K_POST, PG_K_ROOT, PG_K_PRE, PG_K_GSUM = range(5)
PG_K_COUNT = 5
PG_NOALLOC_MAX_BYTES = 64 << 20
KERNEL_NAMES = ("pmat", "post", "root", "pre", "gsum")

ERROR_NAMES = {
    PG_E_INVALID: "PG_E_INVALID", PG_E_TREE: "PG_E_TREE", PG_E_MODEL: "PG_E_MODEL",
    PG_E_PATTERNS: "PG_E_PATTERNS", PG_E_STATE: "PG_E_STATE", PG_E_OOM: "PG_E_OOM",
    PG_E_DEVICE: "PG_E_DEVICE", PG_E_ZERO_LIK: "PG_E_ZERO_LIK", PG_E_UNSUPPORTED: "PG_E_UNSUPPORTED",
}

# (name, restype, argtypes) for every exported entry point of the header
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_SIGNATURES = [
    ("pg_create", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(_vp)]),
    ("pg_destroy", None, [_vp]),
    ("pg_last_error", ctypes.c_char_p, [_vp]),
    ("pg_set_stream", ctypes.c_int, [_vp, _vp]),
    ("pg_set_tree", ctypes.c_int, [_vp, _i32, _vp]),
    ("pg_set_patterns", ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
    ("pg_set_model", ctypes.c_int, [_vp, _i32, _vp, _vp, _i32, _vp, _vp]),
    ("pg_set_branch_models", ctypes.c_int, [_vp, _i32, _vp, _vp]),
    ("pg_logL_and_grad", ctypes.c_int, [_vp, _vp, _vp, _vp]),
    ("pg_logL", ctypes.c_int, [_vp, _vp, _vp]),
    ("pg_logL_update", ctypes.c_int, [_vp, _i32, _vp, _vp, _vp]),
    ("pg_grad", ctypes.c_int, [_vp, _vp]),
    ("pg_hessian_diag", ctypes.c_int, [_vp, _vp, _vp]),
    ("pg_logL_and_grad_device", ctypes.c_int, [_vp, _vp, _vp, _vp]),
    ("pg_grad_device", ctypes.c_int, [_vp, _vp]),
    ("pg_logL_and_grad_noalloc", ctypes.c_int, [_vp, _vp, _vp, _vp]),
    ("pg_status", ctypes.c_int, [_vp]),
    ("pg_set_timing", ctypes.c_int, [_vp, ctypes.c_int]),
    ("pg_get_timing", ctypes.c_int, [_vp, _vp, _vp]),
    ("pg_device_bytes", _i64, [_vp]),
    ("pg_footprint_bytes", _i64, [_i32, _i32, _i32, _i32, ctypes.c_int]),
    ("pg_eigensystem", ctypes.c_int, [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    ("pg_server_create", ctypes.c_int, [ctypes.c_int, ctypes.c_int, _i64, _i32, ctypes.POINTER(_vp)]),
    ("pg_server_destroy", None, [_vp]),
    ("pg_server_last_error", ctypes.c_char_p, [_vp]),
    ("pg_server_open", ctypes.c_int, [_vp, _i32, _vp, _i32, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp,
                                      ctypes.POINTER(_i64)]),
    ("pg_server_submit", ctypes.c_int, [_vp, _i64, _vp, _i32, ctypes.POINTER(_i64)]),
    ("pg_server_wait", ctypes.c_int, [_vp, _i64, _vp, _vp, ctypes.POINTER(_i64)]),
    ("pg_server_close", ctypes.c_int, [_vp, _i64]),
    ("pg_server_stats", ctypes.c_int, [_vp, _vp, _i32]),
]
EXPORTED = [name for name, _, _ in _SIGNATURES]


class PhyloGradError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load libphylograd.so (built by paper_1905_12146_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise PhyloGradError(PG_E_DEVICE, f"{LIB_PATH} is missing: run paper_1905_12146_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in _SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(ctx, code):
    if code != PG_OK:
        msg = load().pg_last_error(ctx).decode(errors="replace")
        raise PhyloGradError(code, msg)


# -- thin wrappers with the header's names ----------------------------------

def pg_create(device=0, precision=PG_FP64):
    h = ctypes.c_void_p()
    code = load().pg_create(int(device), int(precision), ctypes.byref(h))
    _check(None, code)
    return h


def pg_destroy(ctx):
    load().pg_destroy(ctx)


def pg_last_error(ctx=None):
    return load().pg_last_error(ctx).decode(errors="replace")


def pg_set_stream(ctx, stream_handle):
    _check(ctx, load().pg_set_stream(ctx, ctypes.c_void_p(stream_handle or 0) if stream_handle else None))


def pg_set_tree(ctx, parent):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    n = (len(parent) + 1) // 2
    _check(ctx, load().pg_set_tree(ctx, n, _ptr(parent)))


def pg_set_patterns(ctx, tip_masks, weights, n_states):
    tip_masks = np.ascontiguousarray(tip_masks, dtype=np.uint64)
    weights = np.ascontiguousarray(weights, dtype=np.float64)
    if tip_masks.ndim != 2 or weights.shape != (tip_masks.shape[1],):
        raise PhyloGradError(PG_E_INVALID, "tip_masks must be [N, S] and weights [S]")
    _check(ctx, load().pg_set_patterns(ctx, tip_masks.shape[1], int(n_states), _ptr(tip_masks),
                                       _ptr(weights)))


def pg_set_model(ctx, Q, pi, rates, cat_weights):
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    pi = np.ascontiguousarray(pi, dtype=np.float64)
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    cat_weights = np.ascontiguousarray(cat_weights, dtype=np.float64)
    if Q.ndim != 2 or Q.shape[0] != Q.shape[1] or pi.shape != (Q.shape[0],) \
            or rates.shape != cat_weights.shape or rates.ndim != 1:
        raise PhyloGradError(PG_E_INVALID, "Q [m, m], pi [m], rates and weights [K] expected")
    _check(ctx, load().pg_set_model(ctx, Q.shape[0], _ptr(Q), _ptr(pi), len(rates), _ptr(rates),
                                    _ptr(cat_weights)))


def pg_set_branch_models(ctx, Qs, model_of_branch):
    """Qs [n_models, m, m] and model_of_branch [2N-2]; Qs = None clears."""
    if Qs is None:
        _check(ctx, load().pg_set_branch_models(ctx, 0, None, None))
        return
    Qs = np.ascontiguousarray(Qs, dtype=np.float64)
    model = np.ascontiguousarray(model_of_branch, dtype=np.int32)
    if Qs.ndim != 3 or Qs.shape[1] != Qs.shape[2] or model.ndim != 1:
        raise PhyloGradError(PG_E_INVALID, "Qs [n_models, m, m] and model_of_branch [2N-2] expected")
    _check(ctx, load().pg_set_branch_models(ctx, Qs.shape[0], _ptr(Qs), model.ctypes.data))


def pg_logL_update(ctx, branches, t_new):
    """logL after setting t[branches[i]] = t_new[i] (partial re-evaluation)."""
    b = np.ascontiguousarray(branches, dtype=np.int32)
    tn = np.ascontiguousarray(t_new, dtype=np.float64)
    if b.shape != tn.shape or b.ndim != 1:
        raise PhyloGradError(PG_E_INVALID, "branches and t_new must be vectors of equal length")
    logL = ctypes.c_double()
    _check(ctx, load().pg_logL_update(ctx, len(b), b.ctypes.data, _ptr(tn), ctypes.byref(logL)))
    return logL.value


def _lengths(t, n_branches):
    """t as contiguous FP64; n_branches None (no tree yet) leaves the call-order
    check to the library."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    if n_branches is not None and t.shape != (n_branches,):
        raise PhyloGradError(PG_E_INVALID, f"t must have {n_branches} entries")
    return t


def pg_logL_and_grad(ctx, t, n_branches):
    t = _lengths(t, n_branches)
    logL = np.zeros(1)
    grad = np.zeros(len(t))
    _check(ctx, load().pg_logL_and_grad(ctx, _ptr(t), _ptr(logL), _ptr(grad)))
    return float(logL[0]), grad


def pg_logL(ctx, t, n_branches):
    t = _lengths(t, n_branches)
    logL = np.zeros(1)
    _check(ctx, load().pg_logL(ctx, _ptr(t), _ptr(logL)))
    return float(logL[0])


def pg_grad(ctx, n_branches):
    grad = np.zeros(n_branches)
    _check(ctx, load().pg_grad(ctx, _ptr(grad)))
    return grad


def pg_hessian_diag(ctx, n_branches):
    grad = np.zeros(n_branches)
    hess = np.zeros(n_branches)
    _check(ctx, load().pg_hessian_diag(ctx, _ptr(grad), _ptr(hess)))
    return grad, hess


def pg_logL_and_grad_device(ctx, d_t, d_logL, d_grad):
    """Device addresses (ints); asynchronous on the context's stream."""
    _check(ctx, load().pg_logL_and_grad_device(ctx, ctypes.c_void_p(d_t), ctypes.c_void_p(d_logL),
                                               ctypes.c_void_p(d_grad) if d_grad else None))


def pg_logL_and_grad_noalloc(ctx, d_t, d_logL, d_grad):
    """Device addresses (ints); asynchronous on the context's stream; every
    device buffer in the library's per-device scratch array."""
    _check(ctx, load().pg_logL_and_grad_noalloc(ctx, ctypes.c_void_p(d_t), ctypes.c_void_p(d_logL),
                                                ctypes.c_void_p(d_grad) if d_grad else None))


def pg_grad_device(ctx, d_grad):
    """Device address (int); asynchronous on the context's stream."""
    _check(ctx, load().pg_grad_device(ctx, ctypes.c_void_p(d_grad)))


def pg_status(ctx):
    return load().pg_status(ctx)


def pg_set_timing(ctx, enable):
    _check(ctx, load().pg_set_timing(ctx, 1 if enable else 0))


def pg_get_timing(ctx):
    ms = np.zeros(PG_K_COUNT)
    n = np.zeros(PG_K_COUNT, dtype=np.int64)
    _check(ctx, load().pg_get_timing(ctx, _ptr(ms), _ptr(n)))
    return {KERNEL_NAMES[k]: (float(ms[k]), int(n[k])) for k in range(PG_K_COUNT)}


def pg_device_bytes(ctx):
    return int(load().pg_device_bytes(ctx))


def pg_footprint_bytes(n_tips, n_patterns, n_states, n_cats, precision=PG_FP64):
    return int(load().pg_footprint_bytes(n_tips, n_patterns, n_states, n_cats, precision))


def pg_eigensystem(Q):
    """(V, Vinv, re, im, kind, cond, resid) of the split-BF16 eigen route."""
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    m = Q.shape[0]
    V = np.zeros((m, m))
    Vinv = np.zeros((m, m))
    re = np.zeros(m)
    im = np.zeros(m)
    kind = np.zeros(m, dtype=np.int32)
    cond = ctypes.c_double()
    resid = ctypes.c_double()
    code = load().pg_eigensystem(m, Q.ctypes.data, V.ctypes.data, Vinv.ctypes.data, re.ctypes.data,
                                 im.ctypes.data, kind.ctypes.data, ctypes.byref(cond), ctypes.byref(resid))
    if code != PG_OK:
        raise PhyloGradError(code, "pg_eigensystem")
    return V, Vinv, re, im, kind, cond.value, resid.value


# -- serving -------------------------------------------------------------------

SRV_STAT_NAMES = ("steps", "calls", "max_batch", "admitted_total", "admitted_now", "waiting_now",
                  "in_use_bytes", "peak_bytes", "max_waiting", "peak_held")


def _check_srv(srv, code):
    if code != PG_OK:
        raise PhyloGradError(code, load().pg_server_last_error(srv).decode(errors="replace"))


def pg_server_create(device=0, precision=PG_FP32, hbm_budget_bytes=32 << 30, max_sessions=64):
    h = ctypes.c_void_p()
    code = load().pg_server_create(int(device), int(precision), int(hbm_budget_bytes), int(max_sessions),
                                   ctypes.byref(h))
    if code != PG_OK:
        raise PhyloGradError(code, load().pg_last_error(None).decode(errors="replace") or "pg_server_create")
    return h


def pg_server_destroy(srv):
    load().pg_server_destroy(srv)


def pg_server_last_error(srv):
    return load().pg_server_last_error(srv).decode(errors="replace")


def pg_server_open(srv, parent, tip_masks, weights, Q, pi, rates, cat_weights):
    parent = np.ascontiguousarray(parent, dtype=np.int32)
    tip_masks = np.ascontiguousarray(tip_masks, dtype=np.uint64)
    weights = np.ascontiguousarray(weights, dtype=np.float64)
    Q = np.ascontiguousarray(Q, dtype=np.float64)
    pi = np.ascontiguousarray(pi, dtype=np.float64)
    rates = np.ascontiguousarray(rates, dtype=np.float64)
    cat_weights = np.ascontiguousarray(cat_weights, dtype=np.float64)
    sid = ctypes.c_int64()
    _check_srv(srv, load().pg_server_open(srv, (len(parent) + 1) // 2, _ptr(parent), tip_masks.shape[1],
                                          Q.shape[0], _ptr(tip_masks), _ptr(weights), _ptr(Q), _ptr(pi),
                                          len(rates), _ptr(rates), _ptr(cat_weights), ctypes.byref(sid)))
    return sid.value


def pg_server_submit(srv, session, t, want_grad=True):
    t = np.ascontiguousarray(t, dtype=np.float64)
    tk = ctypes.c_int64()
    _check_srv(srv, load().pg_server_submit(srv, int(session), _ptr(t), 1 if want_grad else 0,
                                            ctypes.byref(tk)))
    return tk.value


def pg_server_wait(srv, ticket, n_branches):
    """Returns (status, logL, grad, latency_ns); status is a PG_* code."""
    logL = np.zeros(1)
    grad = np.zeros(n_branches)
    lat = ctypes.c_int64()
    code = load().pg_server_wait(srv, int(ticket), _ptr(logL), _ptr(grad), ctypes.byref(lat))
    return code, float(logL[0]), grad, lat.value


def pg_server_close(srv, session):
    _check_srv(srv, load().pg_server_close(srv, int(session)))


def pg_server_stats(srv):
    out = np.zeros(len(SRV_STAT_NAMES), dtype=np.int64)
    _check_srv(srv, load().pg_server_stats(srv, _ptr(out), len(out)))
    return dict(zip(SRV_STAT_NAMES, out.tolist()))


class Context:
    """Owner of one pg_ctx: tree, patterns and model in, logL and gradients out."""

    def __init__(self, device=0, precision=PG_FP64):
        self.handle = pg_create(device, precision)
        self.precision = precision
        self.n_branches = None

    def close(self):
        if self.handle:
            pg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_tree(self, parent):
        pg_set_tree(self.handle, parent)
        self.n_branches = len(parent) - 1

    def set_patterns(self, tip_masks, weights, n_states):
        pg_set_patterns(self.handle, tip_masks, weights, n_states)

    def set_model(self, Q, pi, rates, cat_weights):
        pg_set_model(self.handle, Q, pi, rates, cat_weights)

    def set_branch_models(self, Qs, model_of_branch):
        if Qs is not None and len(model_of_branch) != (self.n_branches or 0):
            raise PhyloGradError(PG_E_INVALID, f"model_of_branch needs {self.n_branches} entries")
        pg_set_branch_models(self.handle, Qs, model_of_branch)

    def set_stream(self, stream_handle):
        pg_set_stream(self.handle, stream_handle)

    def set_workload(self, w):
        """Tree, patterns and model of a synth.Workload."""
        self.set_tree(w.parent)
        self.set_patterns(w.tip_masks(), w.weights, w.n_states)
        self.set_model(w.Q, w.pi, w.rates, w.cat_weights)

    def logL_and_grad(self, t):
        return pg_logL_and_grad(self.handle, t, self.n_branches)

    def logL(self, t):
        return pg_logL(self.handle, t, self.n_branches)

    def logL_update(self, branches, t_new):
        return pg_logL_update(self.handle, branches, t_new)

    def grad(self):
        return pg_grad(self.handle, self.n_branches or 0)

    def hessian_diag(self):
        return pg_hessian_diag(self.handle, self.n_branches or 0)

    def logL_and_grad_device(self, d_t, d_logL, d_grad):
        pg_logL_and_grad_device(self.handle, d_t, d_logL, d_grad)

    def grad_device(self, d_grad):
        pg_grad_device(self.handle, d_grad)

    def logL_and_grad_noalloc(self, d_t, d_logL, d_grad):
        pg_logL_and_grad_noalloc(self.handle, d_t, d_logL, d_grad)

    def status(self):
        return pg_status(self.handle)

    def set_timing(self, enable):
        pg_set_timing(self.handle, enable)

    def timing(self):
        return pg_get_timing(self.handle)

    def device_bytes(self):
        return pg_device_bytes(self.handle)
