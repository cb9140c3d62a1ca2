"""Sliding-window cumulant tensors on MI355X (gfx950): Python binding of libcum.

Thin ctypes binding over the C-ABI declared in ``include/cum.h``; every step of
the method (moment update, cumulant combine, norms) runs in the library's HIP
kernels.  The functions keep the C names:

    ctx = cum_init(n, d, b, X, prec="fp32")      # first window, t x n rows
    cum_update(ctx, X_new, X_old)                 # slide by p rows
    C4 = cum_get(ctx, 4)                          # order-4 pyramid, FP64
    fro, nu = cum_norms(ctx)                      # ||C_k||_F and nu_k
    cum_free(ctx)

Arrays may be numpy arrays (host) or torch tensors (host or device); they are
passed by pointer, so they must be C-contiguous with the path's input dtype
(float64 for "fp64", float32 for "fp32" and "bf16x3").  There is no fallback:
importing this package fails if ``libcum.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcum.so")

CUM_FP64, CUM_FP32, CUM_BF16X3 = 0, 1, 2
PRECISIONS = {"fp64": CUM_FP64, "fp32": CUM_FP32, "bf16x3": CUM_BF16X3}
CUM_OK, CUM_EINVAL, CUM_ENOMEM, CUM_EDEVICE, CUM_ESTATE, CUM_ENONFINITE, CUM_ESIZE = 0, -1, -2, -3, -4, -5, -6

EXPORTS = ("cum_init", "cum_update", "cum_get", "cum_get_moments", "cum_norms",
           "cum_norms_device", "cum_sync", "cum_free", "cum_num_blocks", "cum_num_elems",
           "cum_strerror", "cum_last_error", "cum_plan_coverage", "cum_plan_items",
           "cum_profile_enable", "cum_profile_read", "cum_batch_create", "cum_batch_update",
           "cum_batch_sync", "cum_batch_free", "cum_loss_grad",
           "cum_init_fifo", "cum_set_combine", "cum_recompute", "cum_loss_plan_create",
           "cum_loss_plan_grad", "cum_loss_plan_free", "cum_profile_sample", "cum_plan_groups",
           "cum_update_noalloc")


class CumError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        detail = _lib.cum_last_error().decode() if status == CUM_EDEVICE else ""
        super().__init__("%s: %s (status %d) %s" % (where, _lib.cum_strerror(status).decode(),
                                                    status, detail))


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError("libcum.so is not built (run __graft_entry__.build() or "
                          "python paper_1701_06446_amd/build.py): %s" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_size_t
    pd = ctypes.POINTER(ctypes.c_double)
    sig = {
        "cum_init": (i32, [ctypes.POINTER(vp), i32, i32, i32, vp, i64, i32, vp]),
        "cum_update": (i32, [vp, vp, vp, i64]),
        "cum_update_noalloc": (i32, [vp, vp, vp, i64]),
        "cum_get": (i32, [vp, i32, vp, sz]),
        "cum_get_moments": (i32, [vp, i32, vp, sz]),
        "cum_norms": (i32, [vp, pd, pd]),
        "cum_norms_device": (i32, [vp, ctypes.POINTER(vp)]),
        "cum_sync": (i32, [vp]),
        "cum_free": (i32, [vp]),
        "cum_num_blocks": (i64, [i32, i32, i32]),
        "cum_num_elems": (i64, [i32, i32, i32]),
        "cum_strerror": (ctypes.c_char_p, [i32]),
        "cum_last_error": (ctypes.c_char_p, []),
        "cum_plan_coverage": (i64, [i32, i32, i32, ctypes.POINTER(ctypes.c_int32)]),
        "cum_plan_items": (i64, [i32, i32, i32]),
        "cum_plan_groups": (i64, [i32, i32, i32, ctypes.c_void_p, ctypes.c_void_p]),
        "cum_profile_enable": (i32, [vp, i32]),
        "cum_profile_sample": (i32, [vp, i32]),
        "cum_batch_create": (i32, [ctypes.POINTER(vp), ctypes.POINTER(vp), i32]),
        "cum_batch_update": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(i64)]),
        "cum_batch_sync": (i32, [vp]),
        "cum_batch_free": (i32, [vp]),
        "cum_set_combine": (i32, [vp, i32]),
        "cum_recompute": (i32, [vp, vp]),
        "cum_loss_plan_create": (i32, [ctypes.POINTER(vp), i32, i32, i32, i64, vp]),
        "cum_loss_plan_grad": (i32, [vp, vp, vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                                     vp, vp]),
        "cum_loss_plan_free": (i32, [vp]),
        "cum_init_fifo": (i32, [ctypes.POINTER(vp), i32, i32, i32, vp, i64, i64, i32, vp]),
        "cum_loss_grad": (i32, [i32, i32, i32, vp, i64, vp, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double), vp, vp, vp]),
        "cum_profile_read": (i32, [vp, ctypes.POINTER(i64), pd]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


# torch's HIP runtime and the system one share the soname libamdhip64.so.7, but
# torch's own modules ask for the unversioned name: loading libcum.so first
# would put two runtimes in one process.  Import torch first (when present) so
# that libcum.so binds to the runtime that owns torch's device memory.
try:
    import torch as _torch  # noqa: F401
except ImportError:  # plain C-ABI use without torch
    _torch = None

_lib = _load()


def _check(rc: int, where: str):
    if rc != CUM_OK:
        raise CumError(rc, where)


def _dtype_for(prec: int):
    return np.float64 if prec == CUM_FP64 else np.float32


def _pointer(X, prec: int, ncols: int):
    """(address, rows, keep-alive) of a C-contiguous numpy array or torch tensor."""
    want = _dtype_for(prec)
    if hasattr(X, "data_ptr"):  # torch tensor
        import torch

        tdt = torch.float64 if want is np.float64 else torch.float32
        if X.dtype != tdt or not X.is_contiguous() or X.dim() != 2 or X.shape[1] != ncols:
            raise ValueError("expected a contiguous %s tensor with %d columns" % (tdt, ncols))
        return X.data_ptr(), int(X.shape[0]), X
    A = np.asarray(X)
    if A.dtype != want or not A.flags["C_CONTIGUOUS"] or A.ndim != 2 or A.shape[1] != ncols:
        raise ValueError("expected a C-contiguous %s array with %d columns" % (np.dtype(want), ncols))
    return A.ctypes.data, int(A.shape[0]), A


class Context:
    """Owns one ``cum_ctx``; released by ``cum_free`` (or garbage collection)."""

    def __init__(self, handle, n, d, b, t, prec, fifo_p=0):
        self.handle, self.n, self.d, self.b, self.t, self.prec = handle, n, d, b, t, prec
        self.fifo_p = fifo_p

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cum_free(self.handle)
            self.handle = None


def cum_init(n: int, d: int, b: int, X, prec="fp32", stream=None) -> Context:
    """Moments, cumulants and norms of the first window X (t x n)."""
    p = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    addr, t, _keep = _pointer(X, p, n)
    h = ctypes.c_void_p()
    st = None if stream is None else ctypes.c_void_p(int(stream))
    _check(_lib.cum_init(ctypes.byref(h), n, d, b, addr, t, p, st), "cum_init")
    return Context(h, n, d, b, t, p)


def cum_init_fifo(n: int, d: int, b: int, X, p: int, prec="fp32", stream=None) -> Context:
    """Like cum_init, keeping the FIFO of the t/p batch increments of the
    window (updates then contract only the new rows; X_old is not needed)."""
    pr = PRECISIONS[prec] if isinstance(prec, str) else int(prec)
    addr, t, _keep = _pointer(X, pr, n)
    h = ctypes.c_void_p()
    st = None if stream is None else ctypes.c_void_p(int(stream))
    _check(_lib.cum_init_fifo(ctypes.byref(h), n, d, b, addr, t, p, pr, st), "cum_init_fifo")
    return Context(h, n, d, b, t, pr, fifo_p=p)


def cum_recompute(ctx: Context, X):
    """Recalculate moments, cumulants and norms from scratch over the window X
    (t x n, the context's t)."""
    addr, t, _keep = _pointer(X, ctx.prec, ctx.n)
    if t != ctx.t:
        raise ValueError("cum_recompute needs the whole window: %d rows, got %d" % (ctx.t, t))
    _check(_lib.cum_recompute(ctx.handle, addr), "cum_recompute")


COMBINE = {"partitions": 0, "recursion": 1}


def cum_set_combine(ctx: Context, method="partitions"):
    """'partitions' (Alg. 4, default) or 'recursion' (c_I = m_I - sum over B
    holding I's first position of c_B m_{I\\B}); from the next update on."""
    _check(_lib.cum_set_combine(ctx.handle, COMBINE[method] if isinstance(method, str) else int(method)),
           "cum_set_combine")


def cum_update(ctx: Context, X_new, X_old=None):
    """Slide the window: X_new enters, X_old (the p oldest rows) leaves.
    On a FIFO context X_old is not read and may be None."""
    an, pn, _k1 = _pointer(X_new, ctx.prec, ctx.n)
    if X_old is None:
        ao = None
    else:
        ao, po, _k2 = _pointer(X_old, ctx.prec, ctx.n)
        if pn != po:
            raise ValueError("X_new and X_old must have the same number of rows")
    _check(_lib.cum_update(ctx.handle, an, ao, pn), "cum_update")


def cum_update_noalloc(ctx: Context, X_new, X_old=None):
    """cum_update that allocates nothing: host inputs are staged through the
    library's fixed 16 MiB device array; synchronises before returning."""
    an, pn, _k1 = _pointer(X_new, ctx.prec, ctx.n)
    if X_old is None:
        ao = None
    else:
        ao, po, _k2 = _pointer(X_old, ctx.prec, ctx.n)
        if pn != po:
            raise ValueError("X_new and X_old must have the same number of rows")
    _check(_lib.cum_update_noalloc(ctx.handle, an, ao, pn), "cum_update_noalloc")


def cum_num_blocks(n: int, b: int, k: int) -> int:
    return int(_lib.cum_num_blocks(n, b, k))


def cum_num_elems(n: int, b: int, k: int) -> int:
    return int(_lib.cum_num_elems(n, b, k))


def cum_get(ctx: Context, k: int, out=None) -> np.ndarray:
    """Order-k cumulant pyramid (FP64).  ``out`` may be a device tensor."""
    ne = cum_num_elems(ctx.n, ctx.b, k)
    if out is None:
        out = np.empty(ne, dtype=np.float64)
        _check(_lib.cum_get(ctx.handle, k, out.ctypes.data, ne), "cum_get")
        return out
    _check(_lib.cum_get(ctx.handle, k, out.data_ptr(), out.numel()), "cum_get")
    return out


def cum_get_moments(ctx: Context, k: int) -> np.ndarray:
    ne = cum_num_elems(ctx.n, ctx.b, k)
    out = np.empty(ne, dtype=np.float64)
    _check(_lib.cum_get_moments(ctx.handle, k, out.ctypes.data, ne), "cum_get_moments")
    return out


def cum_norms(ctx: Context):
    """(fro, nu), each of length d+1: fro[k] = ||C_k||_F, nu[k] = Eq. (mef)."""
    fro = np.empty(ctx.d + 1)
    nu = np.empty(ctx.d + 1)
    _check(_lib.cum_norms(ctx.handle, fro.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                          nu.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "cum_norms")
    return fro, nu


def cum_norms_device(ctx: Context) -> int:
    p = ctypes.c_void_p()
    _check(_lib.cum_norms_device(ctx.handle, ctypes.byref(p)), "cum_norms_device")
    return int(p.value)


def cum_sync(ctx: Context):
    _check(_lib.cum_sync(ctx.handle), "cum_sync")


def cum_free(ctx: Context):
    if ctx.handle:
        _check(_lib.cum_free(ctx.handle), "cum_free")
        ctx.handle = None


def cum_plan_coverage(n: int, b: int, k: int):
    """Host-only check of the pivot decomposition: (misses, hits-per-element)."""
    hits = np.zeros(max(cum_num_elems(n, b, k), 1), dtype=np.int32)
    bad = _lib.cum_plan_coverage(n, b, k, hits.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    return int(bad), hits


def cum_plan_items(n: int, d: int, b: int) -> int:
    return int(_lib.cum_plan_items(n, d, b))


def cum_plan_groups(n: int, d: int, b: int):
    """(fragments, tiles) per workgroup of the four-tile update launch (host only)."""
    ng = int(_lib.cum_plan_groups(n, d, b, None, None))
    if ng < 0:
        raise CumError(ng, "cum_plan_groups")
    frags = np.zeros(ng, np.int32)
    tiles = np.zeros(ng, np.int32)
    _lib.cum_plan_groups(n, d, b, frags.ctypes.data, tiles.ctypes.data)
    return frags, tiles


PROFILE_CLASSES = {"update": 1, "combine": 2, "norms": 4}


def cum_profile_enable(ctx: Context, on=True, every: int = 1):
    """on: True (every kernel class), False, or an iterable of class names
    ("update", "combine", "norms") to bracket with HIP events; every: bracket
    one launch in that many per class."""
    if on is True:
        mask = 7
    elif not on:
        mask = 0
    else:
        mask = 0
        for name in on:
            mask |= PROFILE_CLASSES[name]
    _check(_lib.cum_profile_enable(ctx.handle, mask), "cum_profile_enable")
    if every != 1:
        _check(_lib.cum_profile_sample(ctx.handle, int(every)), "cum_profile_sample")


def cum_profile_read(ctx: Context):
    """{"update"|"combine"|"norms": (launches, total_ms)} since the last read."""
    n = (ctypes.c_int64 * 3)()
    ms = (ctypes.c_double * 3)()
    _check(_lib.cum_profile_read(ctx.handle, n, ms), "cum_profile_read")
    return {name: (int(n[i]), float(ms[i])) for i, name in enumerate(("update", "combine", "norms"))}


class Batch:
    """Owns one ``cum_batch`` over member contexts (kept alive here)."""

    def __init__(self, handle, ctxs):
        self.handle, self.ctxs = handle, list(ctxs)

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cum_batch_free(self.handle)
            self.handle = None


def cum_batch_create(ctxs) -> Batch:
    """One captured graph that updates every context in ``ctxs``."""
    arr = (ctypes.c_void_p * len(ctxs))(*[c.handle for c in ctxs])
    h = ctypes.c_void_p()
    _check(_lib.cum_batch_create(ctypes.byref(h), arr, len(ctxs)), "cum_batch_create")
    return Batch(h, ctxs)


def cum_batch_update(batch: Batch, X_new, X_old):
    """Slide member i by len(X_new[i]) rows; device tensors only."""
    m = len(batch.ctxs)
    assert len(X_new) == m and len(X_old) == m
    pn = (ctypes.c_void_p * m)()
    po = (ctypes.c_void_p * m)()
    pp = (ctypes.c_int64 * m)()
    keep = []
    for i, c in enumerate(batch.ctxs):
        an, rn, k1 = _pointer(X_new[i], c.prec, c.n)
        if X_old[i] is None:
            ao, k2 = None, None
        else:
            ao, ro, k2 = _pointer(X_old[i], c.prec, c.n)
            if rn != ro:
                raise ValueError("X_new and X_old must have the same number of rows")
        pn[i], po[i], pp[i] = an, ao, rn
        keep += [k1, k2]
    _check(_lib.cum_batch_update(batch.handle, pn, po, pp), "cum_batch_update")


def cum_batch_sync(batch: Batch):
    _check(_lib.cum_batch_sync(batch.handle), "cum_batch_sync")


def cum_batch_free(batch: Batch):
    if batch.handle:
        _check(_lib.cum_batch_free(batch.handle), "cum_batch_free")
        batch.handle = None


class LossPlan:
    """Owns one ``cum_loss_plan`` (buffers and tables for one (n, d, b, t))."""

    def __init__(self, n, d, b, t, stream=None):
        self.n, self.d, self.b, self.t = n, d, b, t
        h = ctypes.c_void_p()
        st = None if stream is None else ctypes.c_void_p(int(stream))
        _check(_lib.cum_loss_plan_create(ctypes.byref(h), n, d, b, t, st), "cum_loss_plan_create")
        self.handle = h

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.cum_loss_plan_free(self.handle)
            self.handle = None


_loss_plans = {}


def cum_loss_grad(X, W, d=4, b=4, weights=None, stream=None):
    """L = sum_k weights[k] ||C_k(X W^T)||_F^2 and (dL/dX, dL/dW) from the HIP
    adjoint.  X: (t, n), W: (n, n), contiguous float32 device tensors.  One
    plan per (n, d, b, t, stream) is kept for the process."""
    import torch

    weights = weights or {3: 1.0, 4: 1.0}
    t, n = X.shape
    if X.dtype != torch.float32 or W.dtype != torch.float32 or W.shape != (n, n) or not X.is_cuda:
        raise ValueError("X (t, n) and W (n, n) must be float32 device tensors")
    X, W = X.contiguous(), W.contiguous()
    dX, dW = torch.empty_like(X), torch.empty_like(W)
    w = (ctypes.c_double * (d + 1))(*[float(weights.get(k, 0.0)) for k in range(d + 1)])
    L = ctypes.c_double()
    st = torch.cuda.current_stream().cuda_stream if stream is None else stream
    key = (n, d, b, t, int(st or 0))
    plan = _loss_plans.get(key)
    if plan is None:
        plan = _loss_plans[key] = LossPlan(n, d, b, t, st)
    _check(_lib.cum_loss_plan_grad(plan.handle, X.data_ptr(), W.data_ptr(), w, ctypes.byref(L), dX.data_ptr(),
                                   dW.data_ptr()), "cum_loss_plan_grad")
    return L.value, dX, dW


def _cum_loss_function():
    import torch

    class CumLoss(torch.autograd.Function):
        """L = sum_k w_k ||C_k(X W^T)||_F^2 with the gradients of the HIP adjoint
        (computed together with the loss, scaled by the incoming gradient)."""

        @staticmethod
        def forward(ctx, X, W, d=4, b=4, weights=((3, 1.0), (4, 1.0))):
            L, dX, dW = cum_loss_grad(X.detach(), W.detach(), d, b, dict(weights))
            ctx.save_for_backward(dX, dW)
            return torch.tensor(L, dtype=torch.float64, device=X.device)

        @staticmethod
        def backward(ctx, gL):
            dX, dW = ctx.saved_tensors
            g = gL.to(torch.float32)
            return g * dX, g * dW, None, None, None

    return CumLoss


if _torch is not None:
    CumLoss = _cum_loss_function()
