"""Thin ctypes binding of libfjofc.so (include/fjofc.h).

Argument marshalling only: every step of fast JOFC runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  The
binding fails loudly when the library is missing; there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfjofc.so")

FJOFC_OK = 0
FJOFC_TOL_NONE, FJOFC_TOL_REL, FJOFC_TOL_PAPER, FJOFC_TOL_TARGET = 0, 1, 2, 3
FJOFC_MAX_M = 32
FJOFC_MAX_D = 8
FJOFC_LAUNCH_LOCKSTEP, FJOFC_LAUNCH_PERSISTENT = 0, 1

# Every symbol include/fjofc.h declares.
EXPORTS = ["fjofc_create", "fjofc_destroy", "fjofc_last_error", "fjofc_strerror",
           "fjofc_embed", "fjofc_embed_w", "fjofc_stress", "fjofc_oos",
           "fjofc_profile_enable", "fjofc_profile_read", "fjofc_batch_create",
           "fjofc_batch_run", "fjofc_batch_set_launch", "fjofc_tile_choice", "fjofc_batch_destroy",
           "fjofc_embed_batched",
           "fjofc_mlp_create", "fjofc_mlp_destroy", "fjofc_mlp_set_params",
           "fjofc_mlp_get_params", "fjofc_mlp_forward", "fjofc_mlp_backward",
           "fjofc_mlp_get_grads", "fjofc_mlp_adam", "fjofc_mlp_train_steps", "fjofc_mlp_features",
           "fjofc_mlp_predict_start", "fjofc_oos_nearest_start", "fjofc_embed_relaxed",
           "fjofc_init_cmds", "fjofc_mlp_loss", "fjofc_mlp_feature_stats",
           "fjofc_oos_consensus", "fjofc_validate_delta", "fjofc_oos_noalloc"]


class FjofcResult(C.Structure):
    _fields_ = [("iters_run", C.c_int), ("converged", C.c_int),
                ("stress", C.c_double), ("stress_norm", C.c_double),
                ("fidelity", C.c_double), ("commens", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FjofcProfile(C.Structure):
    _fields_ = [("stream_launches", C.c_int), ("stream_ms", C.c_double),
                ("stream_bytes", C.c_double), ("edge_launches", C.c_int),
                ("edge_ms", C.c_double), ("edge_bytes", C.c_double),
                ("finalize_launches", C.c_int), ("finalize_ms", C.c_double),
                ("reduce_launches", C.c_int), ("reduce_ms", C.c_double),
                ("oos_launches", C.c_int), ("oos_ms", C.c_double),
                ("oos_bytes", C.c_double), ("batch_launches", C.c_int),
                ("batch_ms", C.c_double), ("batch_bytes", C.c_double),
                ("init_launches", C.c_int), ("init_ms", C.c_double),
                ("init_bytes", C.c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FjofcProblem(C.Structure):
    _fields_ = [("m", C.c_int), ("n", C.c_int), ("d", C.c_int),
                ("delta", C.POINTER(C.c_void_p)), ("wmat", C.POINTER(C.c_double)),
                ("X", C.c_void_p)]


class FjofcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fjofc error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libfjofc.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python paper_1502_03391_amd/build.py`")
        # libfjofc and PyTorch link the same HIP runtime soname; loading
        # torch first makes the process use one runtime (torch's) for both.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        vp, ip, dp = C.c_void_p, C.c_int, C.c_double
        L.fjofc_create.argtypes = [C.POINTER(vp), ip]
        L.fjofc_destroy.argtypes = [vp]
        L.fjofc_destroy.restype = None
        L.fjofc_last_error.restype = C.c_char_p
        L.fjofc_strerror.argtypes = [ip]
        L.fjofc_strerror.restype = C.c_char_p
        L.fjofc_embed.argtypes = [vp, C.POINTER(vp), ip, ip, C.POINTER(dp), ip, vp,
                                  ip, dp, ip, ip, C.POINTER(dp),
                                  C.POINTER(FjofcResult), vp]
        L.fjofc_embed_relaxed.argtypes = [vp, C.POINTER(vp), ip, ip, C.POINTER(dp), ip, vp,
                                          ip, dp, ip, ip, dp, C.POINTER(dp),
                                          C.POINTER(FjofcResult), vp]
        L.fjofc_init_cmds.argtypes = [vp, C.POINTER(vp), ip, ip, ip, vp, ip, C.POINTER(dp), vp]
        L.fjofc_embed_w.argtypes = [vp, C.POINTER(vp), ip, ip, dp, ip, vp,
                                    ip, dp, ip, ip, C.POINTER(dp),
                                    C.POINTER(FjofcResult), vp]
        L.fjofc_stress.argtypes = [vp, C.POINTER(vp), ip, ip, C.POINTER(dp), ip, vp,
                                   C.POINTER(FjofcResult), vp]
        L.fjofc_oos.argtypes = [vp, vp, ip, ip, ip, C.POINTER(dp), vp, ip, vp,
                                ip, dp, vp, vp, vp, ip, vp]
        L.fjofc_oos_noalloc.argtypes = L.fjofc_oos.argtypes
        L.fjofc_batch_create.argtypes = [vp, C.POINTER(FjofcProblem), ip, C.POINTER(vp)]
        L.fjofc_batch_run.argtypes = [vp, ip, dp, ip, ip, C.POINTER(FjofcResult), vp]
        L.fjofc_batch_set_launch.argtypes = [vp, ip]
        L.fjofc_tile_choice.argtypes = [vp, ip, ip, C.POINTER(ip), C.POINTER(ip)]
        L.fjofc_batch_destroy.argtypes = [vp]
        L.fjofc_batch_destroy.restype = None
        L.fjofc_embed_batched.argtypes = [vp, C.POINTER(FjofcProblem), ip, ip, dp, ip, ip,
                                          C.POINTER(FjofcResult), vp]
        L.fjofc_mlp_create.argtypes = [vp, ip, C.POINTER(ip), ip, C.POINTER(vp)]
        L.fjofc_mlp_destroy.argtypes = [vp]
        L.fjofc_mlp_destroy.restype = None
        L.fjofc_mlp_set_params.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
        L.fjofc_mlp_get_params.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
        L.fjofc_mlp_forward.argtypes = [vp, vp, ip, vp, vp]
        L.fjofc_mlp_backward.argtypes = [vp, vp, vp, ip, vp, vp]
        L.fjofc_mlp_predict_start.argtypes = [vp, vp, ip, ip, ip, vp, vp]
        L.fjofc_oos_nearest_start.argtypes = [vp, vp, ip, ip, ip, vp, ip, vp, vp]
        L.fjofc_mlp_get_grads.argtypes = [vp, C.POINTER(vp), C.POINTER(vp), vp]
        L.fjofc_mlp_adam.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float, vp]
        L.fjofc_mlp_train_steps.argtypes = [vp, vp, vp, ip, ip, ip, C.POINTER(C.c_float),
                                            C.c_float, C.c_float, C.c_float, vp, vp]
        L.fjofc_mlp_features.argtypes = [vp, vp, ip, ip, ip, vp, ip, vp, vp, vp, vp]
        L.fjofc_mlp_loss.argtypes = [vp, vp, vp, ip, vp, vp]
        L.fjofc_mlp_feature_stats.argtypes = [vp, vp, ip, ip, dp, vp, vp, vp]
        L.fjofc_oos_consensus.argtypes = [vp, vp, ip, ip, ip, vp, vp]
        L.fjofc_validate_delta.argtypes = [vp, vp, ip, C.POINTER(C.c_longlong), vp]
        L.fjofc_profile_enable.argtypes = [vp, ip]
        L.fjofc_profile_read.argtypes = [vp, C.POINTER(FjofcProfile)]
        _lib = L
    return _lib


def _check(rc: int):
    if rc != FJOFC_OK:
        raise FjofcError(rc, lib().fjofc_last_error().decode())


def _stream_ptr(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _wmat_arg(wmat, m):
    w = np.ascontiguousarray(np.asarray(wmat, dtype=np.float64).reshape(m, m))
    return w, w.ctypes.data_as(C.POINTER(C.c_double))


def _dev_ptr(t, dtype, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    return t.data_ptr()


class Context:
    """Owns a fjofc_ctx (workspace, tile tables) on one device."""

    def __init__(self, device: int = 0):
        self._h = C.c_void_p()
        _check(lib().fjofc_create(C.byref(self._h), int(device)))
        self.device = device

    def close(self):
        if self._h:
            lib().fjofc_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self):
        return self._h


def fjofc_embed(ctx: Context, delta: Sequence, wmat, X, iters: int,
                tol: float = 0.0, tol_mode: int = FJOFC_TOL_REL,
                stress_every: int = 1, want_hist: bool = False, stream=None,
                alpha: float = 1.0):
    """In-sample fJOFC.  delta: m CUDA float32 n x n tensors; X: CUDA
    float32 (m n) x d tensor, X0 in, result out; alpha != 1 runs the relaxed
    transforms (fjofc_embed_relaxed).  Returns (result dict, stress history
    or None)."""
    import torch
    m = len(delta)
    n = int(delta[0].shape[0])
    ptrs = (C.c_void_p * m)(*[_dev_ptr(t, torch.float32, "delta") for t in delta])
    _w, wp = _wmat_arg(wmat, m)
    d = int(X.shape[1])
    res = FjofcResult()
    hist = np.empty(iters + 1) if want_hist else None
    hp = hist.ctypes.data_as(C.POINTER(C.c_double)) if want_hist else None
    if alpha == 1.0:
        _check(lib().fjofc_embed(ctx.handle, ptrs, m, n, wp, d,
                                 _dev_ptr(X, torch.float32, "X"), int(iters),
                                 float(tol), int(tol_mode), int(stress_every), hp,
                                 C.byref(res), _stream_ptr(stream)))
    else:
        _check(lib().fjofc_embed_relaxed(ctx.handle, ptrs, m, n, wp, d,
                                         _dev_ptr(X, torch.float32, "X"), int(iters),
                                         float(tol), int(tol_mode), int(stress_every),
                                         float(alpha), hp, C.byref(res), _stream_ptr(stream)))
    return res.as_dict(), hist


def fjofc_embed_w(ctx: Context, delta: Sequence, w: float, X, iters: int,
                  tol: float = 0.0, tol_mode: int = FJOFC_TOL_REL,
                  stress_every: int = 1, want_hist: bool = False, stream=None):
    """In-sample fJOFC with the uniform weights of eq:W (w_ii = 1, w_ik = w).
    Returns (result dict, stress history or None)."""
    import torch
    m = len(delta)
    n = int(delta[0].shape[0])
    ptrs = (C.c_void_p * m)(*[_dev_ptr(t, torch.float32, "delta") for t in delta])
    d = int(X.shape[1])
    res = FjofcResult()
    hist = np.empty(iters + 1) if want_hist else None
    hp = hist.ctypes.data_as(C.POINTER(C.c_double)) if want_hist else None
    _check(lib().fjofc_embed_w(ctx.handle, ptrs, m, n, float(w), d,
                               _dev_ptr(X, torch.float32, "X"), int(iters), float(tol),
                               int(tol_mode), int(stress_every), hp, C.byref(res),
                               _stream_ptr(stream)))
    return res.as_dict(), hist


def fjofc_init_cmds(ctx: Context, delta: Sequence, X, iters: int = 20, stream=None):
    """The paper's start X0: cMDS of the mean dissimilarity, cMDS of each
    Delta_i, Procrustes fit of each onto the first.  X: CUDA float32
    (m n) x d, written.  Returns the (m + 1) x d largest Ritz values."""
    import torch
    m = len(delta)
    n = int(delta[0].shape[0])
    d = int(X.shape[1])
    if tuple(X.shape) != (m * n, d):
        raise ValueError(f"X must be {m * n} x d")
    ptrs = (C.c_void_p * m)(*[_dev_ptr(t, torch.float32, "delta") for t in delta])
    eig = np.empty((m + 1, d))
    _check(lib().fjofc_init_cmds(ctx.handle, ptrs, m, n, d, _dev_ptr(X, torch.float32, "X"),
                                 int(iters), eig.ctypes.data_as(C.POINTER(C.c_double)),
                                 _stream_ptr(stream)))
    return eig


def fjofc_stress(ctx: Context, delta: Sequence, wmat, X, stream=None):
    """Raw stress of X (FP64 reduction on the GPU)."""
    import torch
    m = len(delta)
    n = int(delta[0].shape[0])
    ptrs = (C.c_void_p * m)(*[_dev_ptr(t, torch.float32, "delta") for t in delta])
    _w, wp = _wmat_arg(wmat, m)
    res = FjofcResult()
    _check(lib().fjofc_stress(ctx.handle, ptrs, m, n, wp, int(X.shape[1]),
                              _dev_ptr(X, torch.float32, "X"), C.byref(res),
                              _stream_ptr(stream)))
    return res.as_dict()


def fjofc_oos(ctx: Context, X_in, wmat, delta_new, Y, iters: int,
              tol: float = 0.0, target=None, stress_out=None, iters_out=None,
              sync: bool = True, stream=None):
    """Out-of-sample embedding.  X_in: (m n) x d; delta_new: k x m x n;
    Y: k x m x d (starts in, results out); target / stress_out (float64, k)
    and iters_out (int32, k) are optional CUDA tensors."""
    _oos_call(lib().fjofc_oos, ctx, X_in, wmat, delta_new, Y, iters, tol, target, stress_out,
              iters_out, sync, stream)


def fjofc_oos_noalloc(ctx: Context, X_in, wmat, delta_new, Y, iters: int,
                      tol: float = 0.0, target=None, stress_out=None, iters_out=None,
                      sync: bool = True, stream=None):
    """fjofc_oos without any device allocation (the library's per-GPU
    scratch array; m <= 8 and a bounded m d n)."""
    _oos_call(lib().fjofc_oos_noalloc, ctx, X_in, wmat, delta_new, Y, iters, tol, target,
              stress_out, iters_out, sync, stream)


def _oos_call(fn, ctx, X_in, wmat, delta_new, Y, iters, tol, target, stress_out, iters_out,
              sync, stream):
    import torch
    k, m, n = (int(s) for s in delta_new.shape)
    d = int(X_in.shape[1])
    _w, wp = _wmat_arg(wmat, m)
    tp = _dev_ptr(target, torch.float64, "target") if target is not None else None
    sp = _dev_ptr(stress_out, torch.float64, "stress_out") if stress_out is not None else None
    itp = _dev_ptr(iters_out, torch.int32, "iters_out") if iters_out is not None else None
    _check(fn(ctx.handle, _dev_ptr(X_in, torch.float32, "X_in"), m, n, d,
              wp, _dev_ptr(delta_new, torch.float32, "delta_new"), k,
              _dev_ptr(Y, torch.float32, "Y"), int(iters), float(tol),
              tp, sp, itp, 1 if sync else 0, _stream_ptr(stream)))


def fjofc_oos_nearest_start(ctx: Context, X_in, delta_new, Y, stream=None):
    """Y[o][i] = the in-sample point of modality i nearest (smallest
    dissimilarity, smallest index on ties) to new object o."""
    import torch
    k, m, n = (int(s) for s in delta_new.shape)
    d = int(X_in.shape[1])
    if tuple(Y.shape) != (k, m, d):
        raise ValueError(f"Y must be {k} x {m} x {d}")
    _check(lib().fjofc_oos_nearest_start(ctx.handle, _dev_ptr(X_in, torch.float32, "X_in"), m, n,
                                         d, _dev_ptr(delta_new, torch.float32, "delta_new"), k,
                                         _dev_ptr(Y, torch.float32, "Y"), _stream_ptr(stream)))
    return Y


def fjofc_profile_enable(ctx: Context, on: bool = True):
    """Start (and reset) or stop per-kernel event timing in the library."""
    _check(lib().fjofc_profile_enable(ctx.handle, 1 if on else 0))


def fjofc_profile_read(ctx: Context) -> dict:
    """Summed kernel durations (ms) and algorithmic bytes since enabling."""
    p = FjofcProfile()
    _check(lib().fjofc_profile_read(ctx.handle, C.byref(p)))
    return p.as_dict()


class Batch:
    """A planned batch of independent in-sample problems (fjofc_batch).

    problems: sequence of (delta list, wmat, X) with CUDA float32 tensors;
    the tensors are referenced, not copied, and must outlive the plan."""

    def __init__(self, ctx: Context, problems, launch: str = "lockstep"):
        import torch
        self.ctx = ctx
        self._keep = []
        arr = (FjofcProblem * len(problems))()
        for p, (delta, wmat, X) in enumerate(problems):
            m = len(delta)
            ptrs = (C.c_void_p * m)(*[_dev_ptr(t, torch.float32, "delta") for t in delta])
            w, wp = _wmat_arg(wmat, m)
            self._keep += [ptrs, w]
            arr[p] = FjofcProblem(m, int(delta[0].shape[0]), int(X.shape[1]),
                                  C.cast(ptrs, C.POINTER(C.c_void_p)), wp,
                                  _dev_ptr(X, torch.float32, "X"))
        self._arr = arr
        self.count = len(problems)
        self._h = C.c_void_p()
        _check(lib().fjofc_batch_create(ctx.handle, arr, self.count, C.byref(self._h)))
        if launch != "lockstep":
            self.set_launch(launch)

    def set_launch(self, launch: str):
        """"lockstep" (FJOFC_LAUNCH_LOCKSTEP) or "persistent"."""
        code = {"lockstep": FJOFC_LAUNCH_LOCKSTEP, "persistent": FJOFC_LAUNCH_PERSISTENT}
        if launch not in code:
            raise ValueError(f"unknown batch launch {launch!r}")
        _check(lib().fjofc_batch_set_launch(self._h, code[launch]))
        self.launch = launch

    def run(self, iters: int, tol: float = 0.0, tol_mode: int = FJOFC_TOL_REL,
            stress_every: int = 1, want_results: bool = True, stream=None):
        res = (FjofcResult * self.count)() if want_results else None
        _check(lib().fjofc_batch_run(self._h, int(iters), float(tol), int(tol_mode),
                                     int(stress_every), res, _stream_ptr(stream)))
        return [r.as_dict() for r in res] if want_results else None

    def close(self):
        if self._h:
            lib().fjofc_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fjofc_batch_create(ctx: Context, problems) -> Batch:
    return Batch(ctx, problems)


def fjofc_batch_run(batch: Batch, iters: int, **kw):
    return batch.run(iters, **kw)


def fjofc_tile_choice(ctx: Context, n: int, d: int):
    """(tile height, kernel variant) the library plans for an (n, d) problem."""
    th, var = C.c_int(), C.c_int()
    _check(lib().fjofc_tile_choice(ctx.handle, int(n), int(d), C.byref(th), C.byref(var)))
    return th.value, var.value


def fjofc_batch_set_launch(batch: Batch, launch: str):
    batch.set_launch(launch)


def fjofc_batch_destroy(batch: Batch):
    batch.close()


def fjofc_embed_batched(ctx: Context, problems, iters: int, tol: float = 0.0,
                        tol_mode: int = FJOFC_TOL_REL, stress_every: int = 1,
                        stream=None):
    """Plan, run and release a batch in one call; returns the results."""
    b = Batch(ctx, problems)
    try:
        return b.run(iters, tol=tol, tol_mode=tol_mode, stress_every=stress_every,
                     stream=stream)
    finally:
        b.close()


class Mlp:
    """Warm-start network (fjofc_mlp): dims = [in, hidden..., out]."""

    def __init__(self, ctx: Context, dims, max_batch: int):
        self.ctx = ctx
        self.dims = [int(x) for x in dims]
        self.L = len(self.dims) - 1
        self.max_batch = int(max_batch)
        self._h = C.c_void_p()
        arr = (C.c_int * len(self.dims))(*self.dims)
        _check(lib().fjofc_mlp_create(ctx.handle, self.L, arr, self.max_batch, C.byref(self._h)))

    def _ptrs(self, tensors, dtype, name):
        return (C.c_void_p * self.L)(*[_dev_ptr(t, dtype, name) for t in tensors])

    def set_params(self, W, b, stream=None):
        import torch
        _check(lib().fjofc_mlp_set_params(self._h, self._ptrs(W, torch.float32, "W"),
                                          self._ptrs(b, torch.float32, "b"), _stream_ptr(stream)))

    def get_params(self, stream=None):
        import torch
        W = [torch.empty((a, c), dtype=torch.float32, device="cuda")
             for a, c in zip(self.dims[:-1], self.dims[1:])]
        b = [torch.empty(c, dtype=torch.float32, device="cuda") for c in self.dims[1:]]
        _check(lib().fjofc_mlp_get_params(self._h, self._ptrs(W, torch.float32, "W"),
                                          self._ptrs(b, torch.float32, "b"), _stream_ptr(stream)))
        return W, b

    def forward(self, x, out=None, stream=None):
        import torch
        B = int(x.shape[0])
        if out is None:
            out = torch.empty((B, self.dims[-1]), dtype=torch.float32, device="cuda")
        _check(lib().fjofc_mlp_forward(self._h, _dev_ptr(x, torch.bfloat16, "x"), B,
                                       _dev_ptr(out, torch.float32, "out"), _stream_ptr(stream)))
        return out

    def predict_start(self, x, Y, stream=None):
        """Y (B x m x d): the network's point for every modality (output
        width d) or one point per modality (output width m d)."""
        import torch
        _check(lib().fjofc_mlp_predict_start(self._h, _dev_ptr(x, torch.bfloat16, "x"),
                                             int(x.shape[0]), int(Y.shape[1]), int(Y.shape[2]),
                                             _dev_ptr(Y, torch.float32, "Y"), _stream_ptr(stream)))
        return Y

    def backward(self, x, y, loss=None, stream=None):
        import torch
        lp = _dev_ptr(loss, torch.float64, "loss") if loss is not None else None
        _check(lib().fjofc_mlp_backward(self._h, _dev_ptr(x, torch.bfloat16, "x"),
                                        _dev_ptr(y, torch.float32, "y"), int(x.shape[0]), lp,
                                        _stream_ptr(stream)))

    def get_grads(self, stream=None):
        import torch
        dW = [torch.empty((a, c), dtype=torch.float32, device="cuda")
              for a, c in zip(self.dims[:-1], self.dims[1:])]
        db = [torch.empty(c, dtype=torch.float32, device="cuda") for c in self.dims[1:]]
        _check(lib().fjofc_mlp_get_grads(self._h, self._ptrs(dW, torch.float32, "dW"),
                                         self._ptrs(db, torch.float32, "db"), _stream_ptr(stream)))
        return dW, db

    def loss(self, x, y, loss, stream=None):
        """loss (device FP64, 1 element) = mean squared error of network(x)
        against y; gradients untouched."""
        import torch
        _check(lib().fjofc_mlp_loss(self._h, _dev_ptr(x, torch.bfloat16, "x"),
                                    _dev_ptr(y, torch.float32, "y"), int(x.shape[0]),
                                    _dev_ptr(loss, torch.float64, "loss"), _stream_ptr(stream)))
        return loss

    def train_steps(self, x, y, batch, lrs, loss_sum=None, beta1=0.9, beta2=0.999, eps=1e-8,
                    stream=None):
        """len(lrs) training steps on consecutive batches of `batch` rows of
        x (BF16) and y (FP32); each step's MSE is added to loss_sum (device
        FP64, optional)."""
        import torch
        if (x.dim() != 2 or y.dim() != 2 or x.shape[0] != y.shape[0]
                or x.shape[1] != self.dims[0] or y.shape[1] != self.dims[-1]):
            raise ValueError("x and y must be N x dims[0] and N x dims[-1]")
        lr = (C.c_float * len(lrs))(*[float(v) for v in lrs])
        lp = _dev_ptr(loss_sum, torch.float64, "loss_sum") if loss_sum is not None else None
        _check(lib().fjofc_mlp_train_steps(self._h, _dev_ptr(x, torch.bfloat16, "x"),
                                           _dev_ptr(y, torch.float32, "y"), int(x.shape[0]),
                                           int(batch), len(lrs), lr, float(beta1), float(beta2),
                                           float(eps), lp, _stream_ptr(stream)))

    def adam(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().fjofc_mlp_adam(self._h, float(lr), float(beta1), float(beta2), float(eps),
                                    _stream_ptr(stream)))

    def close(self):
        if self._h:
            lib().fjofc_mlp_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fjofc_mlp_features(ctx: Context, delta_new, landmarks, mu, inv_sd, x, stream=None):
    """x (k x m L, bfloat16) = standardised dissimilarities to the landmarks."""
    import torch
    k, m, n = (int(s) for s in delta_new.shape)
    L = int(landmarks.shape[0])
    lm = landmarks.detach()
    if int(lm.min()) < 0 or int(lm.max()) >= n:
        raise ValueError("landmark index out of range")
    _check(lib().fjofc_mlp_features(ctx.handle, _dev_ptr(delta_new, torch.float32, "delta_new"),
                                    k, m, n, _dev_ptr(lm, torch.int32, "landmarks"), L,
                                    _dev_ptr(mu, torch.float32, "mu"),
                                    _dev_ptr(inv_sd, torch.float32, "inv_sd"),
                                    _dev_ptr(x, torch.bfloat16, "x"), _stream_ptr(stream)))
    return x


def fjofc_mlp_feature_stats(ctx: Context, raw, mu, inv_sd, min_sd: float = 1e-6, stream=None):
    """mu, inv_sd (F FP32) = column means and 1 / max(sample SD, min_sd) of
    raw (N x F FP32)."""
    import torch
    N, F = (int(s) for s in raw.shape)
    _check(lib().fjofc_mlp_feature_stats(ctx.handle, _dev_ptr(raw, torch.float32, "raw"), N, F,
                                         float(min_sd), _dev_ptr(mu, torch.float32, "mu"),
                                         _dev_ptr(inv_sd, torch.float32, "inv_sd"),
                                         _stream_ptr(stream)))
    return mu, inv_sd


def fjofc_oos_consensus(ctx: Context, Y, out, stream=None):
    """out (k x d) = mean over the m modality points of each object in Y
    (k x m x d)."""
    import torch
    k, m, d = (int(s) for s in Y.shape)
    _check(lib().fjofc_oos_consensus(ctx.handle, _dev_ptr(Y, torch.float32, "Y"), k, m, d,
                                     _dev_ptr(out, torch.float32, "out"), _stream_ptr(stream)))
    return out


def fjofc_validate_delta(ctx: Context, delta, stream=None) -> int:
    """Check one n x n dissimilarity matrix (finite, >= 0, symmetric, zero
    diagonal).  Returns -1 when valid; raises FjofcError (code 1) naming the
    first offending entry otherwise (its row-major index is in .where)."""
    import torch
    n = int(delta.shape[0])
    if delta.dim() != 2 or int(delta.shape[1]) != n:
        raise ValueError("delta must be n x n")
    where = C.c_longlong(-1)
    rc = lib().fjofc_validate_delta(ctx.handle, _dev_ptr(delta, torch.float32, "delta"), n,
                                    C.byref(where), _stream_ptr(stream))
    if rc != FJOFC_OK:
        err = FjofcError(rc, lib().fjofc_last_error().decode())
        err.where = int(where.value)
        raise err
    return int(where.value)

