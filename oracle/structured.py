"""ctypes front-end of the plain FP64 C oracle (test infrastructure only).

Every function takes numpy arrays; dissimilarities are passed as FP32 (the
values the GPU reads) and promoted to FP64 inside the oracle.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libfjofc_oracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_fp = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build
            build.build()
        L = C.CDLL(_LIB_PATH)
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.restype = C.c_int
        L.orc_wmod.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.orc_inverse.argtypes = [C.c_int, _dp, _dp]
        L.orc_block_bx.argtypes = [C.c_int, C.c_int, C.c_double, _fp, _dp, _dp,
                                   C.c_int, C.c_int]
        L.orc_guttman.argtypes = [C.c_int, C.c_int, C.c_int, _fp, _dp, _dp, _dp]
        L.orc_fidelity_block.argtypes = [C.c_int, C.c_int, _fp, _dp]
        L.orc_fidelity_block.restype = C.c_double
        L.orc_commens_pair.argtypes = [C.c_int, C.c_int, _dp, _dp]
        L.orc_commens_pair.restype = C.c_double
        L.orc_stress.argtypes = [C.c_int, C.c_int, C.c_int, _fp, _dp, _dp, _dp]
        L.orc_embed.argtypes = [C.c_int, C.c_int, C.c_int, _fp, _dp, _dp,
                                C.c_int, C.c_double, C.c_int, C.c_int,
                                C.c_double, C.c_void_p, _dp]
        L.orc_oos_stress.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _fp, _dp]
        L.orc_oos_stress.restype = C.c_double
        L.orc_oos_step.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _dp, _fp,
                                   _dp, _dp]
        L.orc_oos.argtypes = [C.c_int, C.c_int, C.c_int, _dp, _dp, _fp, C.c_int,
                              _dp, C.c_int, C.c_double, C.c_void_p, C.c_void_p,
                              C.c_void_p]
        _lib = L
    return _lib


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _stack_delta(delta) -> np.ndarray:
    if isinstance(delta, np.ndarray) and delta.ndim == 3:
        return _f32(delta)
    return _f32(np.stack([np.asarray(x) for x in delta]))


def wmod(wmat: np.ndarray, n: int) -> np.ndarray:
    """The m x m matrix of eq:modW."""
    wmat = _f64(wmat)
    m = wmat.shape[0]
    out = np.empty((m, m))
    lib().orc_wmod(m, n, wmat, out)
    return out


def inverse(A: np.ndarray) -> np.ndarray:
    A = _f64(A)
    out = np.empty_like(A)
    if lib().orc_inverse(A.shape[0], A, out):
        raise np.linalg.LinAlgError("singular")
    return out


def block_bx(delta_i, X_i, wii=1.0, rows=None) -> np.ndarray:
    """B_i X^(i) from eq:B for one modality block (optionally a row range)."""
    dl = _f32(delta_i)
    X = _f64(X_i)
    n, d = X.shape
    r0, r1 = rows if rows is not None else (0, n)
    out = np.empty((r1 - r0, d))
    lib().orc_block_bx(n, d, float(wii), dl, X, out, r0, r1)
    return out


def guttman(delta, wmat, X) -> np.ndarray:
    """One structured Guttman transform (eq:update)."""
    dl = _stack_delta(delta)
    m, n, _ = dl.shape
    X = _f64(X)
    d = X.shape[1]
    out = np.empty_like(X)
    if lib().orc_guttman(m, n, d, dl, _f64(wmat), X, out):
        raise np.linalg.LinAlgError("eq:modW matrix singular")
    return out


def stress(delta, wmat, X):
    """(sigma, weighted fidelity, weighted commensurability)."""
    dl = _stack_delta(delta)
    m, n, _ = dl.shape
    X = _f64(X)
    out = np.empty(3)
    lib().orc_stress(m, n, X.shape[1], dl, _f64(wmat), X, out)
    return float(out[0]), float(out[1]), float(out[2])


def embed(delta, wmat, X0, iters, tol=0.0, tol_mode=1, stress_every=1,
          want_hist=True, alpha=1.0):
    """Algorithm 2's loop from X0 (alpha != 1: the relaxed update
    X + alpha (Gamma(X) - X) of the Conclusion; tol_mode 3: stop once the
    stress is <= tol).  Returns (X, stats dict, hist)."""
    dl = _stack_delta(delta)
    m, n, _ = dl.shape
    X = _f64(X0).copy()
    d = X.shape[1]
    hist = np.empty(iters + 1) if want_hist else None
    stats = np.empty(6)
    rc = lib().orc_embed(m, n, d, dl, _f64(wmat), X, int(iters), float(tol),
                         int(tol_mode), int(stress_every), float(alpha),
                         hist.ctypes.data if want_hist else None, stats)
    if rc:
        raise RuntimeError(f"oracle embed failed ({rc})")
    res = dict(iters_run=int(stats[0]), converged=int(stats[1]),
               stress=stats[2], stress_norm=stats[3], fidelity=stats[4],
               commens=stats[5])
    return X, res, hist


def oos_stress(X, wmat, dnew, y) -> float:
    """eq:joos for one new object: dnew (m x n), y (m x d)."""
    X = _f64(X)
    wmat = _f64(wmat)
    dn = _f32(dnew)
    m, n = dn.shape
    return lib().orc_oos_stress(m, n, X.shape[1], X, wmat, dn, _f64(y))


def oos_step(X, wmat, dnew, y) -> np.ndarray:
    X = _f64(X)
    wmat = _f64(wmat)
    dn = _f32(dnew)
    m, n = dn.shape
    Li = inverse(wmod(wmat, n))
    out = np.empty((m, X.shape[1]))
    lib().orc_oos_step(m, n, X.shape[1], X, wmat, Li, dn, _f64(y), out)
    return out


def oos(X, wmat, dnew, Y0, iters, tol=0.0, target: Optional[np.ndarray] = None):
    """Out-of-sample embedding of k objects.  dnew: k x m x n, Y0: k x m x d.
    Returns (Y, stress per object, iterations per object)."""
    X = _f64(X)
    wmat = _f64(wmat)
    dn = _f32(dnew)
    k, m, n = dn.shape
    Y = _f64(Y0).copy()
    st = np.empty(k)
    it = np.empty(k, dtype=np.int32)
    tg = _f64(target) if target is not None else None
    rc = lib().orc_oos(m, n, X.shape[1], X, wmat, dn, k, Y, int(iters),
                       float(tol), tg.ctypes.data if tg is not None else None,
                       st.ctypes.data, it.ctypes.data)
    if rc:
        raise RuntimeError(f"oracle oos failed ({rc})")
    return Y, st, it


def threads() -> int:
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().orc_get_threads())


def set_threads(t: int) -> None:
    """Set the OpenMP threads of the oracle's parallel loops (timing)."""
    lib().orc_set_threads(int(t))
