"""CPU oracle for the sorting-based median filter (arXiv:1406.1717).

TEST INFRASTRUCTURE ONLY.  The test suite, the smoke check and the
benchmark's CPU-baseline leg are the only callers; the product library
never imports, links or runs anything in this package.  It shares no code
with the HIP path.

Functions (all on numpy arrays of float32, int32, float64 or int64,
single-threaded C underneath):

  sortmedian(x, k)            the paper's method: piecewise stable sort,
                              block data structure on dancing links and the
                              postprocessing driver (Sections 3-6), with the
                              invariant of eq. (inv) checked at every step.
  window_median(x, k, outs)   the problem statement of Section 1 applied to
                              the listed windows one by one (sort the
                              window's (value, index) pairs, take rank h).
  backward(grad_y, argmed, n, k)
                              scatter of the upstream gradient to the
                              selected inputs, float64 accumulation in
                              increasing output index, one rounding.
  backward_f64(grad_y, argmed, n, k)
                              the same for a float64 upstream gradient
                              (float64 result, no rounding).
  sortmedian_batched(x, offsets, ks)
                              sortmedian applied per signal of a packed
                              ragged batch.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class OracleError(RuntimeError):
    pass


_CODES = {-1: "invalid argument", -2: "out of memory",
          -3: "invariant (inv) violated"}


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        lib = ctypes.CDLL(_build.LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        I32 = ctypes.c_int32
        for name in ("oracle_sortmedian_f32", "oracle_sortmedian_i32",
                     "oracle_sortmedian_f64", "oracle_sortmedian_i64"):
            f = getattr(lib, name)
            f.argtypes = [P, I64, I32, P, P]
            f.restype = ctypes.c_int
        for name in ("oracle_window_median_f32", "oracle_window_median_i32",
                     "oracle_window_median_f64", "oracle_window_median_i64"):
            f = getattr(lib, name)
            f.argtypes = [P, I64, I32, P, I64, P]
            f.restype = ctypes.c_int
        lib.oracle_backward.argtypes = [P, P, I64, I32, P, P]
        lib.oracle_backward.restype = ctypes.c_int
        lib.oracle_backward_f64.argtypes = [P, P, I64, I32, P]
        lib.oracle_backward_f64.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _check(rc):
    if rc != 0:
        raise OracleError(_CODES.get(rc, "error %d" % rc))


def _as_signal(x):
    x = np.ascontiguousarray(x)
    if x.dtype == np.float32:
        return x, "f32"
    if x.dtype == np.int32:
        return x, "i32"
    if x.dtype == np.float64:
        return x, "f64"
    if x.dtype == np.int64:
        return x, "i64"
    raise TypeError("oracle supports float32, int32, float64 and int64 signals, got %s" % x.dtype)


def sortmedian(x, k):
    """(y, argmed) for every window of x, by the paper's method."""
    x, tag = _as_signal(x)
    n = x.shape[0]
    k = int(k)
    if k < 1 or k % 2 == 0 or n < k:
        raise OracleError("invalid argument")
    y = np.empty(n - k + 1, dtype=x.dtype)
    argmed = np.empty(n - k + 1, dtype=np.int32)
    _check(getattr(_lib(), "oracle_sortmedian_" + tag)(_ptr(x), n, k, _ptr(y), _ptr(argmed)))
    return y, argmed


def window_median(x, k, outs):
    """argmed of the windows x[o:o+k] for o in outs (the plain definition)."""
    x, tag = _as_signal(x)
    outs = np.ascontiguousarray(outs, dtype=np.int64)
    argmed = np.empty(outs.shape[0], dtype=np.int32)
    _check(getattr(_lib(), "oracle_window_median_" + tag)(
        _ptr(x), x.shape[0], int(k), _ptr(outs), outs.shape[0], _ptr(argmed)))
    return argmed


def backward(grad_y, argmed, n, k):
    """(grad_x as float32, grad_x as float64)."""
    grad_y = np.ascontiguousarray(grad_y, dtype=np.float32)
    argmed = np.ascontiguousarray(argmed, dtype=np.int32)
    g64 = np.empty(int(n), dtype=np.float64)
    g32 = np.empty(int(n), dtype=np.float32)
    _check(_lib().oracle_backward(_ptr(grad_y), _ptr(argmed), int(n), int(k),
                                  _ptr(g64), _ptr(g32)))
    return g32, g64


def backward_f64(grad_y, argmed, n, k):
    """grad_x (float64) for a float64 upstream gradient."""
    grad_y = np.ascontiguousarray(grad_y, dtype=np.float64)
    argmed = np.ascontiguousarray(argmed, dtype=np.int32)
    g = np.empty(int(n), dtype=np.float64)
    _check(_lib().oracle_backward_f64(_ptr(grad_y), _ptr(argmed), int(n), int(k), _ptr(g)))
    return g


def sortmedian_batched(x, offsets, ks):
    """Per-signal sortmedian over a packed ragged batch.

    Signal s is x[offsets[s]:offsets[s+1]] with window ks[s]; outputs are
    packed in signal order, argmed local to each signal."""
    ys, ams = [], []
    for s in range(len(ks)):
        y, a = sortmedian(x[offsets[s]:offsets[s + 1]], int(ks[s]))
        ys.append(y)
        ams.append(a)
    return np.concatenate(ys), np.concatenate(ams)
