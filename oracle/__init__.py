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
  sortmedian_parallel(x, k, threads)
                              sortmedian over contiguous output ranges, one
                              thread per range (each range reads its windows'
                              k-1 item halo); outputs identical to sortmedian.

The C functions keep no state between calls, and ctypes releases the GIL
while one runs, so calls from several Python threads run in parallel.
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


def sortmedian_parallel(x, k, threads=None, ranges=None):
    """(y, argmed) of every window of x by the paper's method, the outputs
    cut into `ranges` contiguous ranges run on `threads` threads.  Range
    [o0, o1) runs sortmedian on x[o0 : o1 + k - 1] (its own piecewise sort,
    so blocks on a range border are sorted twice) and shifts its argmed by
    o0."""
    from concurrent.futures import ThreadPoolExecutor
    x, _ = _as_signal(x)
    n = x.shape[0]
    k = int(k)
    if k < 1 or k % 2 == 0 or n < k:
        raise OracleError("invalid argument")
    nout = n - k + 1
    threads = int(threads or os.cpu_count() or 1)
    ranges = int(ranges or threads)
    ranges = max(1, min(ranges, nout))
    cuts = [nout * r // ranges for r in range(ranges + 1)]
    y = np.empty(nout, dtype=x.dtype)
    argmed = np.empty(nout, dtype=np.int32)

    def run(r):
        o0, o1 = cuts[r], cuts[r + 1]
        if o1 <= o0:
            return
        yr, ar = sortmedian(x[o0:o1 + k - 1], k)
        y[o0:o1] = yr
        argmed[o0:o1] = ar + o0

    with ThreadPoolExecutor(max_workers=threads) as ex:
        list(ex.map(run, range(ranges)))
    return y, argmed
