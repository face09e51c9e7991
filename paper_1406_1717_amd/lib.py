"""ctypes binding of libmf.so (include/mf.h), one Python function per C entry
point with the same name.  Argument marshalling only: tensors are passed as
device pointers, torch's current HIP stream as the stream argument, and a
failing status raises MFError with the library's message.

The binding refuses to run without the built library: there is no fallback.
"""
import ctypes
import os

import torch

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmf.so")

MF_OK = 0
_lib = None


class MFError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s (status %d): %s" % (status_string(status), status, message))
        self.status = status


def load():
    """Load libmf.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libmf.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    sig = {
        "mf_median_filter": [P, I64, I32, P, P, P],
        "mf_median_filter_i32": [P, I64, I32, P, P, P],
        "mf_median_filter_noalloc": [P, I64, I32, P, P, P],
        "mf_median_filter_f64": [P, I64, I32, P, P, P],
        "mf_median_filter_i64": [P, I64, I32, P, P, P],
        "mf_median_filter_rows": [P, I64, I64, I32, P, P, P],
        "mf_median_filter_rows_i32": [P, I64, I64, I32, P, P, P],
        "mf_median_filter_rows_f64": [P, I64, I64, I32, P, P, P],
        "mf_median_filter_rows_i64": [P, I64, I64, I32, P, P, P],
        "mf_median_filter_batched": [P, P, P, I32, P, P, P],
        "mf_median_filter_batched_i32": [P, P, P, I32, P, P, P],
        "mf_median_filter_batched_f64": [P, P, P, I32, P, P, P],
        "mf_median_filter_batched_i64": [P, P, P, I32, P, P, P],
        "mf_plan_execute_f64": [P, P, P, P, P],
        "mf_plan_execute_i64": [P, P, P, P, P],
        "mf_median_filter_backward": [P, P, I64, I32, P, P],
        "mf_median_filter_backward_rows": [P, P, I64, I64, I32, P, P],
        "mf_median_filter_backward_f64": [P, P, I64, I32, P, P],
        "mf_median_filter_backward_rows_f64": [P, P, I64, I64, I32, P, P],
        "mf_median_filter_backward_batched": [P, P, P, P, I32, P, P],
        "mf_plan_create_batched": [P, P, I32, P],
        "mf_plan_execute": [P, P, P, P, P],
        "mf_plan_execute_i32": [P, P, P, P, P],
        "mf_plan_execute_backward": [P, P, P, P, P],
        "mf_plan_autotune": [P, P, P, P, I32, P],
        "mf_plan_set_config": [P, I32],
        "mf_plan_get_config": [P, P, P],
        "mf_plan_get_tile_threads": [P, I32, P],
        "mf_check_device_error": [P],
    }
    for name, args in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.mf_plan_output_length.argtypes = [P]
    L.mf_plan_output_length.restype = I64
    L.mf_plan_destroy.argtypes = [P]
    L.mf_plan_destroy.restype = None
    L.mf_output_length.argtypes = [I64, I32]
    L.mf_output_length.restype = I64
    L.mf_status_string.argtypes = [ctypes.c_int]
    L.mf_status_string.restype = ctypes.c_char_p
    L.mf_last_error.argtypes = []
    L.mf_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def status_string(status):
    return load().mf_status_string(int(status)).decode()


def last_error():
    return load().mf_last_error().decode()


def _check(status):
    if status != MF_OK:
        raise MFError(status, last_error())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _host_i64(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(ctypes.c_void_p)


def _host_i32(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.c_void_p)


# --- entry points (same names as the C ABI) ---------------------------------

def mf_median_filter(x, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter(_ptr(x), int(n), int(k), _ptr(y), _ptr(argmed), _stream(stream)))


def mf_median_filter_noalloc(x, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_noalloc(_ptr(x), int(n), int(k), _ptr(y), _ptr(argmed), _stream(stream)))


def mf_median_filter_i32(x, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_i32(_ptr(x), int(n), int(k), _ptr(y), _ptr(argmed), _stream(stream)))


def mf_median_filter_f64(x, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_f64(_ptr(x), int(n), int(k), _ptr(y), _ptr(argmed), _stream(stream)))


def mf_median_filter_i64(x, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_i64(_ptr(x), int(n), int(k), _ptr(y), _ptr(argmed), _stream(stream)))


def mf_median_filter_rows(x, rows, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_rows(_ptr(x), int(rows), int(n), int(k), _ptr(y), _ptr(argmed),
                                        _stream(stream)))


def mf_median_filter_rows_i32(x, rows, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_rows_i32(_ptr(x), int(rows), int(n), int(k), _ptr(y), _ptr(argmed),
                                            _stream(stream)))


def mf_median_filter_rows_f64(x, rows, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_rows_f64(_ptr(x), int(rows), int(n), int(k), _ptr(y), _ptr(argmed),
                                            _stream(stream)))


def mf_median_filter_rows_i64(x, rows, n, k, y, argmed, stream=None):
    _check(load().mf_median_filter_rows_i64(_ptr(x), int(rows), int(n), int(k), _ptr(y), _ptr(argmed),
                                            _stream(stream)))


def mf_median_filter_batched(x, x_offsets, ks, num_signals, y, argmed, stream=None):
    off, offp = _host_i64(x_offsets)
    kk, kp = _host_i32(ks)
    _check(load().mf_median_filter_batched(_ptr(x), offp, kp, int(num_signals), _ptr(y), _ptr(argmed),
                                           _stream(stream)))


def mf_median_filter_batched_i32(x, x_offsets, ks, num_signals, y, argmed, stream=None):
    off, offp = _host_i64(x_offsets)
    kk, kp = _host_i32(ks)
    _check(load().mf_median_filter_batched_i32(_ptr(x), offp, kp, int(num_signals), _ptr(y), _ptr(argmed),
                                               _stream(stream)))


def mf_median_filter_batched_f64(x, x_offsets, ks, num_signals, y, argmed, stream=None):
    off, offp = _host_i64(x_offsets)
    kk, kp = _host_i32(ks)
    _check(load().mf_median_filter_batched_f64(_ptr(x), offp, kp, int(num_signals), _ptr(y), _ptr(argmed),
                                               _stream(stream)))


def mf_median_filter_batched_i64(x, x_offsets, ks, num_signals, y, argmed, stream=None):
    off, offp = _host_i64(x_offsets)
    kk, kp = _host_i32(ks)
    _check(load().mf_median_filter_batched_i64(_ptr(x), offp, kp, int(num_signals), _ptr(y), _ptr(argmed),
                                               _stream(stream)))


def mf_median_filter_backward(grad_y, argmed, n, k, grad_x, stream=None):
    _check(load().mf_median_filter_backward(_ptr(grad_y), _ptr(argmed), int(n), int(k), _ptr(grad_x),
                                            _stream(stream)))


def mf_median_filter_backward_f64(grad_y, argmed, n, k, grad_x, stream=None):
    _check(load().mf_median_filter_backward_f64(_ptr(grad_y), _ptr(argmed), int(n), int(k), _ptr(grad_x),
                                                _stream(stream)))


def mf_median_filter_backward_rows_f64(grad_y, argmed, rows, n, k, grad_x, stream=None):
    _check(load().mf_median_filter_backward_rows_f64(_ptr(grad_y), _ptr(argmed), int(rows), int(n), int(k),
                                                     _ptr(grad_x), _stream(stream)))


def mf_median_filter_backward_rows(grad_y, argmed, rows, n, k, grad_x, stream=None):
    _check(load().mf_median_filter_backward_rows(_ptr(grad_y), _ptr(argmed), int(rows), int(n), int(k),
                                                 _ptr(grad_x), _stream(stream)))


def mf_median_filter_backward_batched(grad_y, argmed, x_offsets, ks, num_signals, grad_x, stream=None):
    off, offp = _host_i64(x_offsets)
    kk, kp = _host_i32(ks)
    _check(load().mf_median_filter_backward_batched(_ptr(grad_y), _ptr(argmed), offp, kp, int(num_signals),
                                                    _ptr(grad_x), _stream(stream)))


def mf_output_length(n, k):
    return int(load().mf_output_length(int(n), int(k)))


def mf_check_device_error(stream=None):
    _check(load().mf_check_device_error(_stream(stream)))


def _is_i32(t):
    return str(getattr(t, "dtype", "")) in ("torch.int32", "int32")


def _plan_tensors(*specs):
    """Plan arguments (tensor, name, dtypes, min_numel, may_be_none): each a
    tensor of one of dtypes with at least min_numel entries (the C side
    cannot see tensor sizes), then each a contiguous GPU tensor."""
    for t, name, dtypes, min_numel, may_be_none in specs:
        if t is None and may_be_none:
            continue
        if not isinstance(t, torch.Tensor):
            raise TypeError("%s must be a tensor" % name)
        if t.dtype not in dtypes:
            raise TypeError("%s must be %s, got %s" % (name, " or ".join(str(d) for d in dtypes), t.dtype))
        if t.numel() < min_numel:
            raise ValueError("%s has %d entries, the plan needs %d" % (name, t.numel(), min_numel))
    for t, name, _, _, _ in specs:
        if t is not None and (not t.is_cuda or not t.is_contiguous()):
            raise ValueError("%s must be a contiguous GPU tensor" % name)


class Plan:
    """mf_plan_* for one ragged batch layout (host offsets and windows)."""

    def __init__(self, x_offsets, ks):
        self._off, offp = _host_i64(x_offsets)
        self._ks, kp = _host_i32(ks)
        if self._off.ndim != 1 or self._ks.ndim != 1 or len(self._off) != len(self._ks) + 1:
            raise ValueError("x_offsets needs len(ks) + 1 entries")
        h = ctypes.c_void_p()
        _check(load().mf_plan_create_batched(offp, kp, len(self._ks), ctypes.byref(h)))
        self._h = h

    @property
    def output_length(self):
        return int(load().mf_plan_output_length(self._h))

    def _check_forward(self, x, y, argmed):
        xd = getattr(x, "dtype", None)
        _plan_tensors((x, "x", (torch.float32, torch.int32, torch.float64, torch.int64), int(self._off[-1]), False),
                      (y, "y", (xd,), self.output_length, False),
                      (argmed, "argmed", (torch.int32,), self.output_length, True))

    def execute(self, x, y, argmed, stream=None):
        self._check_forward(x, y, argmed)
        L = load()
        fn = {torch.int32: L.mf_plan_execute_i32, torch.float64: L.mf_plan_execute_f64,
              torch.int64: L.mf_plan_execute_i64}.get(x.dtype, L.mf_plan_execute)
        _check(fn(self._h, _ptr(x), _ptr(y), _ptr(argmed), _stream(stream)))

    def execute_backward(self, grad_y, argmed, grad_x, stream=None):
        _plan_tensors((grad_y, "grad_y", (torch.float32,), self.output_length, False),
                      (argmed, "argmed", (torch.int32,), self.output_length, False),
                      (grad_x, "grad_x", (torch.float32,), int(self._off[-1]), False))
        _check(load().mf_plan_execute_backward(self._h, _ptr(grad_y), _ptr(argmed), _ptr(grad_x),
                                               _stream(stream)))

    def autotune(self, x, y, argmed, reps=2, stream=None):
        """Times each launch configuration on these buffers and keeps the
        fastest.  Returns {"config": c, "tuned_ms": [ms per configuration]}."""
        if getattr(x, "dtype", None) != torch.float32:
            raise TypeError("autotune runs on float32 signals")
        self._check_forward(x, y, argmed)
        _check(load().mf_plan_autotune(self._h, _ptr(x), _ptr(y), _ptr(argmed), int(reps), _stream(stream)))
        return self.config_info()

    def set_config(self, config):
        _check(load().mf_plan_set_config(self._h, int(config)))

    def tile_threads(self, k):
        """Threads per tile used for window k (512 or 1024; 0 when k is not
        served by LDS tiles)."""
        t = ctypes.c_int32()
        _check(load().mf_plan_get_tile_threads(self._h, int(k), ctypes.byref(t)))
        return int(t.value)

    def config_info(self):
        c = ctypes.c_int32()
        ms = (ctypes.c_float * 3)()
        _check(load().mf_plan_get_config(self._h, ctypes.byref(c), ms))
        return {"config": int(c.value), "tuned_ms": [float(v) for v in ms]}

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            load().mf_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
