"""Sorting-based median filter (Suomela, arXiv:1406.1717) on AMD MI355X.

Tensor-level API over libmf.so (see include/mf.h); torch supplies device
memory and streams, every step of the filter runs in the library's HIP
kernels.

  median_filter(x, k)                 -> (y, argmed); x float32/int32 on a
                                         GPU (also float64/int64), shape (n,)
                                         or (rows, n)
  median_filter_batched(x, offsets, ks) -> packed (y, argmed) of a ragged batch
  median_filter_backward(grad_y, argmed, n, k) -> grad_x
  MedianFilterFn.apply(x, k)          autograd: y, with grad routed to argmed
  Plan                                explicit ragged-batch plan
"""
import numpy as np
import torch

from . import lib
from .lib import MFError, Plan

__all__ = ["median_filter", "median_filter_batched", "median_filter_backward",
           "median_filter_backward_batched", "MedianFilterFn", "Plan", "MFError",
           "output_offsets"]


def _require_gpu(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


_SIGNAL_TYPES = (torch.float32, torch.int32, torch.float64, torch.int64)


def _batch_layout(x_offsets, ks):
    """Host offsets and windows of a ragged batch, checked: 1-D, len(offsets)
    = len(ks) + 1, offsets start at 0 and never decrease, every window odd
    and within its signal.  Returns (offsets int64, ks int32)."""
    off = np.asarray(x_offsets)
    kk = np.asarray(ks)
    if off.ndim != 1 or kk.ndim != 1:
        raise ValueError("x_offsets and ks must be 1-D")
    if len(kk) < 1:
        raise ValueError("a batch needs at least one signal")
    if len(off) != len(kk) + 1:
        raise ValueError("x_offsets has %d entries for %d signals (needs %d)" % (len(off), len(kk), len(kk) + 1))
    if not (np.issubdtype(off.dtype, np.integer) and np.issubdtype(kk.dtype, np.integer)):
        raise ValueError("x_offsets and ks must hold integers")
    off = off.astype(np.int64)
    kk64 = kk.astype(np.int64)
    if off[0] != 0:
        raise ValueError("x_offsets[0] must be 0")
    lens = off[1:] - off[:-1]
    if np.any(lens < 1):
        raise ValueError("every signal needs at least one item (x_offsets must increase)")
    if np.any(kk64 < 1) or np.any(kk64 % 2 == 0) or np.any(kk64 > lens):
        s = int(np.nonzero((kk64 < 1) | (kk64 % 2 == 0) | (kk64 > lens))[0][0])
        raise ValueError("signal %d: window %d must be odd and within its length %d" % (s, int(kk64[s]), int(lens[s])))
    if np.any(kk64 > np.iinfo(np.int32).max):
        raise ValueError("windows must fit int32")
    return off, kk.astype(np.int32)


def _check_tensor(t, name, dtypes, min_numel=None, numel=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a tensor" % name)
    if t.dtype not in dtypes:
        raise TypeError("%s must be %s, got %s" % (name, " or ".join(str(d) for d in dtypes), t.dtype))
    if numel is not None and t.numel() != numel:
        raise ValueError("%s has %d entries, needs %d" % (name, t.numel(), numel))
    if min_numel is not None and t.numel() < min_numel:
        raise ValueError("%s has %d entries, needs at least %d" % (name, t.numel(), min_numel))


def median_filter(x, k, with_argmed=True):
    """Sliding-window median of odd window k over the last dimension."""
    _check_tensor(x, "x", _SIGNAL_TYPES)
    if x.dim() not in (1, 2):
        raise ValueError("x must have 1 or 2 dimensions")
    _require_gpu(x, "x")
    k = int(k)
    n = x.shape[-1]
    nout = lib.mf_output_length(n, k)
    if nout < 0:
        raise ValueError("invalid window k=%d for length %d" % (k, n))
    y = torch.empty(x.shape[:-1] + (nout,), dtype=x.dtype, device=x.device)
    am = torch.empty(y.shape, dtype=torch.int32, device=x.device) if with_argmed else None
    if x.dim() == 1:
        if x.dtype == torch.float32:
            lib.mf_median_filter(x, n, k, y, am)
        elif x.dtype == torch.int32:
            lib.mf_median_filter_i32(x, n, k, y, am)
        elif x.dtype == torch.float64:
            lib.mf_median_filter_f64(x, n, k, y, am)
        elif x.dtype == torch.int64:
            lib.mf_median_filter_i64(x, n, k, y, am)
        else:
            raise TypeError("x must be float32, int32, float64 or int64")
    elif x.dim() == 2:
        if x.dtype == torch.float32:
            lib.mf_median_filter_rows(x, x.shape[0], n, k, y, am)
        elif x.dtype == torch.int32:
            lib.mf_median_filter_rows_i32(x, x.shape[0], n, k, y, am)
        elif x.dtype == torch.float64:
            lib.mf_median_filter_rows_f64(x, x.shape[0], n, k, y, am)
        elif x.dtype == torch.int64:
            lib.mf_median_filter_rows_i64(x, x.shape[0], n, k, y, am)
        else:
            raise TypeError("x must be float32, int32, float64 or int64")
    else:
        raise ValueError("x must have 1 or 2 dimensions")
    return y, am


def output_offsets(x_offsets, ks):
    """Start of each signal's outputs in the packed ragged layout."""
    x_offsets = np.asarray(x_offsets, dtype=np.int64)
    ks = np.asarray(ks, dtype=np.int64)
    out = np.zeros(len(ks) + 1, dtype=np.int64)
    out[1:] = np.cumsum((x_offsets[1:] - x_offsets[:-1]) - ks + 1)
    return out


def median_filter_batched(x, x_offsets, ks, with_argmed=True):
    """Ragged batch: signal s = x[x_offsets[s]:x_offsets[s+1]], window ks[s]."""
    _check_tensor(x, "x", _SIGNAL_TYPES)
    if x.dim() != 1:
        raise ValueError("x must be 1-D (the signals packed back to back)")
    x_offsets, ks = _batch_layout(x_offsets, ks)
    if x.numel() < x_offsets[-1]:
        raise ValueError("x has %d items, the offsets need %d" % (x.numel(), int(x_offsets[-1])))
    _require_gpu(x, "x")
    yo = output_offsets(x_offsets, ks)
    y = torch.empty(int(yo[-1]), dtype=x.dtype, device=x.device)
    am = torch.empty(int(yo[-1]), dtype=torch.int32, device=x.device) if with_argmed else None
    fn = {torch.int32: lib.mf_median_filter_batched_i32, torch.float64: lib.mf_median_filter_batched_f64,
          torch.int64: lib.mf_median_filter_batched_i64}.get(x.dtype, lib.mf_median_filter_batched)
    fn(x, x_offsets, ks, len(ks), y, am)
    return y, am


def median_filter_backward(grad_y, argmed, n, k):
    """grad_x of y = x[argmed], of the grad_y's type (float32 or float64),
    for one signal or rows."""
    _check_tensor(grad_y, "grad_y", (torch.float32, torch.float64))
    _check_tensor(argmed, "argmed", (torch.int32,))
    n, k = int(n), int(k)
    nout = lib.mf_output_length(n, k)
    if nout < 0:
        raise ValueError("invalid window k=%d for length %d" % (k, n))
    if grad_y.dim() not in (1, 2):
        raise ValueError("grad_y must have 1 or 2 dimensions")
    if grad_y.shape[-1] != nout:
        raise ValueError("grad_y has %d outputs per row, n-k+1 = %d" % (grad_y.shape[-1], nout))
    if tuple(argmed.shape) != tuple(grad_y.shape):
        raise ValueError("argmed shape %s differs from grad_y shape %s" % (tuple(argmed.shape), tuple(grad_y.shape)))
    _require_gpu(grad_y, "grad_y")
    _require_gpu(argmed, "argmed")
    if grad_y.dtype == torch.float64:
        if grad_y.dim() == 1:
            gx = torch.empty(n, dtype=torch.float64, device=grad_y.device)
            lib.mf_median_filter_backward_f64(grad_y, argmed, n, k, gx)
        else:
            gx = torch.empty((grad_y.shape[0], n), dtype=torch.float64, device=grad_y.device)
            lib.mf_median_filter_backward_rows_f64(grad_y, argmed, grad_y.shape[0], n, k, gx)
        return gx
    if grad_y.dim() == 1:
        gx = torch.empty(n, dtype=torch.float32, device=grad_y.device)
        lib.mf_median_filter_backward(grad_y, argmed, n, k, gx)
    else:
        gx = torch.empty((grad_y.shape[0], n), dtype=torch.float32, device=grad_y.device)
        lib.mf_median_filter_backward_rows(grad_y, argmed, grad_y.shape[0], n, k, gx)
    return gx


def median_filter_backward_batched(grad_y, argmed, x_offsets, ks):
    """grad_x (float32, packed like x) of a ragged batch's y = x[argmed]."""
    x_offsets, ks = _batch_layout(x_offsets, ks)
    nout = int(output_offsets(x_offsets, ks)[-1])
    _check_tensor(grad_y, "grad_y", (torch.float32,), numel=nout)
    _check_tensor(argmed, "argmed", (torch.int32,), numel=nout)
    _require_gpu(grad_y, "grad_y")
    _require_gpu(argmed, "argmed")
    gx = torch.empty(int(x_offsets[-1]), dtype=torch.float32, device=grad_y.device)
    lib.mf_median_filter_backward_batched(grad_y, argmed, x_offsets, ks, len(ks), gx)
    return gx


class MedianFilterFn(torch.autograd.Function):
    """y = median filter of x (float32 or float64, shape (n,) or (rows, n)).

    The backward routes each upstream gradient entry to the input selected as
    that window's median (argmed), summed per input in increasing output
    index in float64 (and rounded once for float32): deterministic run to
    run."""

    @staticmethod
    def forward(ctx, x, k):
        x = x.contiguous()
        y, am = median_filter(x, k)
        ctx.save_for_backward(am)
        ctx.n = x.shape[-1]
        ctx.k = int(k)
        ctx.f64 = x.dtype == torch.float64
        ctx.mark_non_differentiable(am)
        return y, am

    @staticmethod
    def backward(ctx, grad_y, grad_am):
        (am,) = ctx.saved_tensors
        g = grad_y.contiguous()
        g = g.double() if ctx.f64 else g.float()
        gx = median_filter_backward(g, am, ctx.n, ctx.k)
        return gx, None
