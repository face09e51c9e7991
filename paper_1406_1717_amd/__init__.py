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


def median_filter(x, k, with_argmed=True):
    """Sliding-window median of odd window k over the last dimension."""
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
    _require_gpu(x, "x")
    if x.dtype not in (torch.float32, torch.int32):
        raise TypeError("batched signals must be float32 or int32")
    yo = output_offsets(x_offsets, ks)
    y = torch.empty(int(yo[-1]), dtype=x.dtype, device=x.device)
    am = torch.empty(int(yo[-1]), dtype=torch.int32, device=x.device) if with_argmed else None
    if x.dtype == torch.int32:
        lib.mf_median_filter_batched_i32(x, x_offsets, ks, len(ks), y, am)
    else:
        lib.mf_median_filter_batched(x, x_offsets, ks, len(ks), y, am)
    return y, am


def median_filter_backward(grad_y, argmed, n, k):
    """grad_x of y = x[argmed], of the grad_y's type (float32 or float64),
    for one signal or rows."""
    _require_gpu(grad_y, "grad_y")
    _require_gpu(argmed, "argmed")
    if grad_y.dtype == torch.float64:
        if grad_y.dim() == 1:
            gx = torch.empty(int(n), dtype=torch.float64, device=grad_y.device)
            lib.mf_median_filter_backward_f64(grad_y, argmed, n, k, gx)
        else:
            gx = torch.empty((grad_y.shape[0], int(n)), dtype=torch.float64, device=grad_y.device)
            lib.mf_median_filter_backward_rows_f64(grad_y, argmed, grad_y.shape[0], n, k, gx)
        return gx
    if grad_y.dim() == 1:
        gx = torch.empty(int(n), dtype=torch.float32, device=grad_y.device)
        lib.mf_median_filter_backward(grad_y, argmed, n, k, gx)
    else:
        gx = torch.empty((grad_y.shape[0], int(n)), dtype=torch.float32, device=grad_y.device)
        lib.mf_median_filter_backward_rows(grad_y, argmed, grad_y.shape[0], n, k, gx)
    return gx


def median_filter_backward_batched(grad_y, argmed, x_offsets, ks):
    _require_gpu(grad_y, "grad_y")
    gx = torch.empty(int(np.asarray(x_offsets)[-1]), dtype=torch.float32, device=grad_y.device)
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
