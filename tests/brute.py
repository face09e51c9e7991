"""Brute-force median filters used to pin the oracle (tiny inputs only).

Two formulations, both independent of the oracle's code:
  rank_count_argmed  counts, for every window item, how many window items
                     are below it in (value, index) order and picks the one
                     with exactly h below (Section 1 with the tie rule of
                     Sections 5.2 / 6.3);
  argsort_argmed     numpy's stable argsort of each window, rank h.
Float order convention: -0.0 equals +0.0; NaN is above +inf.
"""
import numpy as np
from numpy.lib.stride_tricks import sliding_window_view


def value_rank(x):
    """Dense rank of each value under the float/int convention."""
    x = np.asarray(x)
    if x.dtype.kind == "f":
        with np.errstate(invalid="ignore"):      # NaN payloads
            v = x.astype(np.float64)
        nan = np.isnan(v)
        v = np.where(nan, 0.0, v)
        v = np.where(v == 0.0, 0.0, v)          # fold -0.0 onto +0.0
        order = np.lexsort((v, nan))             # primary: nan flag
        keys = np.stack([nan[order], v[order]], axis=1)
    else:
        v = x.astype(np.int64)
        order = np.argsort(v, kind="stable")
        keys = v[order][:, None]
    new = np.ones(len(order), dtype=bool)
    if len(order) > 1:
        new[1:] = np.any(keys[1:] != keys[:-1], axis=1)
    ranks_sorted = np.cumsum(new) - 1
    r = np.empty(len(order), dtype=np.int64)
    r[order] = ranks_sorted
    return r


def rank_count_argmed(x, k):
    """argmed[o] for every window, by counting ranks (O(n k^2))."""
    n = len(x)
    h = (k - 1) // 2
    vr = value_rank(x)
    W = sliding_window_view(vr, k)                      # (nw, k)
    pos = np.arange(k)
    below = (W[:, :, None] < W[:, None, :]) | (
        (W[:, :, None] == W[:, None, :]) & (pos[:, None] < pos[None, :]))
    rank = below.sum(axis=1)                            # rank of item t
    sel = np.argmax(rank == h, axis=1)
    assert np.all(rank[np.arange(W.shape[0]), sel] == h)
    return (np.arange(n - k + 1) + sel).astype(np.int32)


def argsort_argmed(x, k):
    """argmed[o] via numpy's stable argsort of each window."""
    h = (k - 1) // 2
    x = np.asarray(x)
    if x.dtype.kind == "f":
        x = np.where(x == 0, np.zeros_like(x), x)       # -0.0 -> +0.0
    W = sliding_window_view(x, k)
    return (np.arange(W.shape[0]) + np.argsort(W, axis=1, kind="stable")[:, h]).astype(np.int32)
