"""Argument checks of the tensor API, on the CPU.

The C side sees only pointers and sizes, so the Python layer checks what
it cannot: tensor dtypes, element counts against the offsets and output
lengths, and the shape of a batch layout.  Every check runs before the
tensors' device is looked at, so CPU tensors exercise each rejection here;
a well-formed call on CPU tensors reaches the device check and stops there.
"""
import numpy as np
import pytest
import torch

import paper_1406_1717_amd as mf
from paper_1406_1717_amd import lib


def test_median_filter_rejects_types_and_dims():
    with pytest.raises(TypeError):
        mf.median_filter(torch.zeros(10, dtype=torch.float16), 3)
    with pytest.raises(TypeError):
        mf.median_filter(np.zeros(10, dtype=np.float32), 3)
    with pytest.raises(ValueError, match="1 or 2 dimensions"):
        mf.median_filter(torch.zeros(2, 3, 4), 3)
    with pytest.raises(ValueError, match="GPU"):
        mf.median_filter(torch.zeros(10), 3)


@pytest.mark.parametrize("off,ks,msg", [
    ([0, 10], [3, 3], "entries for 2 signals"),
    ([0, 10, 20], [3], "entries for 1 signals"),
    ([1, 10], [3], r"x_offsets\[0\] must be 0"),
    ([0, 10, 10], [3, 1], "at least one item"),
    ([0, 10, 5], [3, 1], "at least one item"),
    ([0, 10], [4], "must be odd"),
    ([0, 10], [11], "within its length"),
    ([0, 10], [-1], "must be odd"),
    ([0, 10], [], "at least one signal"),
    ([[0, 10]], [3], "1-D"),
    ([0.0, 10.0], [3], "integers"),
])
def test_batch_layout_rejections(off, ks, msg):
    with pytest.raises(ValueError, match=msg):
        mf.median_filter_batched(torch.zeros(100), off, ks)


def test_batched_rejects_short_x_and_bad_dtype():
    with pytest.raises(ValueError, match="the offsets need 30"):
        mf.median_filter_batched(torch.zeros(29), [0, 10, 30], [3, 5])
    with pytest.raises(TypeError):
        mf.median_filter_batched(torch.zeros(30, dtype=torch.float16), [0, 10, 30], [3, 5])
    with pytest.raises(ValueError, match="1-D"):
        mf.median_filter_batched(torch.zeros(3, 10), [0, 10, 30], [3, 5])
    with pytest.raises(ValueError, match="GPU"):
        mf.median_filter_batched(torch.zeros(30), [0, 10, 30], [3, 5])


def test_backward_rejections():
    n, k = 100, 5
    g = torch.zeros(n - k + 1)
    a = torch.zeros(n - k + 1, dtype=torch.int32)
    with pytest.raises(TypeError, match="argmed"):
        mf.median_filter_backward(g, a.long(), n, k)
    with pytest.raises(TypeError, match="grad_y"):
        mf.median_filter_backward(g.half(), a, n, k)
    with pytest.raises(ValueError, match="outputs per row"):
        mf.median_filter_backward(torch.zeros(n - k), a[:-1], n, k)
    with pytest.raises(ValueError, match="shape"):
        mf.median_filter_backward(g, a[:-1], n, k)
    with pytest.raises(ValueError, match="shape"):
        mf.median_filter_backward(g.reshape(1, -1), a, n, k)
    with pytest.raises(ValueError, match="invalid window"):
        mf.median_filter_backward(g, a, n, 4)
    with pytest.raises(ValueError, match="GPU"):
        mf.median_filter_backward(g, a, n, k)


def test_backward_batched_rejections():
    off, ks = [0, 10, 30], [3, 5]
    nout = (10 - 3 + 1) + (20 - 5 + 1)
    g = torch.zeros(nout)
    a = torch.zeros(nout, dtype=torch.int32)
    with pytest.raises(ValueError, match="needs %d" % nout):
        mf.median_filter_backward_batched(g[:-1], a, off, ks)
    with pytest.raises(ValueError, match="needs %d" % nout):
        mf.median_filter_backward_batched(g, a[:-1], off, ks)
    with pytest.raises(TypeError):
        mf.median_filter_backward_batched(g.double(), a, off, ks)
    with pytest.raises(ValueError, match="must be odd"):
        mf.median_filter_backward_batched(g, a, off, [3, 4])
    with pytest.raises(ValueError, match="GPU"):
        mf.median_filter_backward_batched(g, a, off, ks)


class _FakePlan(lib.Plan):
    """The plan's Python checks without a device plan behind them."""

    def __init__(self, off, ks, nout):
        self._off = np.asarray(off, dtype=np.int64)
        self._ks = np.asarray(ks, dtype=np.int32)
        self._nout = nout
        self._h = None

    @property
    def output_length(self):
        return self._nout


def test_plan_tensor_checks():
    P = _FakePlan([0, 10, 30], [3, 5], 24)
    x, y, a = torch.zeros(30), torch.zeros(24), torch.zeros(24, dtype=torch.int32)
    with pytest.raises(ValueError, match="x has 29 entries"):
        P.execute(torch.zeros(29), y, a)
    with pytest.raises(ValueError, match="y has 23 entries"):
        P.execute(x, torch.zeros(23), a)
    with pytest.raises(TypeError, match="y must be"):
        P.execute(x, torch.zeros(24, dtype=torch.int32), a)
    with pytest.raises(TypeError, match="argmed"):
        P.execute(x, y, a.long())
    with pytest.raises(ValueError, match="argmed has 23"):
        P.execute(x, y, a[:-1])
    with pytest.raises(TypeError, match="x must be"):
        P.execute(x.half(), y.half(), a)
    with pytest.raises(TypeError, match="y must be"):
        P.execute(x.double(), y, a)
    with pytest.raises(ValueError, match="GPU"):
        P.execute(x, y, a)
    with pytest.raises(ValueError, match="GPU"):
        P.execute(x, y, None)
    with pytest.raises(ValueError, match="grad_x has 29"):
        P.execute_backward(y, a, torch.zeros(29))
    with pytest.raises(ValueError, match="grad_y has 23"):
        P.execute_backward(torch.zeros(23), a, x)
    with pytest.raises(TypeError, match="float32 signals"):
        P.autotune(x.int(), y.int(), a)
