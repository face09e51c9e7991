"""GPU backward parity: grad_x from the HIP path vs the CPU oracle.

The backward sums, for every input j, the upstream gradients of the outputs
whose argmedian is j, in float64 and in increasing output order, rounded
once to float32.  The oracle does exactly that, so the results must be
bitwise equal; they must also be bitwise equal run to run, and agree with
central finite differences of the GPU forward.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1406_1717_amd as mf
from paper_1406_1717_amd import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def gpu_forward_backward(x, k, g):
    xt = torch.from_numpy(x).to(DEV)
    y, am = mf.median_filter(xt, k)
    gx = mf.median_filter_backward(torch.from_numpy(g).to(DEV), am, x.shape[-1], k)
    torch.cuda.synchronize()
    return y.cpu().numpy(), am.cpu().numpy(), gx.cpu().numpy()


@pytest.mark.parametrize("k", [1, 3, 31, 201, 1001, 1025, 1027, 4095, 5001])
def test_backward_bitwise_vs_oracle(k):
    rng = np.random.default_rng(600 + k)
    n = max(3 * k, 30_000) + 7
    x = rng.standard_normal(n).astype(np.float32)
    g = rng.standard_normal(n - k + 1).astype(np.float32)
    _, am, gx = gpu_forward_backward(x, k, g)
    _, ao = oracle.sortmedian(x, k)
    assert np.array_equal(am, ao)
    g32, g64 = oracle.backward(g, ao, n, k)
    assert np.array_equal(gx.view(np.uint32), g32.view(np.uint32))


@pytest.mark.parametrize("k", [3, 101, 1001, 1025, 1027])
def test_backward_with_ties_heavy_reuse(k):
    """Few distinct values: one input can be the median of many windows."""
    rng = np.random.default_rng(700 + k)
    n = 40_000
    x = rng.integers(0, 3, n).astype(np.float32)
    g = (rng.standard_normal(n - k + 1) * np.exp(rng.uniform(-20, 20, n - k + 1))).astype(np.float32)
    _, am, gx = gpu_forward_backward(x, k, g)
    _, ao = oracle.sortmedian(x, k)
    assert np.array_equal(am, ao)
    g32, g64 = oracle.backward(g, ao, n, k)
    assert np.array_equal(gx.view(np.uint32), g32.view(np.uint32))
    nz = g64 != 0
    assert np.all(np.abs(gx[nz].astype(np.float64) - g64[nz]) <= 1e-6 * np.abs(g64[nz]))
    assert np.all(gx[~nz] == 0)


def test_backward_deterministic():
    rng = np.random.default_rng(801)
    n, k = 200_000, 201
    x = rng.integers(0, 50, n).astype(np.float32)
    g = rng.standard_normal(n - k + 1).astype(np.float32)
    xt = torch.from_numpy(x).to(DEV)
    _, am = mf.median_filter(xt, k)
    gt = torch.from_numpy(g).to(DEV)
    a = mf.median_filter_backward(gt, am, n, k)
    b = mf.median_filter_backward(gt, am, n, k)
    assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_autograd_rows():
    rows, n, k = 6, 20_003, 101
    x = workloads.distinct_rows(rows, n, 901)
    g = workloads.normal_f32((rows, n - k + 1), 902)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y, am = mf.MedianFilterFn.apply(xt, k)
    y.backward(torch.from_numpy(g).to(DEV))
    gx = xt.grad.cpu().numpy()
    for r in range(rows):
        yo, ao = oracle.sortmedian(x[r], k)
        assert np.array_equal(am[r].cpu().numpy(), ao)
        g32, _ = oracle.backward(g[r], ao, n, k)
        assert np.array_equal(gx[r], g32)


def test_finite_differences_on_gpu_forward():
    """FD slice: 4096 items, k = 31, step 1e-3, close neighbours separated by
    more than twice the step; L = sum(g * y) in float64 from GPU medians."""
    k, n, eps = 31, 4096, 1e-3
    x = workloads.distinct_rows(1, n, workloads.SEEDS["fd_slice"], min_gap=2.5 * eps, window=k)[0]
    g = workloads.normal_f32(n - k + 1, workloads.SEEDS["fd_slice"] + 1000)
    _, am, gx = gpu_forward_backward(x, k, g)
    rng = np.random.default_rng(1)
    probe = np.concatenate([rng.choice(n, 64, replace=False), np.unique(am)[:64]])
    xs = np.repeat(x[None, :], 2 * len(probe), axis=0)
    for q, j in enumerate(probe):
        xs[2 * q, j] = np.float32(x[j] + eps)
        xs[2 * q + 1, j] = np.float32(x[j] - eps)
    yb, _ = mf.median_filter(torch.from_numpy(np.ascontiguousarray(xs)).to(DEV), k)
    yb = yb.cpu().numpy().astype(np.float64)
    L = yb @ g.astype(np.float64)
    for q, j in enumerate(probe):
        fd = (L[2 * q] - L[2 * q + 1]) / (float(xs[2 * q, j]) - float(xs[2 * q + 1, j]))
        assert abs(fd - gx[j]) <= 1e-4 * (1 + abs(fd)), (j, fd, gx[j])


@pytest.mark.parametrize("k", [1, 3, 101, 1001, 1025, 1027, 4095])
def test_backward_f64_bitwise_vs_oracle(k):
    """float64 signal and gradient: forward on the GPU, backward on the GPU
    against the oracle's float64 scatter, bit for bit."""
    from paper_1406_1717_amd import workloads
    n = max(3 * k, 30_000) + 11
    x = workloads.random_walk_f64(n, 40 + k)
    g = np.random.default_rng(41 + k).standard_normal(n - k + 1)
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y, am = mf.MedianFilterFn.apply(xt, k)
    y.backward(torch.from_numpy(g).to(DEV))
    torch.cuda.synchronize()
    _, ao = oracle.sortmedian(x, k)
    assert np.array_equal(am.cpu().numpy(), ao)
    want = oracle.backward_f64(g, ao, n, k)
    got = xt.grad.cpu().numpy()
    assert got.dtype == np.float64
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


def test_backward_f64_gradcheck():
    """torch.autograd.gradcheck in float64 on well-separated values."""
    n, k = 600, 31
    x = torch.from_numpy(np.random.default_rng(42).permutation(n).astype(np.float64) * 1e-2).to(DEV)
    x.requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: mf.MedianFilterFn.apply(t, k)[0], (x,), eps=1e-6, atol=1e-7)


def test_backward_f64_rows():
    """float64 rows through autograd: each row's gradient bit for bit against
    the oracle's float64 scatter."""
    rows, n, k = 3, 20_011, 101
    x = np.stack([workloads.random_walk_f64(n, 60 + r) for r in range(rows)])
    g = np.random.default_rng(61).standard_normal((rows, n - k + 1))
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y, am = mf.MedianFilterFn.apply(xt, k)
    y.backward(torch.from_numpy(g).to(DEV))
    torch.cuda.synchronize()
    got = xt.grad.cpu().numpy()
    for r in range(rows):
        _, ao = oracle.sortmedian(x[r], k)
        assert np.array_equal(am[r].cpu().numpy(), ao)
        want = oracle.backward_f64(g[r], ao, n, k)
        assert np.array_equal(got[r].view(np.uint64), want.view(np.uint64)), r
