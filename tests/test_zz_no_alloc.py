"""The entry point that allocates nothing (mf_median_filter_noalloc), through
the C ABI, against mf_median_filter on the same inputs: medians and
argmedians bit for bit.  Two calls in a row on the fixed device scratch,
the second on a smaller input, for each kernel family: windows above 4096
(the global path, whose per-workgroup slots live in the fixed scratch),
the LDS tiles and k = 1."""
import numpy as np
import pytest
import torch

from paper_1406_1717_amd import lib, workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def both(x, k):
    n = x.numel()
    nout = n - k + 1
    y0 = torch.empty(nout, dtype=torch.float32, device=DEV)
    a0 = torch.empty(nout, dtype=torch.int32, device=DEV)
    y1 = torch.full((nout,), float("nan"), dtype=torch.float32, device=DEV)
    a1 = torch.full((nout,), -1, dtype=torch.int32, device=DEV)
    lib.mf_median_filter(x, n, k, y0, a0)
    lib.mf_median_filter_noalloc(x, n, k, y1, a1)
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    return (y0.cpu().numpy().view(np.uint32), a0.cpu().numpy(),
            y1.cpu().numpy().view(np.uint32), a1.cpu().numpy())


@pytest.mark.parametrize("first,second", [
    ((4_000_003, 30001, 701), (300_001, 5001, 702)),    # global path, 42 then 59 slots
    ((2_500_000, 16385, 703), (200_000, 9001, 704)),    # 128 KB then 64 KB tiles
    ((1_000_000, 1001, 705), (50_001, 101, 706)),       # LDS tiles
    ((100_000, 3001, 707), (1_000, 1, 708)),            # 1024-thread tiles, then k = 1
])
def test_noalloc_matches_mf_median_filter(first, second):
    for n, k, seed in (first, second):
        print("noalloc: n=%d k=%d seed=%d" % (n, k, seed), flush=True)
        x = torch.from_numpy(workloads.random_walk_f32(n, seed)).to(DEV)
        y0, a0, y1, a1 = both(x, k)
        assert np.array_equal(a1, a0), (n, k)
        assert np.array_equal(y1, y0), (n, k)


def test_noalloc_argmed_null_and_errors():
    n, k = 200_000, 20001
    x = torch.from_numpy(workloads.random_walk_f32(n, 709)).to(DEV)
    y0 = torch.empty(n - k + 1, device=DEV)
    y1 = torch.empty(n - k + 1, device=DEV)
    lib.mf_median_filter(x, n, k, y0, None)
    lib.mf_median_filter_noalloc(x, n, k, y1, None)
    torch.cuda.synchronize()
    assert torch.equal(y0.view(torch.int32), y1.view(torch.int32))
    with pytest.raises(lib.MFError):
        lib.mf_median_filter_noalloc(x, n, 4, y1, None)
    with pytest.raises(lib.MFError):
        lib.mf_median_filter_noalloc(x, n, 32769, y1, None)
