"""GPU forward at the size limits, against the oracle.

  * the longest signal, n = 2^31 - 1 (the largest argmed index), k = 1001:
    sampled windows (the first, the last and random ones) against the
    definition oracle, and every argmed inside its window;
  * the widest window, k = 32767, over several tiles with a ragged last
    block: every output against the paper's method in the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1406_1717_amd as mf
from paper_1406_1717_amd import lib

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def test_longest_signal():
    n, k = 2**31 - 1, 1001
    nout = n - k + 1
    print("longest signal: n=%d k=%d" % (n, k), flush=True)
    gen = torch.Generator(device=DEV)
    gen.manual_seed(901)
    x = torch.rand(n, device=DEV, generator=gen)
    y, am = mf.median_filter(x, k)
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    rng = np.random.default_rng(902)
    outs = np.unique(np.concatenate([[0, 1, nout // 2, nout - 2, nout - 1],
                                     rng.integers(0, nout, 1000),
                                     nout - 1 - rng.integers(0, 3 * k, 200)])).astype(np.int64)
    idx = torch.from_numpy(outs).to(DEV)[:, None] + torch.arange(k, device=DEV)[None, :]
    wins = x[idx].cpu().numpy()
    got_a = am[torch.from_numpy(outs).to(DEV)].cpu().numpy()
    got_y = y[torch.from_numpy(outs).to(DEV)].cpu().numpy()
    for q, o in enumerate(outs):
        rel = int(oracle.window_median(wins[q], k, np.array([0]))[0])
        assert got_a[q] == o + rel, (o, got_a[q], o + rel)
        assert got_y[q].view(np.uint32) == wins[q][rel].view(np.uint32)
    del idx, wins
    step = 1 << 28
    for start in range(0, nout, step):
        end = min(nout, start + step)
        o = torch.arange(start, end, device=DEV, dtype=torch.int64)
        a = am[start:end].to(torch.int64)
        assert bool(((a >= o) & (a < o + k)).all()), start
        del o, a


@pytest.mark.parametrize("dtype", ["f32", "i32"])
def test_widest_window(dtype):
    k = 32767
    rng = np.random.default_rng(903)
    n = 5 * k + 12_345
    x = rng.standard_normal(n).astype(np.float32) if dtype == "f32" else rng.integers(0, 50, n).astype(np.int32)
    xt = torch.from_numpy(x).to(DEV)
    y, am = mf.median_filter(xt, k)
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    yo, ao = oracle.sortmedian(x, k)
    assert np.array_equal(am.cpu().numpy(), ao)
    assert np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32))
