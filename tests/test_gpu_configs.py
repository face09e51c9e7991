"""The benchmark workloads at full size on the GPU, against the CPU oracle.

  uniform_f32_1m        float32 U[0,1), n = 10^6, k = 101        full compare
  int32_full_64m        int32 full range, n = 2^26, k = 1001     full compare
  int32_bytes_64m       int32 in 0..255, n = 2^26, k = 1001      full compare
  random_walk_f32_16m   n = 2^24, k in {3, 31, 301, 3001, 30001}, and the
                        same walk sorted                          full compare
  ragged_impulse_10k    10,000 ragged signals (about 1.47e9 items)
                        40 whole signals, 20,000 sampled windows
  distinct_normal_256   256 x 262,144, k = 201, forward + backward
                        8 whole rows, sampled windows on all rows, float64
                        reference gradient within 1e-6 relative
The launch configuration is the one bench.py times (one call per signal or
batch through the C ABI).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1406_1717_amd as mf
from paper_1406_1717_amd import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def run(x, k):
    y, am = mf.median_filter(torch.from_numpy(x).to(DEV), k)
    torch.cuda.synchronize()
    mf.lib.mf_check_device_error()
    return y.cpu().numpy(), am.cpu().numpy()


def full_compare(x, k, tag):
    print("  %s: n=%d k=%d" % (tag, len(x), k), flush=True)
    y, am = run(x, k)
    yo, ao = oracle.sortmedian(x, k)
    bad = np.nonzero(am != ao)[0]
    assert bad.size == 0, "%s k=%d: %d mismatches, first %s" % (tag, k, bad.size, bad[:5])
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))


def test_uniform_f32_1m():
    w = workloads.workload("uniform_f32_1m")
    full_compare(w["x"], w["k"], "uniform_f32_1m")


@pytest.mark.parametrize("name", ["int32_full_64m", "int32_bytes_64m"])
def test_int32_64m(name):
    w = workloads.workload(name)
    full_compare(w["x"], w["k"], name)


@pytest.mark.parametrize("name", ["random_walk_f32_16m", "sorted_walk_f32_16m"])
def test_walk_window_sweep(name):
    w = workloads.workload(name)
    for k in w["ks"]:
        full_compare(w["x"], k, name)
    if name == "sorted_walk_f32_16m":
        # nondecreasing input: the median of window o is item o + h
        x = w["x"]
        for k in w["ks"]:
            _, am = run(x, k)
            assert np.array_equal(am, np.arange(len(x) - k + 1) + (k - 1) // 2)


def test_ragged_impulse_10k():
    x, off, ks = workloads.ragged_impulse(10_000, workloads.SEEDS["ragged_impulse_10k"])
    print("  ragged: %d signals, %d items" % (len(ks), off[-1]), flush=True)
    xt = torch.from_numpy(x).to(DEV)
    y, am = mf.median_filter_batched(xt, off, ks)
    torch.cuda.synchronize()
    mf.lib.mf_check_device_error()
    yo = mf.output_offsets(off, ks)
    rng = np.random.default_rng(0)
    # whole signals, including the longest window and the longest signal
    sig = set(rng.choice(len(ks), 38, replace=False).tolist())
    sig.add(int(np.argmax(ks)))
    sig.add(int(np.argmax(off[1:] - off[:-1])))
    for s in sorted(sig):
        a = am[yo[s]:yo[s + 1]].cpu().numpy()
        v = y[yo[s]:yo[s + 1]].cpu().numpy()
        vo, ao = oracle.sortmedian(x[off[s]:off[s + 1]], int(ks[s]))
        assert np.array_equal(a, ao), "signal %d" % s
        assert np.array_equal(v.view(np.uint32), vo.view(np.uint32))
    # sampled windows over every signal
    s_idx = rng.integers(0, len(ks), 20_000)
    nout = (off[1:] - off[:-1]) - ks + 1
    o_loc = (rng.random(20_000) * nout[s_idx]).astype(np.int64)
    got = am[torch.from_numpy(yo[s_idx] + o_loc).to(DEV)].cpu().numpy()
    for q in range(20_000):
        s = s_idx[q]
        ref = oracle.window_median(x[off[s]:off[s + 1]], int(ks[s]), o_loc[q:q + 1])
        assert got[q] == ref[0], (s, o_loc[q])


def test_distinct_normal_256_fwd_bwd():
    rows, n, k = 256, 262_144, 201
    x = workloads.distinct_rows(rows, n, workloads.SEEDS["distinct_normal_256"])
    g = workloads.normal_f32((rows, n - k + 1), workloads.SEEDS["distinct_normal_256_grad"])
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y, am = mf.MedianFilterFn.apply(xt, k)
    y.backward(torch.from_numpy(g).to(DEV))
    torch.cuda.synchronize()
    amh = am.cpu().numpy()
    gx = xt.grad.cpu().numpy()
    rng = np.random.default_rng(3)
    for r in rng.choice(rows, 8, replace=False):
        yo, ao = oracle.sortmedian(x[r], k)
        assert np.array_equal(amh[r], ao), "row %d" % r
        g32, g64 = oracle.backward(g[r], ao, n, k)
        assert np.array_equal(gx[r], g32)
        nz = g64 != 0
        assert np.all(np.abs(gx[r][nz] - g64[nz]) <= 1e-6 * np.abs(g64[nz]))
    for r in range(rows):
        outs = rng.integers(0, n - k + 1, 64)
        assert np.array_equal(amh[r][outs], oracle.window_median(x[r], k, outs)), "row %d" % r


def test_workspace_limit_and_log(monkeypatch, capfd):
    """MF_WS_LIMIT makes workspace requests above it fail with
    MF_ERR_NOMEM before anything is enqueued (the outputs stay untouched),
    and the library works again without it; MF_LOG=1 reports plan and
    autotune decisions on stderr."""
    import paper_1406_1717_amd as mf
    from paper_1406_1717_amd import lib
    import oracle
    dev = torch.device("cuda:0")
    n, k = 40_000, 5001
    x = torch.from_numpy(workloads.random_walk_f32(n, 7)).to(dev)
    y = torch.full((n - k + 1,), -1.0, device=dev)
    am = torch.full((n - k + 1,), -1, dtype=torch.int32, device=dev)
    monkeypatch.setenv("MF_WS_LIMIT", "4096")
    with pytest.raises(lib.MFError) as e:
        lib.mf_median_filter(x, n, k, y, am)
    assert e.value.status == 3 and "MF_WS_LIMIT" in str(e.value)
    torch.cuda.synchronize()
    assert bool((am == -1).all())
    x64 = torch.from_numpy(workloads.int64_words(n, 8)).to(dev)
    with pytest.raises(lib.MFError) as e:
        mf.median_filter(x64, 3001)
    assert e.value.status == 3
    monkeypatch.delenv("MF_WS_LIMIT")
    y2, am2 = mf.median_filter(x, k)
    torch.cuda.synchronize()
    assert np.array_equal(am2.cpu().numpy(), oracle.sortmedian(x.cpu().numpy(), k)[1])
    monkeypatch.setenv("MF_LOG", "1")
    off = np.array([0, 20_000, 45_000], dtype=np.int64)
    ks = np.array([101, 3001], dtype=np.int32)
    xb = torch.from_numpy(workloads.uniform_f32(45_000, 9)).to(dev)
    yb = torch.empty(45_000 - 100 - 3000, device=dev)
    ab = torch.empty_like(yb, dtype=torch.int32)
    plan = mf.Plan(off, ks)
    plan.autotune(xb, yb, ab, reps=1)
    plan.close()
    err = capfd.readouterr().err
    assert "mf: plan of 2 signals" in err and "mf: autotune" in err
