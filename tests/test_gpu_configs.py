"""The benchmark workloads at full size on the GPU, against the CPU oracle.

  uniform_f32_1m        float32 U[0,1), n = 10^6, k = 101        full compare
  int32_full_64m        int32 full range, n = 2^26, k = 1001     full compare
  int32_bytes_64m       int32 in 0..255, n = 2^26, k = 1001      full compare
  random_walk_f32_16m   n = 2^24, k in {3, 31, 301, 3001, 30001}, and the
                        same walk sorted                          full compare
  ragged_impulse_10k    10,000 ragged signals (about 1.47e9 items)
                        every signal whole, under every launch
                        configuration and the autotuned one
  distinct_normal_256   256 x 262,144, k = 201, forward + backward
                        every row whole, gradient bit for bit and within
                        1e-6 relative of the float64 sums
The launch configurations include the ones bench.py times.  The oracle
runs in host threads (its C functions release the GIL).
"""
import os
from concurrent.futures import ThreadPoolExecutor

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
    yo, ao = oracle.sortmedian_parallel(x, k, threads=_threads())
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


def _threads():
    return max(1, min(16, os.cpu_count() or 1))


def _check_signals(x, off, ks, yo, results, label):
    """Every signal of a packed batch against the oracle (threads over
    signals): argmed equal, y the bit copy of x at the oracle's argmed.
    results: [(name, y_host, argmed_host)] of the launch configurations."""
    def one(s):
        xs = x[off[s]:off[s + 1]]
        _, ao = oracle.sortmedian(xs, int(ks[s]))
        want_y = xs[ao].view(np.uint32)
        for name, y, am in results:
            if not np.array_equal(am[yo[s]:yo[s + 1]], ao):
                bad = np.nonzero(am[yo[s]:yo[s + 1]] != ao)[0]
                return "%s %s signal %d (k=%d, n=%d): %d argmed mismatches, first %s" % (
                    label, name, s, ks[s], len(xs), bad.size, bad[:5])
            if not np.array_equal(y[yo[s]:yo[s + 1]].view(np.uint32), want_y):
                return "%s %s signal %d: y differs" % (label, name, s)
        return None

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        errs = [e for e in ex.map(one, range(len(ks))) if e]
    assert not errs, errs[:5]


@pytest.mark.timeout(1200)
def test_ragged_impulse_10k():
    """All 10,000 signals (about 1.47e9 outputs), whole, against the oracle,
    under every launch configuration of the plan: the one-call entry's
    (persistent), each configuration set explicitly, and the one the
    autotuner picks (the one the benchmark times)."""
    x, off, ks = workloads.ragged_impulse(10_000, workloads.SEEDS["ragged_impulse_10k"])
    print("  ragged: %d signals, %d items" % (len(ks), off[-1]), flush=True)
    yo = mf.output_offsets(off, ks)
    nout = int(yo[-1])
    xt = torch.from_numpy(x).to(DEV)
    results = []
    y, am = mf.median_filter_batched(xt, off, ks)
    torch.cuda.synchronize()
    mf.lib.mf_check_device_error()
    results.append(("one-call", y.cpu().numpy(), am.cpu().numpy()))
    plan = mf.Plan(off, ks)
    for config in (0, 1, 2):
        plan.set_config(config)
        y.fill_(-1.0)
        am.fill_(-1)
        plan.execute(xt, y, am)
        torch.cuda.synchronize()
        results.append(("config %d" % config, y.cpu().numpy(), am.cpu().numpy()))
    tune = plan.autotune(xt, y, am, reps=1)
    y.fill_(-1.0)
    am.fill_(-1)
    plan.execute(xt, y, am)
    torch.cuda.synchronize()
    mf.lib.mf_check_device_error()
    results.append(("autotuned (config %d)" % tune["config"], y.cpu().numpy(), am.cpu().numpy()))
    plan.close()
    del xt, y, am
    print("  ragged: %d outputs per configuration, oracle on %d threads" % (nout, _threads()), flush=True)
    _check_signals(x, off, ks, yo, results, "ragged_impulse_10k")


@pytest.mark.timeout(600)
def test_distinct_normal_256_fwd_bwd():
    """All 256 rows: forward (y, argmed) against the oracle, and the
    autograd backward bit for bit against the oracle's scatter of the
    oracle's argmed (and within 1e-6 of its float64 sums)."""
    rows, n, k = 256, 262_144, 201
    x = workloads.distinct_rows(rows, n, workloads.SEEDS["distinct_normal_256"])
    g = workloads.normal_f32((rows, n - k + 1), workloads.SEEDS["distinct_normal_256_grad"])
    xt = torch.from_numpy(x).to(DEV).requires_grad_(True)
    y, am = mf.MedianFilterFn.apply(xt, k)
    y.backward(torch.from_numpy(g).to(DEV))
    torch.cuda.synchronize()
    amh = am.cpu().numpy()
    yh = y.detach().cpu().numpy()
    gx = xt.grad.cpu().numpy()

    def one(r):
        _, ao = oracle.sortmedian(x[r], k)
        if not np.array_equal(amh[r], ao):
            return "row %d: argmed differs" % r
        if not np.array_equal(yh[r].view(np.uint32), x[r][ao].view(np.uint32)):
            return "row %d: y differs" % r
        g32, g64 = oracle.backward(g[r], ao, n, k)
        if not np.array_equal(gx[r].view(np.uint32), g32.view(np.uint32)):
            return "row %d: grad_x differs" % r
        nz = g64 != 0
        if not (np.all(np.abs(gx[r][nz] - g64[nz]) <= 1e-6 * np.abs(g64[nz])) and np.all(gx[r][~nz] == 0)):
            return "row %d: grad_x outside 1e-6 of the float64 sums" % r
        return None

    with ThreadPoolExecutor(max_workers=_threads()) as ex:
        errs = [e for e in ex.map(one, range(rows)) if e]
    assert not errs, errs[:5]


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
