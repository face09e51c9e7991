"""Concurrent use: calls on two HIP streams from two host threads at once,
on the paths that share the library's workspace (windows above 4096 and
64-bit signals) and on the LDS path, each result against the oracle.  The
header states that entry points may be called from several host threads;
workspace users are serialized by an event."""
import threading

import numpy as np
import pytest
import torch

import oracle
import paper_1406_1717_amd as mf
from paper_1406_1717_amd import lib, workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _case(kind, k, seed):
    n = 3 * k + 5003
    if kind == "f32":
        return workloads.random_walk_f32(n, seed), k
    if kind == "i64":
        return workloads.int64_words(n, seed), k
    return workloads.f64_specials(n, seed), k


CASES = [("f32", 5001, 1), ("f32", 20001, 2), ("i64", 3001, 3), ("f64", 9999, 4), ("f32", 101, 5),
         ("i64", 1001, 6)]


def test_two_streams_two_threads():
    inputs = [_case(kind, k, seed) for kind, k, seed in CASES]
    want = [oracle.sortmedian(x, k)[1] for x, k in inputs]
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    results = {}
    errors = []

    def worker(w):
        try:
            with torch.cuda.stream(streams[w]):
                for rep in range(3):
                    for c in range(w, len(inputs), 2):
                        x, k = inputs[c]
                        xt = torch.from_numpy(x).to(DEV, non_blocking=False)
                        y, am = mf.median_filter(xt, k)
                        streams[w].synchronize()
                        results[(c, rep)] = (y.cpu().numpy(), am.cpu().numpy())
        except Exception as e:   # reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(w,)) for w in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    for (c, rep), (y, am) in results.items():
        x, k = inputs[c]
        assert np.array_equal(am, want[c]), (CASES[c], rep)
        assert np.array_equal(y.view(np.uint8), x[want[c]].view(np.uint8)), (CASES[c], rep)
    assert len(results) == 3 * len(inputs)


def test_lease_held_while_others_call(monkeypatch):
    """Each workspace lease waits 0.2 s before its launches are enqueued
    (MF_LEASE_HOLD_US), so the other thread reaches the workspace while it
    is held; the second window needs more workspace than the first, so a
    thread that got in would also have to grow (free) the buffer the first
    one is about to use.  Both results must match the oracle."""
    monkeypatch.setenv("MF_LEASE_HOLD_US", "200000")
    cases = [(workloads.random_walk_f32(60_000, 31), 5001), (workloads.random_walk_f32(150_000, 32), 30001),
             (workloads.int64_words(40_000, 33), 3001), (workloads.random_walk_f32(70_000, 34), 16385)]
    want = [oracle.sortmedian(x, k)[1] for x, k in cases]
    streams = [torch.cuda.Stream() for _ in cases]
    xs = [torch.from_numpy(x).to(DEV) for x, _ in cases]
    torch.cuda.synchronize()
    out = {}
    errors = []

    def worker(c):
        try:
            with torch.cuda.stream(streams[c]):
                y, am = mf.median_filter(xs[c], cases[c][1])
                streams[c].synchronize()
                out[c] = (y.cpu().numpy(), am.cpu().numpy())
        except Exception as e:   # reported below
            errors.append(e)

    threads = [threading.Thread(target=worker, args=(c,)) for c in range(len(cases))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    lib.mf_check_device_error()
    for c, (x, k) in enumerate(cases):
        y, am = out[c]
        assert np.array_equal(am, want[c]), c
        assert np.array_equal(y.view(np.uint8), x[want[c]].view(np.uint8)), c


def test_batched_same_layout_two_streams():
    """Two one-call batched forwards with the same layout (so the same
    cached plan, with its persistent work counters) on two streams, enqueued
    back to back without a synchronization between them, on different
    data: both results against the oracle per signal."""
    rng = np.random.default_rng(77)
    lens = rng.integers(2_000, 60_000, 40)
    ks = np.array([min(int(2 * rng.integers(1, 1500) + 1), int(L) - (1 - L % 2)) for L in lens], dtype=np.int32)
    ks = np.where(ks % 2 == 0, ks - 1, ks).astype(np.int32)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xa = rng.standard_normal(int(off[-1])).astype(np.float32)
    xb = np.cumsum(rng.standard_normal(int(off[-1]))).astype(np.float32)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ta, tb = torch.from_numpy(xa).to(DEV), torch.from_numpy(xb).to(DEV)
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        ya, aa = mf.median_filter_batched(ta, off, ks)
    with torch.cuda.stream(s2):
        yb, ab = mf.median_filter_batched(tb, off, ks)
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    yo = mf.output_offsets(off, ks)
    for x, am in ((xa, aa.cpu().numpy()), (xb, ab.cpu().numpy())):
        for s in range(len(ks)):
            _, ao = oracle.sortmedian(x[off[s]:off[s + 1]], int(ks[s]))
            assert np.array_equal(am[yo[s]:yo[s + 1]], ao), s
