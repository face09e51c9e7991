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
