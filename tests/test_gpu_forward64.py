"""GPU forward parity for 64-bit signals (float64, int64): HIP path vs the
CPU oracle.  Medians (bit patterns) and argmedians must be identical.

Cases: every window family (k = 1; 512- and 1024-thread tiles up to
k = 4095; one-pair tiles of the workspace path up to k = 32767), several
tiles and ragged last blocks,
n = k and n = k + 1, values ordered only by their high or only by their low
32-bit word, float64 specials, presorted signals, argmed = NULL, the
full-size workloads on sampled windows, the paper's generator families,
and the argument errors.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1406_1717_amd as mf
from paper_1406_1717_amd import lib, workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")
KS = [1, 3, 5, 7, 15, 31, 33, 101, 129, 301, 701, 1001, 1025, 2047, 2049, 3001, 4095,
      4097, 5001, 8191, 9999, 16385, 20001, 32767]
GENS = {"f64_specials": workloads.f64_specials, "int64_words": workloads.int64_words,
        "int64_full": workloads.int64_full, "walk_f64": workloads.random_walk_f64}


def run_gpu(x, k, with_argmed=True):
    xt = torch.from_numpy(x).to(DEV)
    y, am = mf.median_filter(xt, k, with_argmed=with_argmed)
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    return y.cpu().numpy(), (am.cpu().numpy() if am is not None else None)


def assert_same(x, k, y, am, tag=""):
    yo, ao = oracle.sortmedian(x, k)
    if am is not None:
        bad = np.nonzero(am != ao)[0]
        assert bad.size == 0, "%s k=%d n=%d: %d argmed mismatches, first at %s (gpu %s, oracle %s)" % (
            tag, k, len(x), bad.size, bad[:5], am[bad[:5]], ao[bad[:5]])
    assert np.array_equal(y.view(np.uint64), yo.view(np.uint64)), tag


@pytest.mark.parametrize("kind", sorted(GENS))
@pytest.mark.parametrize("k", KS)
def test_64bit_several_tiles(kind, k):
    rng = np.random.default_rng(3000 + k)
    n = int(max(3 * k, 12_000) + rng.integers(0, k + 1))     # ragged last block
    x = GENS[kind](n, 3100 + k)
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, kind)


@pytest.mark.parametrize("k", [21, 201, 2001, 3001, 5001])
def test_paper_families_int64(k):
    # the seven generator families of Section 7.3 at 64 bits, on every
    # 64-bit tile kind (in-tile ranks, rank pre-pass, pair pre-pass)
    for fam in ("asc", "desc", "r-asc", "r-desc", "r-large", "r-small", "r-block"):
        x = workloads.paper_family(fam, 40_000 + k // 3, seed=70 + k, bits=64)
        y, am = run_gpu(x, k)
        assert_same(x, k, y, am, fam)


@pytest.mark.parametrize("k", [1, 3, 101, 1001, 2049, 4095, 5001, 32767])
def test_64bit_degenerate_lengths(k):
    for n in (k, k + 1, 2 * k - 1, 2 * k, 2 * k + 1):
        for x in (workloads.f64_specials(n, n), workloads.int64_words(n, n)):
            y, am = run_gpu(x, k)
            assert_same(x, k, y, am, "n=%d" % n)


@pytest.mark.parametrize("k", [3, 301, 3001, 9999])
def test_64bit_presorted_and_reversed(k):
    n = 20_000 + 17
    walk = workloads.random_walk_f64(n, 41)
    for x in (np.sort(walk), np.sort(walk)[::-1].copy(), np.full(n, -0.0), np.arange(n, dtype=np.int64) << 32):
        y, am = run_gpu(x, k)
        assert_same(x, k, y, am, "sorted")


@pytest.mark.parametrize("k", [1, 5, 1001, 4095, 5001, 20001])
def test_64bit_without_argmed(k):
    n = 3 * k + 1000
    x = workloads.int64_words(n, 77)
    y, _ = run_gpu(x, k, with_argmed=False)
    assert_same(x, k, y, None, "no argmed")


def _sampled(x, k, am, y, count, seed):
    rng = np.random.default_rng(seed)
    n = len(x)
    outs = rng.integers(0, n - k + 1, count)
    outs[:4] = [0, 1, n - k, (n - k) // 2]
    want = oracle.window_median(x, k, outs)
    assert np.array_equal(am[outs], want)
    assert np.array_equal(y[outs].view(np.uint64), x[want].view(np.uint64))
    # every argmed lies in its window
    o = np.arange(n - k + 1)
    assert np.all((am >= o) & (am < o + k))


def test_64bit_full_size_int64_full_64m():
    w = workloads.workload("int64_full_64m")
    x, k = w["x"], w["k"]
    y, am = run_gpu(x, k)
    _sampled(x, k, am, y, 3000, 5)


@pytest.mark.parametrize("k", [301, 3001, 30001])
def test_64bit_full_size_random_walk_f64_16m(k):
    x = workloads.workload("random_walk_f64_16m")["x"]
    y, am = run_gpu(x, k)
    _sampled(x, k, am, y, 3000, 6)


def test_64bit_errors():
    x = torch.zeros(10_000, dtype=torch.float64, device=DEV)
    y = torch.empty(10_000, dtype=torch.float64, device=DEV)
    am = torch.empty(10_000, dtype=torch.int32, device=DEV)
    for k, status in ((2, 1), (0, 1), (10_001, 1)):
        with pytest.raises(lib.MFError) as e:
            lib.mf_median_filter_f64(x, 10_000, k, y, am)
        assert e.value.status == status, k
    big = torch.zeros(40_000, dtype=torch.float64, device=DEV)
    with pytest.raises(lib.MFError) as e:
        lib.mf_median_filter_f64(big, 40_000, 32769, y, am)
    assert e.value.status == 2
    assert lib.load().mf_median_filter_i64(None, 100, 3, ctypes.c_void_p(y.data_ptr()), None, None) == 1
    # the library stays usable after the errors
    xs = workloads.int64_words(5000, 1)
    yy, aa = run_gpu(xs, 101)
    assert_same(xs, 101, yy, aa, "after errors")


@pytest.mark.parametrize("k", [1, 101, 1001, 3001, 5001, 20001])
@pytest.mark.parametrize("dtype", ["f64", "i64"])
def test_64bit_rows(dtype, k):
    """64-bit rows on every path (k = 1, in-LDS ranking, the 1024-thread
    pre-pass, the pair pre-pass): each row against the oracle."""
    rows = 3
    n = 2 * k + 3001
    gen = workloads.f64_specials if dtype == "f64" else workloads.int64_words
    x = np.stack([gen(n, 900 + 10 * k + r) for r in range(rows)])
    y, am = mf.median_filter(torch.from_numpy(x).to(DEV), k)
    torch.cuda.synchronize()
    lib.mf_check_device_error()
    y = y.cpu().numpy()
    am = am.cpu().numpy()
    for r in range(rows):
        yo, ao = oracle.sortmedian(x[r], k)
        assert np.array_equal(am[r], ao), (dtype, k, r)
        assert np.array_equal(y[r].view(np.uint64), yo.view(np.uint64)), (dtype, k, r)
