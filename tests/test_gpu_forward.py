"""GPU forward parity: HIP path vs the CPU oracle, element by element.

Medians (bit patterns) and argmedians must be identical.  Cases span every
kernel family (k = 1; LDS tiles with 256 and 512 threads; the global-memory
path above k = 4096), several tiles per launch and ragged last blocks, the
degenerate shapes (n = k, one output; n = k + 1; k = 1) and float specials.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1406_1717_amd as mf
from paper_1406_1717_amd import workloads

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def run_gpu(x, k):
    xt = torch.from_numpy(x).to(DEV)
    y, am = mf.median_filter(xt, k)
    torch.cuda.synchronize()
    mf.lib.mf_check_device_error()
    return y.cpu().numpy(), am.cpu().numpy()


def assert_same(x, k, y, am, tag=""):
    yo, ao = oracle.sortmedian(x, k)
    bad = np.nonzero(am != ao)[0]
    assert bad.size == 0, "%s k=%d n=%d: %d argmed mismatches, first at %s (gpu %s, oracle %s)" % (
        tag, k, len(x), bad.size, bad[:5], am[bad[:5]], ao[bad[:5]])
    assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), tag


KS = [1, 3, 5, 7, 15, 17, 31, 33, 63, 65, 101, 129, 255, 301, 511, 513, 1001, 1023, 1025,
      2047, 2049, 3001, 4001, 4095, 4097, 5001, 8191, 9999]


@pytest.mark.parametrize("k", KS)
def test_float_random_several_tiles(k):
    rng = np.random.default_rng(1000 + k)
    n = int(max(3 * k, 20_000) + rng.integers(0, k + 1))     # ragged last block
    x = rng.standard_normal(n).astype(np.float32)
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, "f32")


@pytest.mark.parametrize("k", KS)
def test_int_duplicates(k):
    rng = np.random.default_rng(2000 + k)
    n = int(max(3 * k, 20_000) + rng.integers(0, k + 1))
    x = rng.integers(0, 7, n).astype(np.int32)
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, "i32 dup")


@pytest.mark.parametrize("k", [3, 101, 1001, 4001, 5001])
def test_int_full_range(k):
    rng = np.random.default_rng(3000 + k)
    n = 5 * k + 77
    x = rng.integers(-2**31, 2**31, n, dtype=np.int32)
    x[::97] = np.iinfo(np.int32).min
    x[::89] = np.iinfo(np.int32).max
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, "i32 full")


@pytest.mark.parametrize("k", [3, 9, 101, 1001, 4095, 4097])
def test_float_specials(k):
    rng = np.random.default_rng(4000 + k)
    n = 4 * k + 13
    x = rng.standard_normal(n).astype(np.float32)
    pool = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1.0, -1.0], np.float32)
    m = rng.random(n) < 0.4
    x[m] = rng.choice(pool, int(m.sum()))
    x[rng.integers(0, n)] = np.frombuffer(np.uint32(0x7FC00123).tobytes(), np.float32)[0]
    x[rng.integers(0, n)] = np.frombuffer(np.uint32(0xFF800001).tobytes(), np.float32)[0]
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, "specials")


@pytest.mark.parametrize("k", [4097, 5001, 9999, 20001])
def test_global_tiles_crowded_maps(k):
    """Global-memory tiles (k > 4096): N(0,1) with 5 % impulses of +-50 (the
    linear bucket map crowds, the logarithmic one is used), values with
    moderate ties (0..3999), and a second pair of windows per launch."""
    rng = np.random.default_rng(6000 + k)
    n = 3 * k + int(rng.integers(0, k))
    x = rng.standard_normal(n).astype(np.float32)
    m = rng.random(n) < 0.05
    x[m] = rng.uniform(-50, 50, int(m.sum())).astype(np.float32)
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, "impulse")
    xi = rng.integers(0, 4000, n).astype(np.int32)
    y, am = run_gpu(xi, k)
    assert_same(xi, k, y, am, "ties 0..3999")


@pytest.mark.parametrize("k", [5001, 16383, 16385, 30001, 32767])
def test_workspace_path_windows(k):
    """The k > 4096 path on both sides of its two kernel forms (two tiles
    per CU up to k = 16383, one above): every output of a random walk and of
    full-range int32 over four pairs and a ragged last block."""
    rng = np.random.default_rng(7000 + k)
    n = 5 * k + int(rng.integers(1, k))
    print("workspace path: k=%d n=%d" % (k, n), flush=True)
    xw = np.cumsum(rng.standard_normal(n)).astype(np.float32)
    y, am = run_gpu(xw, k)
    assert_same(xw, k, y, am, "walk")
    xi = rng.integers(-2**31, 2**31, n, dtype=np.int64).astype(np.int32)
    y, am = run_gpu(xi, k)
    assert_same(xi, k, y, am, "int32")


@pytest.mark.parametrize("k,n", [(1, 1), (1, 7), (3, 3), (3, 4), (3, 5), (5, 5), (101, 101), (101, 102),
                                 (101, 202), (101, 203), (1001, 1001), (1001, 2001), (1001, 2002),
                                 (4095, 4095), (4095, 8191), (4097, 4097), (4097, 8195), (9999, 9999),
                                 (30001, 30001), (30001, 60003)])
def test_degenerate_shapes(k, n):
    rng = np.random.default_rng(k * 7 + n)
    x = rng.standard_normal(n).astype(np.float32)
    y, am = run_gpu(x, k)
    assert_same(x, k, y, am, "shape")


@pytest.mark.parametrize("k", [3, 31, 301, 3001, 30001])
def test_monotone_and_constant(k):
    n = 3 * k + 5
    h = (k - 1) // 2
    for x in (np.arange(n, dtype=np.float32), np.arange(n, 0, -1).astype(np.float32),
              np.full(n, 2.5, np.float32)):
        y, am = run_gpu(x, k)
        assert np.array_equal(am, np.arange(n - k + 1) + h)


def test_paper_families_int32():
    for fam in ("asc", "desc", "r-asc", "r-desc", "r-large", "r-small", "r-block"):
        x = workloads.paper_family(fam, 50_000, seed=5)
        for k in (21, 201, 2001):
            y, am = run_gpu(x, k)
            assert_same(x, k, y, am, fam)


def test_rows_matches_single():
    rng = np.random.default_rng(9)
    rows, n, k = 7, 5003, 201
    x = rng.standard_normal((rows, n)).astype(np.float32)
    y, am = mf.median_filter(torch.from_numpy(x).to(DEV), k)
    y = y.cpu().numpy()
    am = am.cpu().numpy()
    for r in range(rows):
        yo, ao = oracle.sortmedian(x[r], k)
        assert np.array_equal(am[r], ao) and np.array_equal(y[r], yo)


@pytest.mark.parametrize("k", [3, 201, 3001, 5001])
def test_rows_int32(k):
    """int32 rows (the LDS paths and the workspace path), each row against
    the oracle, with rows of full-range values and of heavy ties."""
    rng = np.random.default_rng(10 + k)
    rows, n = 5, 3 * k + 2001
    x = rng.integers(-2**31, 2**31, (rows, n), dtype=np.int32)
    x[1] = rng.integers(0, 5, n)
    y, am = mf.median_filter(torch.from_numpy(x).to(DEV), k)
    torch.cuda.synchronize()
    mf.lib.mf_check_device_error()
    y = y.cpu().numpy()
    am = am.cpu().numpy()
    for r in range(rows):
        yo, ao = oracle.sortmedian(x[r], k)
        assert np.array_equal(am[r], ao) and np.array_equal(y[r], yo), r


def test_without_argmed():
    rng = np.random.default_rng(10)
    x = rng.standard_normal(10_000).astype(np.float32)
    y, am = mf.median_filter(torch.from_numpy(x).to(DEV), 101, with_argmed=False)
    assert am is None
    yo, _ = oracle.sortmedian(x, 101)
    assert np.array_equal(y.cpu().numpy(), yo)


@pytest.mark.parametrize("k", [5, 101, 1001, 3001])
def test_presorted_inputs(k):
    """Ascending data (the presorted path), with ties, and with one descent
    that must send its tile through the sort."""
    rng = np.random.default_rng(900 + k)
    n = 40 * k + 17
    cases = [np.sort(rng.random(n)).astype(np.float32),
             np.sort(rng.integers(0, 40, n)).astype(np.int32),
             (np.arange(n, dtype=np.int32) // 3)]
    bump = np.sort(rng.random(n)).astype(np.float32)
    bump[n // 2] = -1.0
    cases.append(bump)
    for x in cases:
        xt = torch.from_numpy(x).to(DEV)
        y, am = mf.median_filter(xt, k)
        torch.cuda.synchronize()
        mf.lib.mf_check_device_error()
        yo, ao = oracle.sortmedian(x, k)
        assert np.array_equal(am.cpu().numpy(), ao), (k, x.dtype)
        assert np.array_equal(y.cpu().numpy().view(np.uint32), yo.view(np.uint32))
