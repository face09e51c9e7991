"""Pins for the CPU oracle: it must agree with things other than itself.

  * hand-derived cases (tests/golden/hand_cases.json),
  * two brute-force formulations on every small vector over {0,1,2},
  * closed forms: monotone / constant inputs, k = 1, k = n,
  * the lower-bound reduction of Section 2 (one filter pass sorts blocks),
  * scipy.signal.medfilt values at interior positions,
  * agreement of the paper's method (sortmedian) with the definition oracle
    (window_median) on larger inputs and on the paper's generator families,
  * planted mistakes in a copy of the oracle source must be caught.
"""
import itertools
import json
import os
import subprocess
import ctypes

import numpy as np
import pytest

import oracle
from tests.brute import rank_count_argmed, argsort_argmed
from paper_1406_1717_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_cases.json")


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _arr(case):
    dt = np.float32 if case["dtype"] == "f32" else np.int32
    return np.array([float(v) if dt == np.float32 else int(v) for v in case["x"]], dtype=dt)


def _same_bits(a, b):
    return a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))


@pytest.mark.parametrize("case", _golden()["cases"], ids=lambda c: c["name"])
def test_hand_cases(case):
    x = _arr(case)
    k = case["k"]
    want = np.array(case["argmed"], dtype=np.int32)
    y, a = oracle.sortmedian(x, k)
    assert np.array_equal(a, want)
    assert _same_bits(y, x[want])
    w = oracle.window_median(x, k, np.arange(len(x) - k + 1))
    assert np.array_equal(w, want)
    assert np.array_equal(rank_count_argmed(x, k), want)


@pytest.mark.parametrize("dtype", [np.int32, np.float32])
def test_exhaustive_small_alphabet(dtype):
    """Every vector over {0,1,2} of length 1..8, every odd k <= n."""
    for n in range(1, 9):
        vecs = np.array(list(itertools.product(range(3), repeat=n)), dtype=dtype)
        for k in range(1, n + 1, 2):
            for v in vecs:
                want = rank_count_argmed(v, k)
                y, a = oracle.sortmedian(v, k)
                assert np.array_equal(a, want), (v, k, a, want)
                assert np.array_equal(y, v[want])


def test_window_oracle_vs_brute_random():
    rng = np.random.default_rng(7)
    for _ in range(200):
        n = int(rng.integers(1, 60))
        k = int(rng.integers(0, (n + 1) // 2)) * 2 + 1
        x = rng.integers(0, 6, n).astype(np.float32)
        want = rank_count_argmed(x, k)
        got = oracle.window_median(x, k, np.arange(n - k + 1))
        assert np.array_equal(got, want)


def _special_vector(rng, n):
    pool = np.array([0.0, -0.0, 1.0, -1.0, 2.5, np.inf, -np.inf, np.nan,
                     np.nan, 3.0, 3.0, -7.0], dtype=np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    pick = rng.random(n) < 0.5
    x[pick] = rng.choice(pool, int(pick.sum()))
    # a NaN with a different payload and sign must still order as NaN
    if n > 3:
        x[rng.integers(0, n)] = np.frombuffer(np.uint32(0xFFC00001).tobytes(), np.float32)[0]
    return x


def test_random_with_specials_float():
    rng = np.random.default_rng(11)
    for _ in range(300):
        n = int(rng.integers(1, 301))
        k = int(rng.integers(0, (n + 1) // 2)) * 2 + 1
        x = _special_vector(rng, n)
        want = argsort_argmed(x, k)
        y, a = oracle.sortmedian(x, k)
        assert np.array_equal(a, want), (n, k)
        assert _same_bits(y, x[want])


def test_random_ties_int():
    rng = np.random.default_rng(12)
    for _ in range(300):
        n = int(rng.integers(1, 301))
        k = int(rng.integers(0, (n + 1) // 2)) * 2 + 1
        hi = int(rng.choice([2, 5, 50, 2**31 - 1]))
        x = rng.integers(-hi, hi, n, dtype=np.int32)
        x[rng.random(n) < 0.05] = np.iinfo(np.int32).max
        x[rng.random(n) < 0.05] = np.iinfo(np.int32).min
        want = argsort_argmed(x, k)
        y, a = oracle.sortmedian(x, k)
        assert np.array_equal(a, want), (n, k)
        assert np.array_equal(y, x[want])


@pytest.mark.parametrize("k", [1, 3, 7, 31, 101])
def test_closed_forms_monotone_constant(k):
    n = 997
    h = (k - 1) // 2
    o = np.arange(n - k + 1)
    rng = np.random.default_rng(k)
    asc = np.sort(rng.integers(0, 40, n)).astype(np.int32)      # with repeats
    desc = np.arange(n, 0, -1).astype(np.float32)               # strictly
    const = np.full(n, 3.25, dtype=np.float32)
    for x in (asc, desc, const):
        y, a = oracle.sortmedian(x, k)
        assert np.array_equal(a, o + h)
    # non-increasing with repeats: ties go to the lower index
    x = np.sort(rng.integers(0, 40, n))[::-1].astype(np.int32).copy()
    assert np.array_equal(oracle.sortmedian(x, k)[1], argsort_argmed(x, k))


def test_k_one_is_identity_and_k_n_is_global_median():
    rng = np.random.default_rng(3)
    x = rng.integers(0, 9, 501).astype(np.float32)
    y, a = oracle.sortmedian(x, 1)
    assert np.array_equal(a, np.arange(501)) and _same_bits(y, x)
    y, a = oracle.sortmedian(x, 501)
    assert a.shape == (1,)
    assert a[0] == np.argsort(x, kind="stable")[250]


@pytest.mark.parametrize("h", [1, 2, 5, 10, 50])
@pytest.mark.parametrize("dtype", [np.float32, np.int32])
def test_lower_bound_reduction(h, dtype):
    """Section 2: pad each block of h+1 items with h copies of the minimum
    before and h copies of the maximum after; one filter pass with k=2h+1
    then lists each block in sorted order."""
    rng = np.random.default_rng(100 + h)
    nblocks = 23
    if dtype == np.float32:
        lo, hi = -np.inf, np.inf
        blocks = rng.integers(-5, 5, (nblocks, h + 1)).astype(np.float32)
    else:
        lo, hi = np.iinfo(np.int32).min, np.iinfo(np.int32).max
        blocks = rng.integers(-2**31 + 1, 2**31 - 1, (nblocks, h + 1)).astype(np.int32)
    unit = 3 * h + 1
    x = np.empty(nblocks * unit, dtype=dtype)
    for b in range(nblocks):
        x[b * unit: b * unit + h] = lo
        x[b * unit + h: b * unit + 2 * h + 1] = blocks[b]
        x[b * unit + 2 * h + 1: (b + 1) * unit] = hi
    y, a = oracle.sortmedian(x, 2 * h + 1)
    for b in range(nblocks):
        assert np.array_equal(y[b * unit: b * unit + h + 1], np.sort(blocks[b]))


def test_scipy_medfilt_values_interior():
    from scipy.signal import medfilt
    rng = np.random.default_rng(5)
    for k in (3, 9, 31, 101):
        x = rng.standard_normal(4000).astype(np.float32)
        h = (k - 1) // 2
        y, _ = oracle.sortmedian(x, k)
        ref = medfilt(x, k)[h: len(x) - h]
        assert np.array_equal(y, ref.astype(np.float32))


@pytest.mark.parametrize("k", [3, 31, 301, 1001])
def test_sortmedian_vs_definition_larger(k):
    rng = np.random.default_rng(k)
    n = 60_000 + 17
    x = rng.integers(0, 200, n).astype(np.int32)
    y, a = oracle.sortmedian(x, k)
    outs = rng.integers(0, n - k + 1, 3000)
    outs[:3] = [0, n - k, (n - k) // 2]
    assert np.array_equal(oracle.window_median(x, k, outs), a[outs])


@pytest.mark.parametrize("family", ["asc", "desc", "r-asc", "r-desc", "r-large", "r-small", "r-block"])
def test_paper_families(family):
    n = 5003
    x = workloads.paper_family(family, n, seed=9)
    for k in (3, 21, 201):
        y, a = oracle.sortmedian(x, k)
        assert np.array_equal(a, argsort_argmed(x, k)), (family, k)


def test_invalid_arguments():
    x = np.zeros(10, dtype=np.float32)
    for k in (0, 2, 11, -1):
        with pytest.raises(oracle.OracleError):
            oracle.sortmedian(x, k)


# --- planted mistakes: the pins above must notice each of them -----------

MUTATIONS = [
    # delete(): the removed cursor item hands the cursor backward, not forward
    ("if (i == B->m) B->m = B->next[i];", "if (i == B->m) B->m = B->prev[i];"),
    # delete(): an item removed ahead of the cursor is not counted out
    ("else if (before_cursor(B, i)) B->ahead -= 1;", "else if (0) B->ahead -= 1;"),
    # undelete(): the cursor count moves the wrong way
    ("if (before_cursor(B, i)) B->ahead += 1;", "if (before_cursor(B, i)) B->ahead -= 1;"),
    # delete(): s drops below zero (the max(0, s-1) of the interface lost)
    ("if (B->s > 0) B->s -= 1;", "B->s -= 1;"),
    # rebalance: peeks compared by value only, so ties go to B instead of A
    ("    return pair_less(v, a, b);\n}", "    return cmp_value(v, a, b) < 0;\n}"),
    # output index off by one
    ("const int64_t o = (j - 1) * (int64_t)k + i + 1;", "const int64_t o = (j - 1) * (int64_t)k + i;"),
    # the pair order ignores the index tie-break
    ("    return a < b;\n}", "    return 0;\n}"),
]


def _build_mutant(tmp_path, old, new, idx):
    src = open(oracle._build.SRC).read()
    assert old in src, old
    path = tmp_path / ("mut%d.c" % idx)
    path.write_text(src.replace(old, new, 1))
    lib = tmp_path / ("mut%d.so" % idx)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", str(lib), str(path), "-lm"],
                   check=True)
    L = ctypes.CDLL(str(lib))
    f = L.oracle_sortmedian_i32
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    return f


@pytest.mark.parametrize("idx", range(len(MUTATIONS)))
def test_planted_mistakes_are_caught(tmp_path, idx):
    old, new = MUTATIONS[idx]
    f = _build_mutant(tmp_path, old, new, idx)
    caught = False
    for n in range(1, 8):
        for v in itertools.product(range(3), repeat=n):
            x = np.array(v, dtype=np.int32)
            for k in range(1, n + 1, 2):
                a = np.empty(n - k + 1, dtype=np.int32)
                y = np.empty(n - k + 1, dtype=np.int32)
                rc = f(x.ctypes.data, n, k, y.ctypes.data, a.ctypes.data)
                if rc != 0 or not np.array_equal(a, rank_count_argmed(x, k)):
                    caught = True
                    break
            if caught:
                break
        if caught:
            break
    assert caught, "mutation %d survived the exhaustive pin" % idx


# --- 64-bit signals (Section 7 benchmarks 32- and 64-bit versions) ---------

@pytest.mark.parametrize("dtype", [np.int64, np.float64])
def test_exhaustive_small_alphabet_64(dtype):
    """Every vector over {0,1,2} of length 1..7, every odd k <= n."""
    for n in range(1, 8):
        vecs = np.array(list(itertools.product(range(3), repeat=n)), dtype=dtype)
        for k in range(1, n + 1, 2):
            for v in vecs:
                want = rank_count_argmed(v, k)
                y, a = oracle.sortmedian(v, k)
                assert np.array_equal(a, want), (v, k, a, want)
                assert _same_bits(y, v[want])


def _special_vector_f64(rng, n):
    # values that collide in float32 but not in float64, and the specials
    pool = np.array([0.0, -0.0, 1.0, 1.0 + 2.0 ** -40, 1.0 - 2.0 ** -50, -1.0, 5e-324, -5e-324,
                     np.inf, -np.inf, np.nan, 3.0, 3.0, 1e300, -1e300], dtype=np.float64)
    x = rng.standard_normal(n)
    pick = rng.random(n) < 0.6
    x[pick] = rng.choice(pool, int(pick.sum()))
    if n > 3:
        x[rng.integers(0, n)] = np.frombuffer(np.uint64(0xFFF8000000000001).tobytes(), np.float64)[0]
    return x


def test_random_with_specials_f64():
    rng = np.random.default_rng(21)
    for _ in range(200):
        n = int(rng.integers(1, 201))
        k = int(rng.integers(0, (n + 1) // 2)) * 2 + 1
        x = _special_vector_f64(rng, n)
        want = argsort_argmed(x, k)
        assert np.array_equal(rank_count_argmed(x, k), want)
        y, a = oracle.sortmedian(x, k)
        assert np.array_equal(a, want), (n, k)
        assert _same_bits(y, x[want])
        assert np.array_equal(oracle.window_median(x, k, np.arange(n - k + 1)), want)


def _i64_vector(rng, n):
    """Values whose order is decided by the high word only, by the low word
    only, or by the sign: a comparison narrower than 64 bits fails."""
    hi = rng.choice(np.array([-2, -1, 0, 1, 7], dtype=np.int64), n)
    lo = rng.choice(np.array([0, 1, 2**31, 2**32 - 1], dtype=np.int64), n)
    x = hi * (1 << 32) + lo
    x[rng.random(n) < 0.05] = np.iinfo(np.int64).max
    x[rng.random(n) < 0.05] = np.iinfo(np.int64).min
    return x


def test_random_ties_i64():
    rng = np.random.default_rng(22)
    for _ in range(200):
        n = int(rng.integers(1, 201))
        k = int(rng.integers(0, (n + 1) // 2)) * 2 + 1
        x = _i64_vector(rng, n)
        want = argsort_argmed(x, k)
        assert np.array_equal(rank_count_argmed(x, k), want)
        y, a = oracle.sortmedian(x, k)
        assert np.array_equal(a, want), (n, k)
        assert np.array_equal(y, x[want])


@pytest.mark.parametrize("k", [3, 101, 1001])
def test_sortmedian_vs_definition_larger_64(k):
    rng = np.random.default_rng(100 + k)
    n = 30_000 + 7
    xi = _i64_vector(rng, n)
    xf = np.cumsum(rng.standard_normal(n)) * 1e-9 + 1.0   # distinct only in float64
    for x in (xi, xf):
        y, a = oracle.sortmedian(x, k)
        outs = rng.integers(0, n - k + 1, 2000)
        outs[:3] = [0, n - k, (n - k) // 2]
        assert np.array_equal(oracle.window_median(x, k, outs), a[outs])
        assert np.array_equal(argsort_argmed(x[: 3 * k + 5], k), a[: 2 * k + 6])


MUTATIONS_64 = [
    # 64-bit integers compared through a 32-bit truncation
    ("const int64_t ia = ((const int64_t *)v->x)[a];\n        const int64_t ib = ((const int64_t *)v->x)[b];",
     "const int32_t ia = (int32_t)((const int64_t *)v->x)[a];\n        const int32_t ib = (int32_t)((const int64_t *)v->x)[b];",
     "i64"),
    # doubles compared in single precision
    ("const double fa = ((const double *)v->x)[a];\n        const double fb = ((const double *)v->x)[b];",
     "const float fa = (float)((const double *)v->x)[a];\n        const float fb = (float)((const double *)v->x)[b];",
     "f64"),
    # the NaN rule dropped for doubles
    ("if (na || nb) return na - nb;\n        return (fa > fb) - (fa < fb);\n    }\n    case T_I64",
     "return (fa > fb) - (fa < fb);\n    }\n    case T_I64", "f64"),
]


@pytest.mark.parametrize("idx", range(len(MUTATIONS_64)))
def test_planted_mistakes_64_are_caught(tmp_path, idx):
    old, new, tag = MUTATIONS_64[idx]
    src = open(oracle._build.SRC).read()
    assert old in src, old
    path = tmp_path / ("mut64_%d.c" % idx)
    path.write_text(src.replace(old, new, 1))
    lib = tmp_path / ("mut64_%d.so" % idx)
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-w", "-o", str(lib), str(path), "-lm"],
                   check=True)
    f = getattr(ctypes.CDLL(str(lib)), "oracle_sortmedian_" + tag)
    f.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    f.restype = ctypes.c_int
    rng = np.random.default_rng(23)
    caught = False
    for _ in range(200):
        n = int(rng.integers(5, 120))
        k = int(rng.integers(1, (n + 1) // 2)) * 2 + 1
        x = _i64_vector(rng, n) if tag == "i64" else _special_vector_f64(rng, n)
        a = np.empty(n - k + 1, dtype=np.int32)
        y = np.empty(n - k + 1, dtype=x.dtype)
        rc = f(x.ctypes.data, n, k, y.ctypes.data, a.ctypes.data)
        if rc != 0 or not np.array_equal(a, argsort_argmed(x, k)):
            caught = True
            break
    assert caught, "64-bit mutation %d survived" % idx


# --- the threaded range split used for full-size checks --------------------

@pytest.mark.parametrize("k", [1, 3, 31, 301])
def test_parallel_ranges_match(k):
    """Output ranges cut anywhere (also shorter than k, and more ranges than
    threads) give the same outputs as one pass, and both match the
    definition on sampled windows."""
    rng = np.random.default_rng(40 + k)
    n = 5 * k + 123
    x = rng.integers(0, 7, n).astype(np.int32)
    y, a = oracle.sortmedian(x, k)
    for ranges in (1, 2, 7, n - k + 1):
        y2, a2 = oracle.sortmedian_parallel(x, k, threads=3, ranges=ranges)
        assert np.array_equal(a2, a) and np.array_equal(y2, y)
    outs = rng.integers(0, n - k + 1, 200)
    assert np.array_equal(oracle.window_median(x, k, outs), a[outs])
