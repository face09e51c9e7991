"""Host check of the tile logic: the phase functions the GPU kernels run
(shared header, compiled for the host by tests/emu/tile_emu.cpp) executed
phase by phase for every thread share, against the CPU oracle.  Covers
both sort paths (bucket sort, and the merge sort it falls back to), one-
and many-chunk walks, partial last blocks and the float specials.  This is
test infrastructure: the library never loads it."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "emu", "tile_emu.cpp")
INC = os.path.join(os.path.dirname(HERE), "paper_1406_1717_amd", "csrc")


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    so = str(tmp_path_factory.mktemp("emu") / "tile_emu.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", "-I", INC, "-o", so, SRC], check=True)
    lib = ctypes.CDLL(so)
    lib.emu_median_filter.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                      ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    lib.emu_fast_tiles.restype = ctypes.c_long
    lib.emu_slow_tiles.restype = ctypes.c_long
    return lib


def threads_for(k):
    S = 1 << int(np.ceil(np.log2(k))) if k > 1 else 1
    return 512 if 2 * S <= 4096 else 1024


def inputs(rng, kind, n):
    if kind == 0:
        return rng.random(n).astype(np.float32)
    if kind == 1:
        return rng.integers(0, 4, n).astype(np.int32)
    if kind == 2:
        return np.sort(rng.random(n)).astype(np.float32)
    if kind == 3:
        return np.cumsum(rng.standard_normal(n)).astype(np.float32)
    if kind == 4:
        return rng.integers(-2**31, 2**31, n, dtype=np.int32)
    pool = np.array([0.0, -0.0, 1.0, np.inf, -np.inf, np.nan, 2.0], np.float32)
    x = rng.standard_normal(n).astype(np.float32)
    m = rng.random(n) < 0.3
    x[m] = rng.choice(pool, int(m.sum()))
    return x


@pytest.mark.parametrize("force_merge,wide", [(0, False), (1, False), (0, True)])
def test_tile_phases_match_oracle(emu, force_merge, wide):
    """wide: every tile with 1024 threads (the one-launch batch configuration
    also runs small windows as 1024-thread tiles)."""
    emu.emu_set_force_merge(force_merge)
    fast0, slow0 = emu.emu_fast_tiles(), emu.emu_slow_tiles()
    rng = np.random.default_rng(7 + force_merge)
    ks = [3, 5, 15, 17, 31, 63, 65, 101, 255, 301, 513, 1001, 2047, 4001]
    for trial in range(60):
        k = ks[trial % len(ks)]
        n = int(rng.integers(k, k * int(rng.integers(1, 8)) + 300))
        x = inputs(rng, trial % 6, n)
        y = np.empty(n - k + 1, x.dtype)
        a = np.empty(n - k + 1, np.int32)
        pm = ctypes.c_int32()
        threads = 1024 if wide else threads_for(k)
        rc = emu.emu_median_filter(x.ctypes.data, n, k, int(x.dtype == np.float32), threads,
                                   y.ctypes.data, a.ctypes.data, ctypes.byref(pm))
        yo, ao = oracle.sortmedian(x, k)
        assert rc == 0, (k, n, trial, rc)
        assert np.array_equal(a, ao), (k, n, trial)
        assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), (k, n, trial)
    fast, slow = emu.emu_fast_tiles() - fast0, emu.emu_slow_tiles() - slow0
    if force_merge:
        assert fast == 0 and slow > 0
    else:
        assert fast > 0 and slow > 0      # duplicates-heavy tiles fall back
    emu.emu_set_force_merge(0)


def test_global_tail_matches_oracle(emu):
    """The tail of the one-pair tiles for k > 4095 (coarse count table,
    walk with position words in flight, output), run on the host after a
    plain sort of each pair, for windows either side of the powers of two
    and random, random-walk, tie-heavy and descending inputs, with the LDS
    budgets of both kernel variants (64 KB up to k = 16383, 128 KB above)."""
    emu.emu_global_tail.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.c_int32,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    rng = np.random.default_rng(53)
    for k in (4097, 5001, 8191, 8193, 16383, 16385, 30001, 32767):
        lds = 65536 if k <= 16383 else 131072
        for kind in range(4):
            n = 3 * k + int(rng.integers(0, k))
            if kind == 0:
                x = rng.random(n).astype(np.float32)
            elif kind == 1:
                x = np.cumsum(rng.standard_normal(n)).astype(np.float32)
            elif kind == 2:
                x = rng.integers(0, 5, n).astype(np.float32)
            else:
                x = np.arange(n, dtype=np.float32)[::-1].copy()
            y = np.empty(n - k + 1, np.float32)
            a = np.empty(n - k + 1, np.int32)
            L = ctypes.c_int32()
            rc = emu.emu_global_tail(x.ctypes.data, n, k, 1, lds, y.ctypes.data, a.ctypes.data, ctypes.byref(L))
            yo, ao = oracle.sortmedian(x, k)
            assert rc == 0, (k, kind, rc)
            assert L.value >= 31 and L.value % 2 == 1
            assert np.array_equal(a, ao), (k, kind)
            assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), (k, kind)


def test_walk_window_slides(emu):
    """Inputs whose median drifts through the merged order step after step
    (ascending, descending, random walks, a sawtooth): the walk's register
    window slides up and down by half its width or falls back to a search
    of M, and every output still matches the oracle."""
    rng = np.random.default_rng(41)
    for k in (15, 31, 33, 101, 301, 1001, 2047, 3001):
        n = 6 * k + int(rng.integers(0, k))
        ramp = np.arange(n, dtype=np.float32)
        saw = (np.arange(n) % (2 * k + 7)).astype(np.float32)
        walk = np.cumsum(rng.standard_normal(n) + 0.3).astype(np.float32)
        for x in (ramp, ramp[::-1].copy(), saw, walk, -walk):
            y = np.empty(n - k + 1, x.dtype)
            a = np.empty(n - k + 1, np.int32)
            pm = ctypes.c_int32()
            rc = emu.emu_median_filter(x.ctypes.data, n, k, 1, threads_for(k), y.ctypes.data, a.ctypes.data,
                                       ctypes.byref(pm))
            yo, ao = oracle.sortmedian(x, k)
            assert rc == 0, (k, n, rc)
            assert np.array_equal(a, ao), (k, n)
            assert np.array_equal(y.view(np.uint32), yo.view(np.uint32)), (k, n)


def test_presorted_tiles(emu):
    """Ascending inputs (with ties) skip the bucket sort; a single descent
    anywhere in a tile must send that tile through the sort."""
    emu.emu_presorted_tiles.restype = ctypes.c_long
    before = emu.emu_presorted_tiles()
    rng = np.random.default_rng(31)
    for trial in range(48):
        k = [5, 33, 101, 513, 1001, 3001][trial % 6]
        n = int(rng.integers(k, 6 * k + 200))
        kind = (trial // 6) % 4
        if kind == 0:
            x = np.sort(rng.random(n)).astype(np.float32)
        elif kind == 1:
            x = np.sort(rng.integers(0, 50, n)).astype(np.int32)
        elif kind == 2:
            x = np.sort(rng.random(n)).astype(np.float32)
            x[rng.integers(0, n)] = -1.0
        else:
            x = (np.arange(n, dtype=np.int32) // 3)
        y = np.empty(n - k + 1, x.dtype)
        a = np.empty(n - k + 1, np.int32)
        pm = ctypes.c_int32()
        rc = emu.emu_median_filter(x.ctypes.data, n, k, int(x.dtype == np.float32), threads_for(k),
                                   y.ctypes.data, a.ctypes.data, ctypes.byref(pm))
        yo, ao = oracle.sortmedian(x, k)
        assert rc == 0 and np.array_equal(a, ao), (k, n, kind, rc)
        assert np.array_equal(y.view(np.uint32), yo.view(np.uint32))
    assert emu.emu_presorted_tiles() > before


def _emu64(emu, x, k, threads):
    emu.emu_median_filter64.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    n = len(x)
    y = np.empty(n - k + 1, dtype=x.dtype)
    am = np.full(n - k + 1, -1, dtype=np.int32)
    rc = emu.emu_median_filter64(x.ctypes.data, n, k, int(x.dtype == np.float64), threads,
                                 y.ctypes.data, am.ctypes.data)
    return rc, y, am


@pytest.mark.parametrize("force_merge", [0, 1])
@pytest.mark.parametrize("kind", ["f64_specials", "int64_words", "int64_full", "walk_f64"])
def test_tile_phases_64bit_match_oracle(emu, kind, force_merge):
    """64-bit signals: the rank pre-pass (bucket sort, or the merge sort it
    falls back to) then the 32-bit tiles on the ranks (each tile reading its
    own span), against the 64-bit oracle."""
    from paper_1406_1717_amd import workloads as W
    gen = {"f64_specials": W.f64_specials, "int64_words": W.int64_words,
           "int64_full": W.int64_full, "walk_f64": W.random_walk_f64}[kind]
    emu.emu_rank_bucket_tiles.restype = ctypes.c_long
    emu.emu_rank_merge_tiles.restype = ctypes.c_long
    emu.emu_set_force_merge(force_merge)
    b0, m0 = emu.emu_rank_bucket_tiles(), emu.emu_rank_merge_tiles()
    try:
        for i, k in enumerate((3, 5, 31, 33, 101, 701, 1001, 2047, 2049, 4095)):
            n = {3: 3001, 5: 999, 31: 4000, 33: 5003, 101: 9000}.get(k, 3 * k + 17 + i)
            x = gen(n, 700 + i)
            rc, y, am = _emu64(emu, x, k, threads_for(k))
            assert rc == 0, (kind, k, rc)
            _, want = oracle.sortmedian(x, k)
            assert np.array_equal(am, want), (kind, k)
            assert np.array_equal(y.view(np.uint64), x[want].view(np.uint64))
    finally:
        emu.emu_set_force_merge(0)
    b, m = emu.emu_rank_bucket_tiles() - b0, emu.emu_rank_merge_tiles() - m0
    emu.emu_ranked_tiles.restype = ctypes.c_long
    if not force_merge:
        assert emu.emu_ranked_tiles() > 0     # tile-order tiles placed straight from the ranks
    if force_merge:
        assert b == 0 and m > 0
    elif kind in ("int64_full", "walk_f64"):
        assert b > 0          # spread keys take the bucket sort
    elif kind == "int64_words":
        assert m > 0          # few distinct values crowd the buckets


def test_tile_phases_64bit_presorted_and_single_block(emu):
    from paper_1406_1717_amd import workloads as W
    for k, n in ((101, 101), (101, 150), (1001, 5000), (3001, 3001)):
        for x in (np.sort(W.random_walk_f64(n, 3)), np.arange(n, 0, -1, dtype=np.int64) << 33):
            rc, y, am = _emu64(emu, x, k, threads_for(k))
            assert rc == 0, (k, n, rc)
            _, want = oracle.sortmedian(x, k)
            assert np.array_equal(am, want), (k, n)


@pytest.mark.parametrize("k,threads", [(3, 512), (31, 512), (1001, 512), (2047, 512), (4095, 1024)])
def test_last_tiles_of_longest_signal(emu, k, threads):
    """The index arithmetic of the last tiles of an n = 2^31 - 1 signal (the
    largest argmed index): only the signal's tail is allocated, and the
    outputs the last three tiles write are checked against the definition."""
    emu.emu_tile_range.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                   ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p]
    emu.emu_ntiles.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.c_int]
    emu.emu_ntiles.restype = ctypes.c_int64
    n = 2**31 - 1
    nt = emu.emu_ntiles(n, k, threads)
    base = n - 3 * 8192 * 4          # before the first item of the last three tiles
    xs = np.random.default_rng(k).random(n - base).astype(np.float32)
    y = np.full(n - base, np.nan, np.float32)
    am = np.full(n - base, -1, np.int32)
    rc = emu.emu_tile_range(xs.ctypes.data, base, n, k, threads, nt - 3, nt, y.ctypes.data, am.ctypes.data)
    assert rc == 0
    nout = n - k + 1
    written = np.nonzero(am >= 0)[0]
    assert written.max() + base == nout - 1
    outs = np.arange(base + written.min(), nout, dtype=np.int64)
    assert np.all(am[outs - base] >= 0)
    sel = outs[:: max(1, len(outs) // 300)]
    want = oracle.window_median(xs, k, sel - base) + base
    assert np.array_equal(am[sel - base], want)
    assert np.array_equal(y[sel - base].view(np.uint32), xs[want - base].view(np.uint32))


@pytest.mark.parametrize("kind", ["f64_specials", "int64_words", "int64_full", "walk_f64"])
def test_pair_ranks_64bit(emu, kind):
    """The pair pre-pass of 64-bit signals on the global path (k > 4095):
    chunks ranked as in LDS, sorted runs merged by merge-path segments; every
    pair's ranks must equal its items' positions in (value, index) order
    (numpy: dense value ranks under the float convention, then lexsort)."""
    from paper_1406_1717_amd import workloads as W
    from tests.brute import value_rank
    gen = {"f64_specials": W.f64_specials, "int64_words": W.int64_words,
           "int64_full": W.int64_full, "walk_f64": W.random_walk_f64}[kind]
    emu.emu_rank_pairs64.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
    for i, k in enumerate((4097, 5001, 8193, 16385, 32767)):
        n = 3 * k + 1234 + i
        x = gen(n, 800 + i)
        stride, tiles = ctypes.c_int64(), ctypes.c_int64()
        assert emu.emu_rank_pairs64(x.ctypes.data, n, k, int(x.dtype == np.float64), None,
                                    ctypes.byref(stride), ctypes.byref(tiles)) == 0
        keys = np.full(tiles.value * stride.value, 0xFFFFFFFF, dtype=np.uint32)
        assert emu.emu_rank_pairs64(x.ctypes.data, n, k, int(x.dtype == np.float64), keys.ctypes.data,
                                    ctypes.byref(stride), ctypes.byref(tiles)) == 0
        for t in range(tiles.value):
            e0 = t * k
            span = min(n - e0, 2 * k)
            seg = x[e0:e0 + span]
            order = np.lexsort((np.arange(span), value_rank(seg)))
            want = np.empty(span, dtype=np.uint32)
            want[order] = np.arange(span, dtype=np.uint32)
            got = keys[t * stride.value: t * stride.value + span]
            assert np.array_equal(got, want), (kind, k, t)


@pytest.mark.parametrize("kind", [0, 1, 2, 3])
def test_key_transforms_order(emu, kind):
    """Sorting by the kernels' unsigned keys (with the index as tie-break)
    gives numpy's stable order under the value convention: -0.0 equal to
    +0.0, every NaN above +inf and equal to the others, signed integers."""
    from tests.brute import value_rank
    rng = np.random.default_rng(50 + kind)
    n = 20_000
    if kind == 0:
        pool = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-45, -1e-45, 3.4e38, -3.4e38, 1.0, -1.0], np.float32)
        x = rng.standard_normal(n).astype(np.float32)
        m = rng.random(n) < 0.3
        x[m] = rng.choice(pool, int(m.sum()))
        x[:3] = np.frombuffer(np.array([0xFFC00001, 0x7F800001, 0xFFFFFFFF], np.uint32).tobytes(), np.float32)
    elif kind == 1:
        x = rng.integers(-2**31, 2**31, n, dtype=np.int32)
        x[:4] = [np.iinfo(np.int32).min, np.iinfo(np.int32).max, 0, -1]
        x[rng.random(n) < 0.2] = 7
    elif kind == 2:
        from paper_1406_1717_amd import workloads as W
        x = W.f64_specials(n, 51)
        x[:3] = np.frombuffer(np.array([0xFFF8000000000001, 0x7FF0000000000001, 0xFFFFFFFFFFFFFFFF],
                                       np.uint64).tobytes(), np.float64)
    else:
        from paper_1406_1717_amd import workloads as W
        x = W.int64_words(n, 52)
    wide = kind >= 2
    out32 = np.zeros(n, np.uint32)
    out64 = np.zeros(n, np.uint64)
    emu.emu_keys.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    emu.emu_keys(x.ctypes.data, n, kind, out32.ctypes.data, out64.ctypes.data)
    keys = out64 if wide else out32
    got = np.lexsort((np.arange(n), keys))
    want = np.lexsort((np.arange(n), value_rank(x)))
    assert np.array_equal(got, want)
    # equal values (and only those) share a key
    vr = value_rank(x)
    assert np.array_equal(keys[got][1:] == keys[got][:-1], vr[got][1:] == vr[got][:-1])


def test_reciprocal_division(emu):
    """The kernels' division of indexes below 2^16 by a launch constant (a
    24-bit high multiply by a scaled reciprocal) is exact."""
    emu.emu_check_udiv16.restype = ctypes.c_long
    assert emu.emu_check_udiv16() == 0
