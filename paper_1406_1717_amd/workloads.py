"""Seeded synthetic inputs for the median filter.

This module only draws numbers: it holds none of the median filter's
arithmetic, and both the HIP path's tests/benchmark and the CPU oracle are
fed from it.  Every generator takes a seed and uses numpy's PCG64.

Workloads (names are what the data is, with its sizes):

  uniform_f32_1m          float32 U[0,1), n = 1,000,000, k = 101
  int32_full_64m          int32 uniform over the full range, n = 2**26, k = 1001
  int32_bytes_64m         int32 uniform over 0..255 (duplicates-heavy), n = 2**26
  random_walk_f32_16m     float32 cumulative sum of N(0,1) steps, n = 2**24
  sorted_walk_f32_16m     the same walk sorted ascending
  ragged_impulse_10k      10,000 float32 signals, lengths log-uniform in
                          [1e3, 1e6], odd windows log-uniform in [3, 4001],
                          N(0,1) values with 5% impulses uniform in (-50, 50)
  distinct_normal_256     256 rows x 262,144 float32 N(0,1), distinct per row,
                          k = 201, with an N(0,1) upstream gradient
  int64_full_64m          int64 uniform over the full range, n = 2**26, k = 1001
  random_walk_f64_16m     float64 cumulative sum of N(0,1) steps, n = 2**24

The seven generator families of the paper's experiments (Section 7.3:
ascending, descending, both with small uniform noise, large and small
uniform integers, piecewise constant with noise) are in `paper_family`.
"""
import numpy as np

SEEDS = {
    "uniform_f32_1m": 101,
    "int32_full_64m": 201,
    "int32_bytes_64m": 202,
    "random_walk_f32_16m": 301,
    "ragged_impulse_10k": 401,
    "distinct_normal_256": 501,
    "distinct_normal_256_grad": 502,
    "fd_slice": 503,
    "int64_full_64m": 601,
    "random_walk_f64_16m": 602,
}


def rng_for(seed):
    return np.random.Generator(np.random.PCG64(seed))


def uniform_f32(n, seed):
    return rng_for(seed).random(n, dtype=np.float32)


def int32_full(n, seed):
    return rng_for(seed).integers(-2**31, 2**31, n, dtype=np.int32)


def int32_bytes(n, seed):
    return rng_for(seed).integers(0, 256, n, dtype=np.int32)


def random_walk_f32(n, seed):
    steps = rng_for(seed).standard_normal(n)
    return np.cumsum(steps).astype(np.float32)


def sorted_walk_f32(n, seed):
    return np.sort(random_walk_f32(n, seed))


def ragged_impulse(num_signals, seed, min_len=1000, max_len=1_000_000,
                   min_k=3, max_k=4001, impulse_rate=0.05, impulse_amp=50.0):
    """Packed ragged batch: returns (x, offsets[int64, S+1], ks[int32, S]).

    Draw order: all lengths, then all windows, then each signal's values in
    turn.  Lengths are exp(U(ln min_len, ln max_len)) truncated to int;
    windows are 2*round((exp(U(ln min_k, ln max_k)) - 1)/2) + 1, clamped to
    the largest odd value not above the signal length."""
    rng = rng_for(seed)
    lens = np.exp(rng.uniform(np.log(min_len), np.log(max_len), num_signals)).astype(np.int64)
    lens = np.maximum(lens, 1)
    kf = np.exp(rng.uniform(np.log(min_k), np.log(max_k), num_signals))
    ks = (2 * np.round((kf - 1.0) / 2.0) + 1).astype(np.int64)
    largest_odd = lens - (1 - (lens & 1))
    ks = np.minimum(ks, largest_odd).astype(np.int32)
    offsets = np.zeros(num_signals + 1, dtype=np.int64)
    np.cumsum(lens, out=offsets[1:])
    x = np.empty(int(offsets[-1]), dtype=np.float32)
    for s in range(num_signals):
        L = int(lens[s])
        v = rng.standard_normal(L, dtype=np.float32)
        hit = rng.random(L) < impulse_rate
        v[hit] = rng.uniform(-impulse_amp, impulse_amp, int(hit.sum())).astype(np.float32)
        x[offsets[s]:offsets[s + 1]] = v
    return x, offsets, ks


def distinct_rows(rows, n, seed, min_gap=0.0, window=None):
    """rows x n float32 N(0,1), every row free of duplicates.

    With min_gap > 0 and a window w, any two entries closer than w positions
    also differ by at least min_gap; violators are redrawn from the same
    generator until none is left."""
    rng = rng_for(seed)
    x = rng.standard_normal((rows, n), dtype=np.float32)
    for r in range(rows):
        row = x[r]
        for _ in range(1000):
            bad = _violators(row, min_gap, window)
            if bad.size == 0:
                break
            row[bad] = rng.standard_normal(bad.size, dtype=np.float32)
        else:
            raise RuntimeError("could not make row %d distinct" % r)
    return x


def _violators(row, min_gap, window):
    """Indices to redraw: duplicates anywhere in the row, and (with a gap
    rule) the later member of any close pair within `window` positions."""
    order = np.argsort(row, kind="stable")
    srt = row[order]
    dup = np.zeros(row.size, dtype=bool)
    eq = srt[1:] == srt[:-1]
    dup[order[1:][eq]] = True
    if min_gap > 0 and window:
        for d in range(1, int(window)):
            close = np.abs(row[d:].astype(np.float64) - row[:-d].astype(np.float64)) < min_gap
            dup[d:][close] = True
    return np.nonzero(dup)[0]


def int64_full(n, seed):
    info = np.iinfo(np.int64)
    return rng_for(seed).integers(info.min, info.max, n, dtype=np.int64, endpoint=True)


def random_walk_f64(n, seed):
    return np.cumsum(rng_for(seed).standard_normal(n))


def int64_words(n, seed):
    """int64 values whose order is decided by the high 32-bit word for some
    pairs and by the low word for others, with many equal values and both
    extremes."""
    rng = rng_for(seed)
    hi = rng.choice(np.array([-3, -1, 0, 1, 5, 2**30], dtype=np.int64), n)
    lo = rng.choice(np.array([0, 1, 7, 2**31 - 1, 2**31, 2**32 - 1], dtype=np.int64), n)
    x = hi * (1 << 32) + lo
    x[rng.random(n) < 0.02] = np.iinfo(np.int64).max
    x[rng.random(n) < 0.02] = np.iinfo(np.int64).min
    return x


def f64_specials(n, seed):
    """float64 N(0,1) with 40% of the items replaced by specials: signed
    zeros, infinities, NaNs (one with a payload), subnormals and values that
    are equal in float32 but not in float64."""
    rng = rng_for(seed)
    pool = np.array([0.0, -0.0, 1.0, 1.0 + 2.0 ** -40, 1.0 - 2.0 ** -50, -1.0, 5e-324, -5e-324,
                     np.inf, -np.inf, np.nan, 3.0, 1e300, -1e300], dtype=np.float64)
    x = rng.standard_normal(n)
    m = rng.random(n) < 0.4
    x[m] = rng.choice(pool, int(m.sum()))
    if n > 0:
        x[rng.integers(0, n)] = np.frombuffer(np.uint64(0xFFF8000000000001).tobytes(), np.float64)[0]
    return x


def normal_f32(shape, seed):
    return rng_for(seed).standard_normal(shape, dtype=np.float32)


def paper_family(name, n, seed, bits=32):
    """The paper's generator families (Section 7.3), as int32/int64 arrays."""
    rng = rng_for(seed)
    dt = np.int32 if bits == 32 else np.int64
    i = np.arange(n, dtype=np.int64)
    if name == "asc":
        v = i
    elif name == "desc":
        v = n - i
    elif name == "r-asc":
        v = i + rng.integers(0, 10**4, n)
    elif name == "r-desc":
        v = n - i + rng.integers(0, 10**4, n)
    elif name == "r-large":
        info = np.iinfo(dt)
        return rng.integers(info.min, info.max, n, dtype=dt, endpoint=True)
    elif name == "r-small":
        v = rng.integers(0, 10**4, n)
    elif name == "r-block":
        # piecewise constant levels with small noise; level length random
        levels = []
        total = 0
        while total < n:
            L = int(rng.integers(1, max(2, n // 8) + 1))
            levels.append(np.full(L, rng.integers(0, 10**6)))
            total += L
        v = np.concatenate(levels)[:n] + rng.integers(0, 10**4, n)
    else:
        raise ValueError(name)
    if bits == 32:
        v = np.clip(v, np.iinfo(np.int32).min, np.iinfo(np.int32).max)
    return v.astype(dt)


# Named full-size workloads -------------------------------------------------

def workload(name):
    """Return a dict describing one named workload (arrays on the host)."""
    if name == "uniform_f32_1m":
        return {"x": uniform_f32(10**6, SEEDS[name]), "k": 101}
    if name == "int32_full_64m":
        return {"x": int32_full(2**26, SEEDS[name]), "k": 1001}
    if name == "int32_bytes_64m":
        return {"x": int32_bytes(2**26, SEEDS[name]), "k": 1001}
    if name == "random_walk_f32_16m":
        return {"x": random_walk_f32(2**24, SEEDS[name]), "ks": [3, 31, 301, 3001, 30001]}
    if name == "int64_full_64m":
        return {"x": int64_full(2**26, SEEDS[name]), "k": 1001}
    if name == "random_walk_f64_16m":
        return {"x": random_walk_f64(2**24, SEEDS[name]), "ks": [3, 31, 301, 3001, 30001]}
    if name == "distinct_normal_256":
        rows, n, k = 256, 262_144, 201
        return {"x": distinct_rows(rows, n, SEEDS[name]), "k": k,
                "grad": normal_f32((rows, n - k + 1), SEEDS["distinct_normal_256_grad"])}
    if name == "sorted_walk_f32_16m":
        return {"x": sorted_walk_f32(2**24, SEEDS["random_walk_f32_16m"]),
                "ks": [3, 31, 301, 3001, 30001]}
    raise KeyError(name)
