// HIP kernels of the sorting-based median filter (arXiv:1406.1717) for
// gfx950.  The per-tile phases live in mf_tile.h; this file runs them:
//
//   k_tile_lds<NT>   k <= 4095: one workgroup per tile, every tile buffer
//                    in LDS (NT = 512 threads for blocks up to 2048 slots,
//                    1024 above); a ranked int32 form runs on the rank keys
//                    of 64-bit signals and copies 64-bit medians.
//   k_tile_lds_persistent  the same tiles for ragged batches: a resident
//                    grid taking units from a work counter.
//   k_tile_global    4096 < k <= 32767: one pair per tile, bucket-sorted
//                    through a per-workgroup global workspace (sort values,
//                    merged order, position maps, staged medians), with a
//                    coarse count table and a copy of the merged order in
//                    LDS; workgroups loop over tiles.
//   k_rank64         64-bit signals: each tile's items ranked by (key,
//                    index) into 32-bit keys.
//   k_identity, k_identity64   k = 1.
//   k_backward_exact, k_backward   the gradient of the forward: the
//                    upstream gradient summed at the argmedians,
//                    deterministically (float32 gradients with k <= 1025
//                    by exact accumulation in LDS, the others in
//                    increasing output order).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <vector>

#include "mf_tile.h"
#include "mf_launch.h"

namespace mf {

// ------------------------------------------------------------------ helpers

// Phase probe: kernels instantiated with STOP = n (only in the phase-probe
// build, MF_PHASE_PROBE) return after the n-th phase boundary of a tile, so
// that timing and counting each stopping point gives the cost of every
// phase.  The library's kernels have STOP = 0 and contain no such return.
// Stops 1-17 are the LDS tiles'; 21-30 the one-pair tiles' in global memory
// (k_tile_global: 21-25 in the pair's bucket sort, 26-30 in its tail), whose
// workgroups go on to their next tile.
#define MF_STOP_AT(n) \
    if constexpr (STOP == (n)) return;
#define MF_STOP_AT_V(n, v) \
    if constexpr (STOP == (n)) return (v);

__device__ __forceinline__ void store_regs(u64 *dst, const u64 (&v)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j += 2) {
        ulonglong2 pr;
        pr.x = v[j];
        pr.y = v[j + 1];
        *(ulonglong2 *)(dst + j) = pr;
    }
}

// Exclusive prefix of `tot` within segments of G consecutive threads (G a
// power of two); wave_tot holds NT/64 wave totals when G > 64.
template <int NT>
__device__ __forceinline__ u32 seg_excl_scan(u32 tot, int G, u32 *wave_tot)
{
    const int lane = threadIdx.x & 63;
    u32 incl;
    if (G >= 64) {
        incl = __ockl_wfscan_add_u32(tot, false) + tot;
    } else {
        incl = tot;
        for (int d = 1; d < G; d <<= 1) {
            const u32 o = (u32)__shfl_up((int)incl, (unsigned)d, G);
            if ((lane & (G - 1)) >= d) incl += o;
        }
    }
    if (G <= 64) return incl - tot;
    const int wave = threadIdx.x >> 6;
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    const int w0 = wave & ~((G >> 6) - 1);
    u32 add = 0u;
    for (int w = w0; w < wave; w++) add += wave_tot[w];
    return incl - tot + add;
}

// Exclusive prefix of a 64-bit value over the workgroup (NT threads);
// wave_tot holds NT/64 wave totals.
template <int NT>
__device__ __forceinline__ u64 excl_scan64(u64 c, u64 *wave_tot)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const u64 incl = (u64)__ockl_wfscan_add_u64((unsigned long)c, false) + c;
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    u64 add = 0ull;
    for (int w = 0; w < wave; w++) add += wave_tot[w];
    return incl - c + add;
}

// Resolves work unit uidx of a launch into its signal and tile.
struct Resolved {
    const u32 *x;
    u32 *y;
    int32_t *argmed;
    int64_t n;
    int32_t k;
    int64_t tile;
};

// Units of a launch without a work list (one signal, or rows), in an order
// that gives each XCD a contiguous run of tiles: workgroups are dispatched
// round the 8 XCDs by index, and neighbouring tiles share their boundary
// block, which then stays in one L2 (each input is fetched from HBM about
// once, and the output gathers hit L2).  A bijection of [0, nunits); a work
// list keeps its own order.
__device__ __forceinline__ int64_t xcd_unit(const Launch &L, int64_t b)
{
    if (L.units) return b;
    const int64_t q = L.nunits >> 3, r = L.nunits & 7, x = b & 7, j = b >> 3;
    return x * q + (x < r ? x : r) + j;
}

__device__ __forceinline__ Resolved unit_of(const Launch &L, int64_t uidx)
{
    SigDesc d;
    int64_t tile;
    if (L.units) {
        const Unit u = L.units[uidx];
        d = L.sigs[u.sig];
        tile = u.tile;
    } else {
        const int64_t row = uidx / L.tpr;
        tile = uidx - row * L.tpr;
        d = L.one;
        d.x_off += row * (L.xrow ? L.xrow : d.n) + tile * L.xshift;
        d.y_off += row * (d.n - d.k + 1);
    }
    Resolved r;
    r.x = (const u32 *)L.x + d.x_off;
    r.y = (u32 *)L.y + d.y_off;
    r.argmed = L.argmed ? L.argmed + d.y_off : nullptr;
    r.n = d.n;
    r.k = d.k;
    r.tile = tile;
    return r;
}

// Phases 3-6 of a tile (pair merge, tables, walk, output); phases 1-2 have
// filled m.srt.  NT threads, barriers between phases.  The medians are
// copied from xo to yo (V: 32- or 64-bit elements).
template <int NT, typename V, int STOP = 0, int GAHEAD = 8>
__device__ __forceinline__ void tile_tail(const Shape &s, const Tile &T, const TileMem &m, const Resolved &d,
                                          const V *xo, V *yo, int *err, bool merged, u32 *rowbuf = nullptr,
                                          u32 *info = nullptr)
{
    const int tid = threadIdx.x;
    if (!merged) {
        tail_pair_pad(s, T, m, tid, NT);
        __syncthreads();
        MF_STOP_AT(15)
        tail_pair_merge(s, T, m, tid, NT, xo, yo, d.argmed);
        __syncthreads();
        MF_STOP_AT(16)
        // the median before each pair's first step is A's median: remember
        // its merged position (before the count tables reuse the sort buffer)
        tail_first_medians(s, T, m, tid, NT);
        __syncthreads();
        MF_STOP_AT(17)
    }
    if (rowbuf) {
        // one-pair tiles in global memory (k > 4095): the coarse count
        // table in LDS (rowbuf) gives each walk chunk its starting column;
        // then the walk and the output read the merged order from a copy
        // in LDS
        if (T.P == 0) return;
        u32 *tb = rowbuf, *gt = rowbuf + s.C * gcols(s);
        gtab_zero(s, tb, tid, NT);
        __syncthreads();
        gtab_hist(s, T, m, tb, tid, NT);
        __syncthreads();
        MF_STOP_AT(26)
        gtab_col_sums(s, tb, gt, tid, NT);
        __syncthreads();
        gtab_col_apply(s, tb, gt, tid, NT);
        __syncthreads();
        MF_STOP_AT(27)
        gtab_rows(s, tb, info, tid, NT);
        __syncthreads();
        MF_STOP_AT(28)
        TileMem ml = m;
        ml.M = (u16 *)rowbuf;
        const MF_GLOBAL uint4 *src = gmem((const uint4 *)m.M);
        uint4 *dst = (uint4 *)rowbuf;
        for (int e = tid; e < s.Mstride / 8; e += NT) dst[e] = src[e];
        __syncthreads();
        MF_STOP_AT(29)
        if (gtail_walk<GAHEAD>(s, T, ml, info, tid, NT, xo, yo, d.argmed)) atomicOr(err, 1);
        __syncthreads();
        MF_STOP_AT(30)
        gtail_output(s, T, ml, tid, NT, xo, yo, d.argmed);
        return;
    }
    if (s.C > 1) {
        if (!merged) {   // tile order counts its items with the pair orders
            tail_table_zero(s, T, m, tid, NT);
            __syncthreads();
            tail_table_hist(s, T, m, tid, NT);
            __syncthreads();
        }
        tail_table_columns(s, T, m, tid, NT);
        __syncthreads();
        MF_STOP_AT(10)
        MF_STOP_AT(11)
        tail_table_rows(s, T, m, tid, NT);
        __syncthreads();
        MF_STOP_AT(12)
    }
    if (tail_walk(s, T, m, tid, NT)) atomicOr(err, 1);
    __syncthreads();
    MF_STOP_AT(13)
    tail_output(s, T, m, tid, NT, xo, yo, d.argmed);
}

// ------------------------------------------------------------------ 64-bit ranks

__device__ __forceinline__ u64 wave_min_u64(u64 v)
{
    for (int d = 32; d > 0; d >>= 1) {
        const u64 o = (u64)__shfl_xor((unsigned long long)v, d);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ u64 wave_max_u64(u64 v)
{
    for (int d = 32; d > 0; d >>= 1) {
        const u64 o = (u64)__shfl_xor((unsigned long long)v, d);
        v = o > v ? o : v;
    }
    return v;
}

// The ranks of the span items at xt by (64-bit key, index), left in LDS
// as u32 per item offset (at lds); span <= NT * kRegs.  The sort is a
// bucket sort over cap buckets, or, for a tile with a crowded bucket, a
// merge sort (registers, then stable merge-path levels).  LDS: keys (8 B
// per position), slots (2 B), 16-bit bucket counters (2 B per bucket); the
// ranks reuse the keys.  Ends with a barrier.
template <int NT, bool F64>
__device__ __forceinline__ void rank_items(const u64 *xt, int32_t span, unsigned char *lds)
{
    __shared__ u64 red_lo[NT / 64], red_hi[NT / 64];
    __shared__ u32 wave_tot[NT / 64];
    __shared__ u32 full;
    static_assert(kRegs == 8, "slots are stored as one 16-byte word per thread");
    const int tid = threadIdx.x;
    const int32_t cap = NT * kRegs;
    u64 *K = (u64 *)lds;
    u16 *S = (u16 *)(lds + 8 * cap);
    u32 *C = (u32 *)(lds + 10 * cap);
    u64 kv[kRegs];
    u32 sv[kRegs];
    rank64_load<F64>(xt, span, tid, kv, sv);
#pragma unroll
    for (int w = 0; w < kRegs / 2; w++) C[tid * (kRegs / 2) + w] = 0u;
    if (tid == 0) full = 0u;
    u64 lo, hi;
    rank64_range(span, kv, sv, lo, hi);
    lo = wave_min_u64(lo);
    hi = wave_max_u64(hi);
    if ((tid & 63) == 0) {
        red_lo[tid >> 6] = lo;
        red_hi[tid >> 6] = hi;
    }
    __syncthreads();
    lo = red_lo[0];
    hi = red_hi[0];
    for (int w = 1; w < NT / 64; w++) {
        lo = red_lo[w] < lo ? red_lo[w] : lo;
        hi = red_hi[w] > hi ? red_hi[w] : hi;
    }
    const int32_t lognb = NT == 512 ? 12 : 13;
    static_assert(NT * kRegs == 512 * 8 || NT * kRegs == 1024 * 8, "cap is 4096 or 8192");
    const u32 sh = rank64_shift(lo, hi, lognb);
    u32 arr[kRegs];
    if (rank64_count(span, kv, sv, lo, sh, C, arr)) full = 1u;
    __syncthreads();
    if (full == 0u) {
        u32 c[kRegs];
        const u32 tot = rank64_scan_local(C, tid, c);
        const u32 excl = seg_excl_scan<NT>(tot, NT, wave_tot);
        rank64_scan_store(C, tid, excl, c);
        __syncthreads();
        rank64_scatter(span, kv, sv, lo, sh, C, arr, K, S);
        __syncthreads();
        u32 fin[kRegs];
        rank64_bucket_rank(span, kv, sv, lo, sh, C, (u32)cap, K, S, fin);
        __syncthreads();
        rank64_place(span, sv, fin, (u32 *)K);
    } else {
        sort_regs_ks(kv, sv);
        for (int w = kRegs; w < cap; w <<= 1) {
            store_regs(K + tid * kRegs, kv);
            uint4 sp;
            sp.x = sv[0] | (sv[1] << 16);
            sp.y = sv[2] | (sv[3] << 16);
            sp.z = sv[4] | (sv[5] << 16);
            sp.w = sv[6] | (sv[7] << 16);
            *(uint4 *)(S + tid * kRegs) = sp;
            __syncthreads();
            merge_level_ks(K, S, w, tid, kv, sv);
            __syncthreads();
        }
        rank64_ranks(span, tid, sv, (u32 *)K);
    }
    __syncthreads();
}

template <int NT, bool F64>
__device__ __forceinline__ void rank_tile(const Shape &s, const Tile &T, const u64 *x, unsigned char *lds)
{
    rank_items<NT, F64>(x + T.e0, tile_items(s, T), lds);
}

// Rank pre-pass of 64-bit signals for tiles ranked outside the tile kernel
// (the 1024-thread tiles): one workgroup per unit u = row * tiles + tile (rows
// of n items at x + row * n) writes its items' ranks to
// keys[u * stride + item offset].
template <int NT, bool F64>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 512 ? 6 : 4))) void k_rank64(const u64 *x, int64_t n, int32_t k, u32 *keys, int64_t stride, int64_t tiles)
{
    extern __shared__ __align__(16) unsigned char lds[];
    Shape s;
    make_shape(n, k, NT, &s);
    const int64_t row = blockIdx.x / tiles;
    const Tile T = make_tile(s, blockIdx.x - row * tiles);
    rank_tile<NT, F64>(s, T, x + row * n, lds);
    const int32_t span = tile_items(s, T);
    u32 *out = keys + (int64_t)blockIdx.x * stride;
    const u32 *rank = (const u32 *)lds;
    for (int32_t i = threadIdx.x; i < span; i += NT) out[i] = rank[i];
}

// ------------------------------------------------------------------ LDS path

// Shape and tile of a work unit for NT-thread tiles.
template <int NT>
__device__ __forceinline__ void unit_shape(const Resolved &d, Shape &s, Tile &T)
{
    make_shape(d.n, d.k, NT, &s);
    T = make_tile(s, d.tile);
}

// One tile of the LDS path, every buffer in the workgroup's LDS; raw holds
// the thread's inputs (load_raw).  RK: the inputs are rank keys of a 64-bit
// signal (each tile's items' distinct tile-order positions).  The medians
// are copied from xo to yo (V: u32, or u64 for a 64-bit signal).
template <int NT, bool F32, bool RK = false, typename V = u32, int STOP = 0>
__device__ __forceinline__ void lds_tile(const Resolved &d, const Shape &s, const Tile &T,
                                         const u32 (&raw)[kRegs], unsigned char *lds, int *err,
                                         const V *xo, V *yo)
{
    const int tid = threadIdx.x;
    Layout l;
    make_layout(s, &l);
    const TileMem m = tile_mem(lds, l);
    __shared__ u32 wave_tot[NT / 64];
    __shared__ u64 wave_tot64[NT / 64];

    // tiles of at most four blocks sort in tile order (pair orders by a
    // prefix count); others, and tile-order tiles whose buckets overflow
    // (heavy ties across the tile), sort block by block and merge each pair
    const Shape st = tile_order_shape(s);
    bool tord = tile_order_ok(s);
    // rank keys are distinct positions: a tile-order tile places each item
    // at its key without sorting
    const bool ranked = RK && tord;
    const int32_t per = tile_buckets(s) / NT;   // counters per thread

    // 1. load into registers
    u64 v[kRegs];
    if (tord) load_tile_values<F32>(s, T, m, raw, tid, v);
    else load_sort_values<F32>(s, T, m, raw, tid, v);

    // 2. bucket sort; tiles with an overfull bucket (or blocks under kRegs
    // slots) take the merge sort below.  Crowded buckets are counted again
    // with the map linear in the float bit pattern (the flag is the same for
    // every thread).
    // Presorted tiles (flag bit 2 clear after the key-range pass) skip the
    // bucket sort.
    bucket_zero_thread(m, tid, per);
    for (int b = tid; b < l.nbmax; b += NT) bucket_info_init(m, b);
    presort_note(s, m, tid, v);
    __syncthreads();
    MF_STOP_AT(1)
    bool fast = s.S >= kRegs;
    bool direct = false;   // items already in sort order
    int pass = 0;          // bucket map: 0 linear, 1 clamped logarithmic
    u32 arr[kRegs];   // arrival numbers (tile order: packed with the bucket)
    if (tord && !ranked) {
        tile_minmax(m, v);
        presort_check(s, T, m, tid, NT, v, true);
        __syncthreads();
        MF_STOP_AT(2)
        direct = (m.flag[0] & 4u) == 0u;
        if (!direct && tile_many_ties(m, tile_items(s, T))) {
            __syncthreads();
            tord = false;
            tile_to_block_values(s, T, tid, v);
            for (int b = tid; b < l.nbmax; b += NT) bucket_info_init(m, b);
            presort_note(s, m, tid, v);
            __syncthreads();
        }
    }
    if (tord && !direct && !ranked) {
        tile_count<F32>(st, m, v, arr, pass);
        __syncthreads();
        MF_STOP_AT(3)
        if ((m.flag[0] & 3u) != 0u) {
            __syncthreads();
            pass = 1;
            bucket_zero_thread(m, tid, per);
            if (tid == 0) m.flag[0] = 0u;
            __syncthreads();
            tile_count<F32>(st, m, v, arr, pass);
            __syncthreads();
        }
        if ((m.flag[0] & 1u) != 0u) {
            __syncthreads();
            tord = false;
            pass = 0;
            tile_to_block_values(s, T, tid, v);
            bucket_zero_thread(m, tid, per);
            for (int b = tid; b < l.nbmax; b += NT) bucket_info_init(m, b);
            presort_note(s, m, tid, v);
            __syncthreads();
        }
    }
    if (!tord && compact_tile(s)) fast = false;   // block order needs cap counters
    if (fast && !tord) {
        bucket_minmax(m, v);
        presort_check(s, T, m, tid, NT, v, false);
        __syncthreads();
        direct = (m.flag[0] & 4u) == 0u;
        if (!direct) {
            bucket_count<F32>(s, T, m, tid, v, arr, pass);
            __syncthreads();
            if ((m.flag[0] & 3u) != 0u) {
                __syncthreads();
                pass = 1;
                bucket_zero_thread(m, tid, per);
                if (tid == 0) m.flag[0] = 0u;
                __syncthreads();
                bucket_count<F32>(s, T, m, tid, v, arr, pass);
                __syncthreads();
            }
        }
    }
    fast = fast && (m.flag[0] & 1u) == 0u;
    bool merged = false;   // pair orders already written (tile order)
    if (fast) {
        const int32_t N = tile_items(s, T);
        if (direct) {
            presort_place(s, m, v, tord);
            __syncthreads();
        } else if (ranked) {
            u32 fin[kRegs];
#pragma unroll
            for (int j = 0; j < kRegs; j++) fin[j] = tv_key(v[j]) ^ 0x80000000u;
            tile_place(m, v, fin);
            __syncthreads();
        } else {
            u32 c[kRegs];
            const u32 tot = bucket_scan_local(m, tid, c, per);
            const u32 excl = seg_excl_scan<NT>(tot, tord ? NT : s.S / kRegs, wave_tot);
            bucket_scan_store(m, tid, excl, c, per);
            __syncthreads();
            MF_STOP_AT(4)
            if (tord) tile_scatter(m, v, arr, tid, N);
            else bucket_scatter<F32>(s, T, m, tid, v, arr, pass);
            __syncthreads();
            MF_STOP_AT(5)
            u32 fin[kRegs];
            if (tord) tile_rank(st, m, v, N, fin, arr);
            else bucket_rank<F32>(s, T, m, tid, v, fin, pass);
            __syncthreads();
            MF_STOP_AT(6)
            if (tord) tile_place(m, v, fin);
            else bucket_place(s, m, v, fin);
            __syncthreads();
            MF_STOP_AT(7)
        }
        if (tord) {
            // 3. pair orders from the per-block counts along the tile order
            u32 w[kRegs];
            const u64 cnt = tile_label_counts(s, m, tid, N, w);
            const u64 ex = excl_scan64<NT>(cnt, wave_tot64);
            if (s.C > 1) {   // the count tables reuse the sort buffer, read above
                tail_table_zero(s, T, m, tid, NT);
                __syncthreads();
            }
            MF_STOP_AT(8)
            tile_positions(s, T, m, ex, w, xo, yo, d.argmed);
            tile_mpad(s, T, m, tid, NT);
            __syncthreads();
            MF_STOP_AT(9)
            merged = true;
        }
    } else {
        // merge sort through the 64-bit buffer (free during the sort), then
        // the sorted blocks into the key and slot arrays
        if (tord) tile_to_block_values(s, T, tid, v);
        sort_regs(v);
        for (int w = kRegs; w < s.S; w <<= 1) {
            store_regs(m.mbuf + tid * kRegs, v);
            __syncthreads();
            merge_level(m.mbuf, w, tid, v);
            __syncthreads();
        }
#pragma unroll
        for (int j = 0; j < kRegs; j++)
            if (sv_valid(v[j])) put_block_value(s, m, tid * kRegs + j, v[j]);
        __syncthreads();
    }
    MF_STOP_AT(14)

    tile_tail<NT, V, STOP>(s, T, m, d, xo, yo, err, merged);
}

// One workgroup per work unit.  512-thread tiles of at most 53 KB run three
// workgroups per CU, which needs at most 80 VGPRs (six waves per SIMD).
// RK, the int32 forms for 64-bit signals: 1, the inputs are rank keys laid
// out by the rank pre-pass; 2 (int64) and 3 (float64), the tile ranks the
// 64-bit signal L.x64 in its own LDS first.  With RK, the medians are copied
// from L.x64 to the 64-bit y.
template <int NT, bool F32, int RK = 0, int STOP = 0>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(NT == 512 ? 6 : 8))) void k_tile_lds(Launch L, int *err)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const int64_t uidx = xcd_unit(L, blockIdx.x);
    const Resolved d = unit_of(L, uidx);
    Shape s;
    Tile T;
    unit_shape<NT>(d, s, T);
    u32 raw[kRegs];
    // a 64-bit signal's elements and medians: its row of the launch (rows
    // of n items, n-k+1 outputs), or its signal of a work list
    const u64 *x64 = (const u64 *)L.x64;
    u64 *y64 = (u64 *)L.y;
    if constexpr (RK != 0) {
        if (L.units) {
            const SigDesc sd = L.sigs[L.units[uidx].sig];
            x64 += sd.x_off;
            y64 += sd.y_off;
        } else {
            const int64_t row = uidx / L.tpr;
            x64 += row * d.n;
            y64 += row * (d.n - d.k + 1);
        }
    }
    if constexpr (RK >= 2) {
        rank_tile<NT, RK == 3>(s, T, x64, lds);
        rank_raw(s, T, (const u32 *)lds, threadIdx.x, raw);
        __syncthreads();   // the tile phases reuse the LDS
    } else {
        load_raw(s, T, d.x, threadIdx.x, raw);
    }
    if constexpr (RK != 0) {
        lds_tile<NT, F32, true>(d, s, T, raw, lds, err, x64, y64);
    } else {
        lds_tile<NT, F32, false, u32, STOP>(d, s, T, raw, lds, err, d.x, d.y);
    }
}

// Persistent form for ragged work lists: a grid sized to the resident
// workgroups takes units in work-list order from the counter *next (zero
// at launch) until the list is exhausted, fetching each next unit (and
// issuing its loads) before working on the current one; every workgroup
// leaves the loop on the same condition.
template <int NT, bool F32>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4))) void k_tile_lds_persistent(Launch L, u32 *next, int *err)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ u32 cur;
    if (threadIdx.x == 0) cur = atomicAdd(next, 1u);
    __syncthreads();
    u32 u = cur;
    if ((int64_t)u >= L.nunits) return;
    Resolved d = unit_of(L, u);
    u32 raw[kRegs];
    {
        Shape s;
        Tile T;
        unit_shape<NT>(d, s, T);
        load_raw(s, T, d.x, threadIdx.x, raw);
    }
    for (;;) {
        __syncthreads();   // every thread has read cur; the last tile is done with LDS
        if (threadIdx.x == 0) cur = atomicAdd(next, 1u);
        __syncthreads();
        const u32 un = cur;
        const bool more = (int64_t)un < L.nunits;
        Resolved dn = d;
        u32 rawn[kRegs];
        if (more) {
            dn = unit_of(L, un);
            Shape sn;
            Tile Tn;
            unit_shape<NT>(dn, sn, Tn);
            load_raw(sn, Tn, dn.x, threadIdx.x, rawn);
        }
        Shape s;
        Tile T;
        unit_shape<NT>(d, s, T);
        lds_tile<NT, F32>(d, s, T, raw, lds, err, d.x, d.y);
        if (!more) break;
        d = dn;
#pragma unroll
        for (int j = 0; j < kRegs; j++) raw[j] = rawn[j];
    }
}

// ------------------------------------------------------------------ 64-bit inputs

// k = 1 for 64-bit elements: y = x, argmed[o] = o.
__global__ __launch_bounds__(256) void k_identity64(const u64 *x, u64 *y, int32_t *argmed, int64_t total,
                                                    int64_t n)
{
    const int64_t o = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (o < total) {
        y[o] = x[o];
        if (argmed) argmed[o] = (int32_t)(o - (o / n) * n);
    }
}

__global__ void k_zero_counters(u32 *c, int n)
{
    const int i = threadIdx.x;
    if (i < n) c[i] = 0u;
}

// ------------------------------------------------------------------ global path

struct GLayout {
    int64_t xv, srt, srt2, M, pos, stage, total;
};
// After the sort, the sorted keys take the xv region and the slots the
// start of srt2; the staged medians overwrite them only after the pair
// orders are done.

__host__ __device__ inline void make_glayout(const Shape &s, GLayout *g)
{
    int64_t off = 0;
    g->xv = off;   off += 4ll * s.cap;
    g->srt = off;  off += 8ll * s.cap;
    g->srt2 = off; off += 8ll * s.cap;
    g->M = off;    off += 2ll * s.Pmax * s.Mstride;
    off = (off + 255) & ~255ll;
    g->pos = off;  off += 4ll * s.Pmax * s.Pstride;
    off = (off + 255) & ~255ll;
    g->total = off;
    g->stage = g->srt2;
}

// One-pair tiles (k > 4095), with the walk chunks that the coarse table in
// the workgroup's dynamic LDS allows.
__host__ __device__ inline int global_shape(int64_t n, int32_t k, Shape *s)
{
    int32_t S = 1;
    while (S < k) S <<= 1;
    const int r = make_shape(n, k, 2 * S / kRegs, s);
    if (r != 0) return r;
    global_chunks(s, S <= 16384 ? kGlobalLdsSmall : kGlobalLdsLarge);
    return 0;
}


// Bucket sort of a one-pair tile in global memory (P = 1).  Blocks A and B
// are sorted together by (key, block, t), which is the pair's merged order
// (A before B on equal keys), so M and the position maps come straight out
// of the sort.  Slot u = b << logS | t.  The counters (nbk 16-bit cells)
// live in LDS, the arrival numbers and the scattered values in the
// workspace.  Fills M (with its padding) and the position maps (the walk's
// chunk starts, chunk 0 included, come from the count table).  GW: slots
// per thread with their loads in flight together (4 in the two-workgroup
// form, whose 64 VGPRs it would otherwise overrun).  Returns false, having
// written only scratch, if a bucket overflows even under the logarithmic
// map; the caller then takes the merge sort.
template <bool F32, typename V, int GW, int STOP = 0>
__device__ __forceinline__ bool global_pair_bucket(const Shape &s, const Tile &T, const TileMem &m, const Resolved &d,
                                   u64 *srt_, u16 *arrv_, u32 *lcnt, u32 *gsh, u32 *wave_tot,
                                   const V *xo, V *yo)
{
    const int tid = threadIdx.x;
    const int NT = kGlobalThreads;
    const int32_t nbk = 2 * s.S;   // at most 65536 cells: 128 KB of LDS
    int32_t lognbk = 0;
    while ((1 << lognbk) < nbk) lognbk++;
    const int32_t lenB = T.lenLast;
    const int32_t N = s.k + lenB;
    const int32_t nslots = 2 * s.S;   // a multiple of kGW * NT
    // the signal and the workspace through global-space pointers (gmem)
    const MF_GLOBAL u32 *xt = gmem(d.x + T.e0);
    MF_GLOBAL u64 *srt = gmem(srt_);
    MF_GLOBAL u16 *arrv = gmem(arrv_);
    MF_GLOBAL u16 *Mg = gmem(m.M);
    // each pass below takes GW slots per thread at a time, u = u0 + q * NT,
    // with their loads in flight together (2S is a multiple of GW * NT)
    constexpr int kGW = GW;
    auto load_group = [&](int u0, u32 (&raw)[kGW], bool (&ok)[kGW]) {
#pragma unroll
        for (int q = 0; q < kGW; q++) {
            const int u = u0 + q * NT, b = u >> s.logS, tt = u & (s.S - 1);
            ok[q] = tt < (b ? lenB : s.k);
            raw[q] = ok[q] ? xt[b * s.k + tt] : 0u;
        }
    };
    auto key_of = [&](u32 raw) { return F32 ? key_of_f32(raw) : key_of_i32(raw); };
    auto cell = [&](u32 bk) { return (lcnt[bk >> 1] >> (16u * (bk & 1u))) & 0xFFFFu; };

    for (int e = tid; e < nbk / 2; e += NT) lcnt[e] = 0u;
    if (tid == 0) {
        gsh[0] = 0xFFFFFFFFu;
        gsh[1] = 0u;
        gsh[2] = 0u;
    }
    __syncthreads();
    // key range
    {
        u32 mn = 0xFFFFFFFFu, mx = 0u;
        for (int u0 = tid; u0 < nslots; u0 += kGW * NT) {
            u32 raw[kGW];
            bool ok[kGW];
            load_group(u0, raw, ok);
#pragma unroll
            for (int q = 0; q < kGW; q++) {
                const u32 key = key_of(raw[q]);
                mn = ok[q] && key < mn ? key : mn;
                mx = ok[q] && key > mx ? key : mx;
            }
        }
        mn = __ockl_wfred_min_u32(mn);
        mx = __ockl_wfred_max_u32(mx);
        if ((tid & 63) == 0 && mn <= mx) {
            atomicMin(gsh + 0, mn);
            atomicMax(gsh + 1, mx);
        }
    }
    __syncthreads();
    MF_STOP_AT_V(21, true)
    // arrival numbers: a crowded linear map is counted again with the
    // logarithmic one; if that overflows but the linear map only crowded,
    // the linear map is counted a third time and kept
    int pass = 0, round = 0;
    u32 fl0 = 0u;
    for (;; round++) {
        const BucketFn f = make_bucket_fn<F32>(nbk, lognbk, gsh[0], gsh[1], pass);
        u32 amax = 0u;
        for (int u0 = tid; u0 < nslots; u0 += kGW * NT) {
            u32 raw[kGW];
            bool ok[kGW];
            load_group(u0, raw, ok);
#pragma unroll
            for (int q = 0; q < kGW; q++) {
                if (!ok[q]) continue;
                const u32 bk = bucket_of<F32>(f, key_of(raw[q]));
                const u32 sh = 16u * (bk & 1u);
                const u32 a = (atomicAdd(lcnt + (bk >> 1), 1u << sh) >> sh) & 0xFFFFu;
                arrv[u0 + q * NT] = (u16)a;
                amax = a > amax ? a : amax;
            }
        }
        if (amax >= (u32)kBucketSoft) atomicOr(gsh + 2, amax >= (u32)kBucketMax ? 3u : 2u);
        __syncthreads();
        const u32 fl = gsh[2];
        if (round == 0) fl0 = fl;
        if ((round == 0 && (fl & 3u) == 0u) || (round == 1 && (fl & 1u) == 0u) || round == 2) break;
        if (round == 1 && (fl0 & 1u) != 0u) return false;
        __syncthreads();   // every thread has read the flag
        pass = round == 0 ? 1 : 0;
        for (int e = tid; e < nbk / 2; e += NT) lcnt[e] = 0u;
        if (tid == 0) gsh[2] = 0u;
        __syncthreads();
    }
    MF_STOP_AT_V(22, true)
    const BucketFn f = make_bucket_fn<F32>(nbk, lognbk, gsh[0], gsh[1], pass);
    // bucket starts: each thread's run of cells, then the runs' totals
    {
        const int32_t nd = nbk / 2 / NT;   // dwords per thread (8, 16 or 32)
        uint4 *cells = (uint4 *)(lcnt + tid * nd);
        u32 tot = 0u;
        for (int q = 0; q < nd / 4; q++) {
            const uint4 v = cells[q];
            tot += (v.x & 0xFFFFu) + (v.x >> 16) + (v.y & 0xFFFFu) + (v.y >> 16) +
                   (v.z & 0xFFFFu) + (v.z >> 16) + (v.w & 0xFFFFu) + (v.w >> 16);
        }
        u32 acc = seg_excl_scan<kGlobalThreads>(tot, NT, wave_tot);
        for (int q = 0; q < nd / 4; q++) {
            const uint4 v = cells[q];
            const u32 in[4] = {v.x, v.y, v.z, v.w};
            u32 out[4];
#pragma unroll
            for (int z = 0; z < 4; z++) {
                const u32 lo = acc, hi = acc + (in[z] & 0xFFFFu);
                acc = hi + (in[z] >> 16);
                out[z] = (lo & 0xFFFFu) | (hi << 16);
            }
            cells[q] = make_uint4(out[0], out[1], out[2], out[3]);
        }
    }
    __syncthreads();
    MF_STOP_AT_V(23, true)
    // scatter
    for (int u0 = tid; u0 < nslots; u0 += kGW * NT) {
        u32 raw[kGW], a[kGW];
        bool ok[kGW];
        load_group(u0, raw, ok);
#pragma unroll
        for (int q = 0; q < kGW; q++) a[q] = ok[q] ? arrv[u0 + q * NT] : 0u;
#pragma unroll
        for (int q = 0; q < kGW; q++) {
            if (!ok[q]) continue;
            const u32 key = key_of(raw[q]);
            srt[cell(bucket_of<F32>(f, key)) + a[q]] = ((u64)key << 32) | (u64)(u0 + q * NT);
        }
    }
    __syncthreads();
    MF_STOP_AT_V(24, true)
    // rank within the bucket, then the merged order and position maps; by
    // position of the scattered array, so that the reads are coalesced and
    // a bucket's other entries sit in the same cache lines
    MF_GLOBAL u16 *pos16 = gmem((u16 *)m.pos);
    for (int r0 = tid; r0 < N; r0 += kGW * NT) {
        u64 v[kGW];
#pragma unroll
        for (int q = 0; q < kGW; q++) v[q] = r0 + q * NT < N ? srt[r0 + q * NT] : 0ull;
#pragma unroll
        for (int q = 0; q < kGW; q++) {
            if (r0 + q * NT >= N) continue;
            const u32 key = (u32)(v[q] >> 32), u = (u32)v[q] & 0xFFFFu;
            const u32 b = u >> s.logS, tt = u & (u32)(s.S - 1);
            const u32 bk = bucket_of<F32>(f, key);
            const u32 x0 = cell(bk), hi = bk + 1u < (u32)nbk ? cell(bk + 1u) : (u32)N;
            const u32 fin = x0 + bucket_below(srt, x0, hi, v[q]);
            Mg[mslot((int32_t)fin)] = (u16)((b << 15) | tt);
            pos16[2 * tt + b] = (u16)fin;
        }
    }
    for (int r = N + tid; r < s.Mstride; r += NT) Mg[mslot(r)] = (u16)kMPad;
    __syncthreads();
    return true;
}

// Position words in flight per walk lane in the two-workgroup form (64
// VGPRs; the one-workgroup form keeps 8).
static const int kGwalkAheadTwo = 2;

// TWO: tiles of k <= 16383 (64 KB of LDS), compiled for two workgroups per
// CU (at most 64 VGPRs).  RK: int32 rank keys of a 64-bit signal (tile t's
// at L.x + t * L.xshift), medians copied from L.x64 to the 64-bit y.
template <bool F32, bool TWO, bool RK = false, int STOP = 0>
__global__ __launch_bounds__(kGlobalThreads) __attribute__((amdgpu_waves_per_eu(TWO ? 8 : 4)))
void k_tile_global(Launch L, unsigned char *ws, int64_t ws_stride, int *err)
{
    extern __shared__ __align__(16) unsigned char lds[];
    __shared__ u32 gsh[3];
    __shared__ u32 wave_tot[kGlobalThreads / 64];
    __shared__ u32 info[kGchunkMax];   // the walk chunks' starting columns
    u64 *sbuf = (u64 *)lds;   // kGlobalThreads * kRegs values
    const int tid = threadIdx.x;
    const int chunk = kGlobalThreads * kRegs;
    unsigned char *base = ws + (int64_t)blockIdx.x * ws_stride;

    for (int64_t uidx = blockIdx.x; uidx < L.nunits; uidx += gridDim.x) {
        const Resolved d = unit_of(L, uidx);
        const int64_t tile = d.tile;
        Shape s;
        global_shape(d.n, d.k, &s);
        GLayout g;
        make_glayout(s, &g);
        TileMem m = {};
        m.xv = (u32 *)(base + g.xv);
        u64 *srt = (u64 *)(base + g.srt);
        m.M = (u16 *)(base + g.M);
        m.pos = (u32 *)(base + g.pos);
        m.stage = (u16 *)(base + g.stage);
        u64 *srt2 = (u64 *)(base + g.srt2);
        const Tile T = make_tile(s, tile);
        const u32 *x = d.x;
        const int64_t row = RK ? uidx / L.tpr : 0;   // rows of a 64-bit launch
        const auto xo = [&]() { if constexpr (RK) return (const u64 *)L.x64 + row * d.n; else return d.x; }();
        const auto yo = [&]() {
            if constexpr (RK) return (u64 *)L.y + row * (d.n - d.k + 1);
            else return d.y;
        }();
        using GV = std::remove_pointer_t<decltype(yo)>;

        __syncthreads();   // the previous tile is done with the workspace
        // one-pair tiles: bucket sort of the pair (the LDS holds its bucket
        // counters, then the coarse count table, then a copy of M)
        if (T.P == 1 && s.S >= 8192 &&
            global_pair_bucket<F32, GV, TWO ? 4 : 8, STOP>(s, T, m, d, srt, (u16 *)srt2, (u32 *)lds, gsh, wave_tot, xo,
                                                           yo)) {
            if constexpr (STOP >= 21 && STOP <= 25) continue;
            tile_tail<kGlobalThreads, GV, STOP, TWO ? kGwalkAheadTwo : 8>(s, T, m, d, xo, yo, err, true, (u32 *)lds,
                                                                          info);
            continue;
        }
        if constexpr (STOP != 0) {   // (the probe times the bucket path only)
            if (threadIdx.x == 0) atomicOr(err, 2);
            continue;
        }
        // otherwise (a single block, or buckets that overflow on heavy ties):
        // merge sort of each block, then merge path per pair
        __syncthreads();
        for (int b = 0; b < T.NB; b++) {
            const int len = block_len(s, T, b);
            for (int t = tid; t < len; t += kGlobalThreads) load_item(s, T, m, x, b, t);
        }
        __syncthreads();

        // sort chunks of `chunk` slots in LDS; blocks larger than a chunk
        // get their last merge levels in global memory, alternating between
        // srt2 and srt so that the last one lands in srt
        int nlev = 0;
        for (int w = chunk; w < s.S; w <<= 1) nlev++;
        u64 *bufs[2] = {srt, srt2};
        int cur = nlev & 1;                 // buffer the LDS pass writes
        const int wmax = s.S < chunk ? s.S : chunk;
        for (int z = 0; z < s.cap / chunk; z++) {
            const int vt = z * kGlobalThreads + tid;
            u64 v[kRegs];
#pragma unroll
            for (int j = 0; j < kRegs; j++) v[j] = sort_value<F32>(s, T, m, vt * kRegs + j);
            sort_regs(v);
            for (int w = kRegs; w < wmax; w <<= 1) {
                store_regs(sbuf + tid * kRegs, v);
                __syncthreads();
                merge_level(sbuf, w, tid, v);
                __syncthreads();
            }
            store_regs((cur ? srt2 : srt) + (int64_t)vt * kRegs, v);
        }
        __syncthreads();
        for (int w = chunk; w < s.S; w <<= 1) {
            const u64 *src = cur ? srt2 : srt;
            u64 *dst = cur ? srt : srt2;
            const int vthreads = s.cap / kRegs;
            for (int vt = tid; vt < vthreads; vt += kGlobalThreads) {
                u64 v[kRegs];
                merge_level(src, w, vt, v);
                store_regs(dst + (int64_t)vt * kRegs, v);
            }
            cur ^= 1;
            __syncthreads();
        }
        (void)bufs;
        m.skey = (u32 *)(base + g.xv);
        m.sslot = (u16 *)(base + g.srt2);
        for (int u = tid; u < s.cap; u += kGlobalThreads) {
            const u64 v = srt[u];
            if (sv_valid(v)) put_block_value(s, m, u, v);
        }
        __syncthreads();
        // the sort buffer is free: it holds the coarse count table, then a
        // copy of M
        tile_tail<kGlobalThreads, GV, 0, TWO ? kGwalkAheadTwo : 8>(s, T, m, d, xo, yo, err, false, (u32 *)lds, info);
    }
}

// Rank pre-pass of a 64-bit signal on the global path (one pair of up to
// 2k items per tile): workgroups loop over tiles; each ranks its pair in
// chunks of kGlobalThreads * kRegs items in LDS, writes each chunk in sorted
// (key, offset) order to its scratch, merges the runs there (two copies;
// output tiles staged through LDS) and writes keys[t * stride + offset] =
// rank.
template <bool F64>
__global__ __launch_bounds__(kGlobalThreads) void k_rank64_pair(const u64 *x, int64_t n, int32_t k, u32 *keys,
                                                                int64_t stride, unsigned char *ws,
                                                                int64_t ws_stride, int64_t ntiles, int64_t nunits)
{
    extern __shared__ __align__(16) unsigned char lds[];
    constexpr int NT = kGlobalThreads;
    __shared__ int32_t split[16];   // two merge-path splits per output tile
    const int tid = threadIdx.x;
    const int32_t C = NT * kRegs;
    const int32_t smax = 2 * k;
    u64 *K0 = (u64 *)(ws + (int64_t)blockIdx.x * ws_stride);
    u64 *K1 = K0 + smax;
    u32 *O0 = (u32 *)(K1 + smax);
    u32 *O1 = O0 + smax;
    Shape s;
    global_shape(n, k, &s);
    for (int64_t u = blockIdx.x; u < nunits; u += gridDim.x) {
        const int64_t row = u / ntiles;
        const Tile T = make_tile(s, u - row * ntiles);
        const int32_t span = tile_items(s, T);
        const u64 *xt = x + row * n + T.e0;
        u64 *LK = (u64 *)lds;
        u32 *LO = (u32 *)(lds + 8 * C);
        for (int32_t c0 = 0; c0 < span; c0 += C) {
            const int32_t len = span - c0 < C ? span - c0 : C;
            rank_items<NT, F64>(xt + c0, len, lds);
            // the chunk in sorted order through LDS, then written contiguously
            u32 rr[kRegs];
            u64 kk[kRegs];
#pragma unroll
            for (int j = 0; j < kRegs; j++) {
                const int32_t i = tid * kRegs + j;
                rr[j] = 0u;
                kk[j] = 0ull;
                if (i < len) {
                    rr[j] = ((const u32 *)lds)[i];
                    kk[j] = F64 ? key_of_f64(xt[c0 + i]) : key_of_i64(xt[c0 + i]);
                }
            }
            __syncthreads();   // every rank is read
#pragma unroll
            for (int j = 0; j < kRegs; j++) {
                const int32_t i = tid * kRegs + j;
                if (i < len) {
                    LK[rr[j]] = kk[j];
                    LO[rr[j]] = (u32)(c0 + i);
                }
            }
            __syncthreads();
            for (int32_t p = tid; p < len; p += NT) {
                K0[c0 + p] = LK[p];
                O0[c0 + p] = LO[p];
            }
            __syncthreads();   // the next chunk reuses the LDS
        }
        u64 *Kin = K0, *Kout = K1;
        u32 *Oin = O0, *Oout = O1;
        const int32_t ntile = (span + C - 1) / C;   // at most 8 (2k < 65536)
        for (int32_t w = C; w < span; w <<= 1) {
            // the merge-path splits at the first and last output of every
            // output tile of the level, searched concurrently
            if (tid < 2 * ntile) {
                int32_t s0, lenA, lenB;
                const int32_t ob = (tid >> 1) * C;
                merge_runs(span, w, ob, s0, lenA, lenB);
                const int32_t d0 = ob - s0;
                const int32_t d1 = d0 + C < lenA + lenB ? d0 + C : lenA + lenB;
                split[tid] = merge_split_ko(Kin + s0, Oin + s0, lenA, Kin + s0 + w, Oin + s0 + w, lenB,
                                            (tid & 1) ? d1 : d0);
            }
            __syncthreads();
            for (int32_t ob = 0; ob < span; ob += C) {
                int32_t s0, lenA, lenB;
                merge_runs(span, w, ob, s0, lenA, lenB);
                const int32_t d0 = ob - s0;
                const int32_t d1 = d0 + C < lenA + lenB ? d0 + C : lenA + lenB;
                const int32_t ti = ob / C;
                const int32_t a0 = split[2 * ti], na = split[2 * ti + 1] - a0;
                const int32_t b0 = d0 - a0, nb = (d1 - d0) - na;
                for (int32_t i = tid; i < na + nb; i += NT) {
                    const int32_t src = i < na ? s0 + a0 + i : s0 + w + b0 + (i - na);
                    LK[i] = Kin[src];
                    LO[i] = Oin[src];
                }
                __syncthreads();
                u64 kv[kRegs];
                u32 ov[kRegs];
                const int32_t cnt = merge_local_ko(LK, LO, na, nb, tid * kRegs, kv, ov);
#pragma unroll
                for (int j = 0; j < kRegs; j++)
                    if (j < cnt) {
                        Kout[ob + tid * kRegs + j] = kv[j];
                        Oout[ob + tid * kRegs + j] = ov[j];
                    }
                __syncthreads();   // the next tile restages the LDS
            }
            u64 *tk = Kin; Kin = Kout; Kout = tk;
            u32 *to = Oin; Oin = Oout; Oout = to;
        }
        u32 *out = keys + u * stride;
        for (int32_t p = tid; p < span; p += NT) out[Oin[p]] = (u32)p;
        __syncthreads();   // the next tile reuses the scratch
    }
}

// ------------------------------------------------------------------ k = 1

__global__ void k_identity(Launch L)
{
    // unit = (signal, tile of 65536 outputs)
    for (int64_t uidx = blockIdx.x; uidx < L.nunits; uidx += gridDim.x) {
        const Resolved d = unit_of(L, uidx);
        const int64_t lo = d.tile * 65536;
        const int64_t hi = (lo + 65536 < d.n) ? lo + 65536 : d.n;
        for (int64_t o = lo + threadIdx.x; o < hi; o += blockDim.x) {
            d.y[o] = d.x[o];
            if (d.argmed) d.argmed[o] = (int32_t)o;
        }
    }
}

// ------------------------------------------------------------------ backward

// grad_x[j] = sum over o with argmed[o] == j of grad_y[o], float64, in
// increasing o.  Each wave owns kBwdTargetsPerWave consecutive targets and
// visits the outputs that can select them (o in [j-k+1, j]) 64 at a time in
// increasing order.  Within a batch, every lane finds the lanes holding its
// target (ten ballots, one per bit of the target); the lowest of them adds
// the batch's terms of that target to its accumulator, lane by lane in
// increasing lane (= increasing o) order, so every accumulator receives its
// terms in increasing o.
__device__ __forceinline__ u64 wave_ballot(bool p) { return (u64)__ballot(p); }

template <typename GT>
__global__ __launch_bounds__(kBwdThreads) void k_backward(BwdLaunch L)
{
    __shared__ double acc[kBwdThreads / 64][kBwdTargetsPerWave];
    __shared__ GT gstage[kBwdThreads / 64][64];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    double *A = acc[wave];
    GT *G = gstage[wave];

    for (int64_t uidx = blockIdx.x; uidx < L.nunits; uidx += gridDim.x) {
        SigDesc sd;
        int64_t tile;
        if (L.units) {
            const Unit u = L.units[uidx];
            sd = L.sigs[u.sig];
            tile = u.tile;
        } else {
            const int64_t row = uidx / L.tpr;
            tile = uidx - row * L.tpr;
            sd = L.one;
            sd.x_off += row * sd.n;
            sd.y_off += row * (sd.n - sd.k + 1);
        }
        struct {
            const GT *grad_y;
            const int32_t *argmed;
            GT *grad_x;
            int64_t n;
            int32_t k;
        } d = {(const GT *)L.grad_y + sd.y_off, L.argmed + sd.y_off, (GT *)L.grad_x + sd.x_off, sd.n, sd.k};
        const int64_t nout = d.n - d.k + 1;
        const int64_t j0 = tile * kBwdTargetsPerBlock + (int64_t)wave * kBwdTargetsPerWave;
        for (int t = lane; t < kBwdTargetsPerWave; t += 64) A[t] = 0.0;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (j0 < d.n) {
            const int64_t olo = (j0 - d.k + 1) > 0 ? (j0 - d.k + 1) : 0;
            int64_t ohi = j0 + kBwdTargetsPerWave;
            if (ohi > nout) ohi = nout;
            // candidates in groups of kBwdGroup batches of 64: the loads of
            // a whole group are issued together, then the batches retire in
            // order (increasing o)
            for (int64_t g0 = olo; g0 < ohi; g0 += 64 * kBwdGroup) {
                int tgt[kBwdGroup];
                GT gv[kBwdGroup];
#pragma unroll
                for (int q = 0; q < kBwdGroup; q++) {
                    const int64_t o = g0 + q * 64 + lane;
                    const bool in = o < ohi;
                    const int64_t oc = in ? o : ohi - 1;
                    const int64_t j = d.argmed[oc];
                    gv[q] = d.grad_y[oc];
                    tgt[q] = (in && j >= j0 && j < j0 + kBwdTargetsPerWave) ? (int)(j - j0) : -1;
                }
#pragma unroll
                for (int q = 0; q < kBwdGroup; q++) {
                    const int t = tgt[q];
                    const bool valid = t >= 0;
                    // lanes of the batch holding the same target as this lane
                    u64 same = wave_ballot(valid);
#pragma unroll
                    for (int bit = 0; bit < 10; bit++) {
                        const u64 ones = wave_ballot(valid && ((t >> bit) & 1));
                        same &= ((t >> bit) & 1) ? ones : ~ones;
                    }
                    G[lane] = gv[q];
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    // the lowest lane of each target adds the target's terms
                    if (valid && ((same & ((1ull << lane) - 1ull)) == 0ull)) {
                        double a = A[t];
                        u64 rem = same;
                        while (rem) {
                            a += (double)G[__ffsll((unsigned long long)rem) - 1];
                            rem &= rem - 1ull;
                        }
                        A[t] = a;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
            for (int t = lane; t < kBwdTargetsPerWave; t += 64)
                if (j0 + t < d.n) d.grad_x[j0 + t] = (GT)A[t];
        }
        __syncthreads();
    }
}

// The same sums for float32 gradients and windows up to kBwdSegMaxK, by
// exact accumulation.  Every term g is a multiple of 2^lsb(g), lsb(g) =
// e - 150 for biased exponent e (subnormals count as e = 1).  When a
// target's terms satisfy sum |g| < 2^(min lsb + 52), every partial sum of
// them, in any order, is an integer multiple of 2^(min lsb) below 2^52 of
// them, so float64 holds it exactly: the sum in increasing o never rounds
// and equals the exact sum, which any order of float64 additions
// reproduces, LDS float64 atomics included.
// Each wave owns kBwdSegTargetsPerWave consecutive targets [j0, j0 + TJ)
// and reads the outputs that can select them, o in [j0 - k + 1, j0 + TJ),
// kBwdInflight batches of 64 at a time (a group's loads issued before its
// first atomic).  A target has at most k terms, each below 2^(emax - 126),
// so a tile whose terms have exponents in [emin, emax] with
// ceil(log2 k) + emax - emin <= 28 is exact for every target (the usual
// case): one atomic per term.  A tile outside that (huge spreads of
// magnitude, infinities, NaN) is redone target by target in the same 8
// bytes per target: first each target's magnitude sum (float32, whose
// relative error over at most 2^11 terms stays below 2^-13, so the test
// asks for half the bound) and least exponent, which give each lane its
// targets' verdicts; then the float64 sums again; a target outside the
// bound is summed again in increasing o from the inputs.
__device__ __forceinline__ u32 bwd_exp(float g)
{
    const u32 e = (__float_as_uint(g) >> 23) & 0xFFu;
    return e > 0u ? e : 1u;
}

__global__ __launch_bounds__(kBwdThreads) void k_backward_exact(BwdLaunch L)
{
    constexpr int TJ = kBwdSegTargetsPerWave;
    constexpr int B = kBwdInflight;
    constexpr int PER = TJ / 64;   // targets per lane: t = lane + 64 i
    // per target: the float64 sum, or (slow tiles, first) the float32
    // magnitude sum and the least biased exponent
    __shared__ double acc_s[kBwdThreads / 64][TJ];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    double *acc = acc_s[wave];
    float *mag = (float *)acc;           // mag[2t]
    u32 *lsb = (u32 *)acc;               // lsb[2t + 1]

    for (int64_t uidx = blockIdx.x; uidx < L.nunits; uidx += gridDim.x) {
        SigDesc sd;
        int64_t tile;
        if (L.units) {
            const Unit u = L.units[uidx];
            sd = L.sigs[u.sig];
            tile = u.tile;
        } else {
            const int64_t row = uidx / L.tpr;
            tile = uidx - row * L.tpr;
            sd = L.one;
            sd.x_off += row * sd.n;
            sd.y_off += row * (sd.n - sd.k + 1);
        }
        const float *grad_y = (const float *)L.grad_y + sd.y_off;
        const int32_t *argmed = L.argmed + sd.y_off;
        float *grad_x = (float *)L.grad_x + sd.x_off;
        // signals are shorter than 2^31: 32-bit indices from here on
        const int32_t n = (int32_t)sd.n, k = sd.k, nout = n - k + 1;
        const int64_t j0l = tile * kBwdSegTargetsPerBlock + (int64_t)wave * TJ;
        if (j0l >= n) continue;   // the waves share no LDS and no barrier
        const int32_t j0 = (int32_t)j0l;
        const int32_t olo = j0 - k + 1 > 0 ? j0 - k + 1 : 0;
        const int32_t ohi = j0 + TJ < nout ? j0 + TJ : nout;

        // pass over the tile's terms: f(t, g) for every output o of a target
        // t in the tile, g = grad_y[o]
        auto terms = [&](auto f) {
            for (int32_t o0 = olo; o0 < ohi; o0 += 64 * B) {
                u32 tt[B];
                float gg[B];
#pragma unroll
                for (int q = 0; q < B; q++) {
                    const int32_t o = o0 + q * 64 + lane;
                    tt[q] = o < ohi ? (u32)(argmed[o] - j0) : 0xFFFFFFFFu;
                }
#pragma unroll
                for (int q = 0; q < B; q++) gg[q] = tt[q] < (u32)TJ ? grad_y[o0 + q * 64 + lane] : 0.0f;
#pragma unroll
                for (int q = 0; q < B; q++)
                    if (tt[q] < (u32)TJ) f(tt[q], gg[q]);
            }
        };

        for (int t = lane; t < TJ; t += 64) acc[t] = 0.0;
        wave_sync();
        u32 emin = 0xFFu, emax = 0u;
        terms([&](u32 t, float g) {
            atomicAdd(&acc[t], (double)g);
            if (g != 0.0f) {
                const u32 e = bwd_exp(g);
                emin = e < emin ? e : emin;
                emax = e > emax ? e : emax;
            }
        });
        emin = __ockl_wfred_min_u32(emin);
        emax = __ockl_wfred_max_u32(emax);
        const u32 lk = 32u - (u32)__clz((int)(k - 1));   // ceil(log2 k)
        const bool exact = emax == 0u || (emax < 255u && lk + emax <= 28u + emin);
        wave_sync();
        u32 slow = 0u;   // bit i: target lane + 64 i needs the ordered sum
        if (!exact) {
            for (int t = lane; t < TJ; t += 64) {
                mag[2 * t] = 0.0f;
                lsb[2 * t + 1] = 0xFFFFFFFFu;
            }
            wave_sync();
            terms([&](u32 t, float g) {
                if (g != 0.0f) {
                    atomicAdd(&mag[2 * t], fabsf(g));
                    atomicMin(&lsb[2 * t + 1], bwd_exp(g));
                }
            });
            wave_sync();
#pragma unroll
            for (int i = 0; i < PER; i++) {
                const int t = lane + 64 * i;
                const u32 e = lsb[2 * t + 1];
                if (e != 0xFFFFFFFFu && !((double)mag[2 * t] < ldexp(1.0, (int)e - 150 + 51))) slow |= 1u << i;
            }
            // (each phase reaches a cell through one type: the fences keep
            // the float and u32 views apart from the float64 one)
            wave_sync();
            for (int t = lane; t < TJ; t += 64) acc[t] = 0.0;
            wave_sync();
            terms([&](u32 t, float g) { atomicAdd(&acc[t], (double)g); });
            wave_sync();
        }
#pragma unroll
        for (int i = 0; i < PER; i++) {
            const int t = lane + 64 * i;
            const int32_t j = j0 + t;
            if (j >= n) break;
            double a = acc[t];
            if ((slow >> i) & 1u) {
                a = 0.0;
                const int32_t lo = j - k + 1 > 0 ? j - k + 1 : 0, hi = j < nout - 1 ? j : nout - 1;
                for (int32_t o = lo; o <= hi; o++)
                    if (argmed[o] == j) a += (double)grad_y[o];
            }
            grad_x[j] = (float)a;
        }
        wave_sync();   // the next unit reuses the wave's LDS
    }
}

// ------------------------------------------------------------------ host side

Path path_for(int32_t k)
{
    if (k == 1) return PATH_IDENTITY;
    int32_t S = 1;
    while (S < k) S <<= 1;
    if (2 * S <= kLdsSmall * kRegs) return PATH_LDS_SMALL;
    if (2 * S <= kLdsLarge * kRegs) return PATH_LDS_LARGE;
    if (k <= 32767) return PATH_GLOBAL;
    return PATH_NONE;
}

int64_t tiles_for(Path p, int64_t n, int32_t k)
{
    Shape s;
    switch (p) {
    case PATH_IDENTITY: return (n + 65535) / 65536;
    case PATH_LDS_SMALL: make_shape(n, k, kLdsSmall, &s); return s.ntiles;
    case PATH_LDS_LARGE: make_shape(n, k, kLdsLarge, &s); return s.ntiles;
    case PATH_GLOBAL: global_shape(n, k, &s); return s.ntiles;
    default: return 0;
    }
}

int64_t lds_bytes_for(Path p, int32_t k)
{
    Shape s;
    Layout l;
    switch (p) {
    case PATH_LDS_SMALL: make_shape(1ll << 20, k, kLdsSmall, &s); make_layout(s, &l); return l.total;
    case PATH_LDS_LARGE: make_shape(1ll << 20, k, kLdsLarge, &s); make_layout(s, &l); return l.total;
    case PATH_GLOBAL: {
        int32_t S = 1;
        while (S < k) S <<= 1;
        return S <= 16384 ? kGlobalLdsSmall : kGlobalLdsLarge;
    }
    default: return 0;
    }
}

int64_t global_ws_slots(size_t lds_bytes)
{
    return lds_bytes <= (size_t)kGlobalLdsSmall ? 512 : 256;
}

int64_t global_ws_stride(int32_t k)
{
    Shape s;
    global_shape(1ll << 30, k, &s);
    GLayout g;
    make_glayout(s, &g);
    return (g.total + 255) & ~255ll;
}

// ------------------------------------------------------------------ fixed scratch

// The scratch of the entry point that allocates nothing, one array per
// device that the library runs on, held until the process ends.  Host code
// never passes this name to a kernel: it stands for the array only on the
// device, so every host use goes through the address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kFixedScratchBytes];

hipError_t fixed_scratch(hipStream_t st, bool create, unsigned char **out)
{
    static std::mutex mu;
    static unsigned char *addr[64] = {};
    *out = nullptr;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev] && create) {
        unsigned char *p = nullptr;
        e = hipGetSymbolAddress((void **)&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        if ((e = prepare_kernels()) != hipSuccess) return e;
        // the flag starts clear: a fill kernel (no memset node), waited for
        hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, (u32 *)p, 1);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return e;
        addr[dev] = p;
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t prepare_kernels()
{
    hipError_t e = hipSuccess;
    const int big = 156 * 1024;   // room for the kernels' small static LDS arrays
    const int gbig = 152 * 1024;  // the one-pair tiles' static arrays take about 4 KB
#define MF_ATTR_BYTES(kern, bytes)                                                           \
    if (e == hipSuccess)                                                                     \
        e = hipFuncSetAttribute((const void *)(kern), hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
#define MF_ATTR(kern) MF_ATTR_BYTES(kern, big)
    MF_ATTR((k_tile_lds<kLdsSmall, true>))
    MF_ATTR((k_tile_lds<kLdsSmall, false>))
    MF_ATTR((k_tile_lds<kLdsLarge, true>))
    MF_ATTR((k_tile_lds<kLdsLarge, false>))
    MF_ATTR((k_tile_lds<kLdsSmall, false, 2>))
    MF_ATTR((k_tile_lds<kLdsSmall, false, 3>))
    MF_ATTR((k_tile_lds<kLdsLarge, false, 1>))
    MF_ATTR((k_tile_lds_persistent<kLdsSmall, true>))
    MF_ATTR((k_tile_lds_persistent<kLdsLarge, true>))
    MF_ATTR((k_tile_lds_persistent<kLdsSmall, false>))
    MF_ATTR((k_tile_lds_persistent<kLdsLarge, false>))
    MF_ATTR_BYTES((k_tile_global<true, false>), gbig)
    MF_ATTR_BYTES((k_tile_global<false, false>), gbig)
    MF_ATTR_BYTES((k_tile_global<true, true>), gbig)
    MF_ATTR_BYTES((k_tile_global<false, true>), gbig)
    MF_ATTR_BYTES((k_tile_global<false, true, true>), gbig)
    MF_ATTR_BYTES((k_tile_global<false, false, true>), gbig)
    MF_ATTR((k_rank64_pair<true>))
    MF_ATTR((k_rank64_pair<false>))
    MF_ATTR((k_rank64<kLdsLarge, true>))
    MF_ATTR((k_rank64<kLdsLarge, false>))
#undef MF_ATTR
#undef MF_ATTR_BYTES
    return e;
}

// Workgroups of `kern` (nt threads, lds bytes of dynamic LDS) resident on
// the current device at once; cached per (kernel, lds) on each device.
static hipError_t resident_workgroups(const void *kern, int nt, size_t lds, int64_t *out)
{
    struct Entry {
        int dev;
        const void *kern;
        size_t lds;
        int64_t n;
    };
    static std::mutex mu;
    static std::vector<Entry> cache;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    {
        std::lock_guard<std::mutex> lk(mu);
        for (const Entry &c : cache)
            if (c.dev == dev && c.kern == kern && c.lds == lds) {
                *out = c.n;
                return hipSuccess;
            }
    }
    int cus = 0, per_cu = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const int64_t n = (int64_t)cus * per_cu;
    std::lock_guard<std::mutex> lk(mu);
    if (cache.size() < 256) cache.push_back(Entry{dev, kern, lds, n});
    *out = n;
    return hipSuccess;
}

hipError_t launch_forward(Path p, bool f32, const Launch &L, size_t lds_bytes,
                          unsigned char *ws, int64_t ws_stride, int64_t ws_slots,
                          int *d_err, hipStream_t st)
{
    if (L.nunits <= 0) return hipSuccess;
    switch (p) {
    case PATH_IDENTITY: {
        const int64_t grid = L.nunits < 65536 ? L.nunits : 65536;
        hipLaunchKernelGGL(k_identity, dim3((unsigned)grid), dim3(256), 0, st, L);
        break;
    }
    case PATH_LDS_SMALL:
    case PATH_LDS_LARGE: {
        const int nt = p == PATH_LDS_SMALL ? kLdsSmall : kLdsLarge;
        const dim3 g((unsigned)L.nunits), b((unsigned)nt);
        if (p == PATH_LDS_SMALL) {
            if (f32) hipLaunchKernelGGL((k_tile_lds<kLdsSmall, true>), g, b, lds_bytes, st, L, d_err);
            else if (L.rank_mode == 2) hipLaunchKernelGGL((k_tile_lds<kLdsSmall, false, 2>), g, b, lds_bytes, st, L, d_err);
            else if (L.rank_mode == 3) hipLaunchKernelGGL((k_tile_lds<kLdsSmall, false, 3>), g, b, lds_bytes, st, L, d_err);
            else if (L.rank_mode != 0) return hipErrorInvalidValue;
            else     hipLaunchKernelGGL((k_tile_lds<kLdsSmall, false>), g, b, lds_bytes, st, L, d_err);
        } else {
            if (f32) hipLaunchKernelGGL((k_tile_lds<kLdsLarge, true>), g, b, lds_bytes, st, L, d_err);
            else if (L.rank_mode == 1) hipLaunchKernelGGL((k_tile_lds<kLdsLarge, false, 1>), g, b, lds_bytes, st, L, d_err);
            else if (L.rank_mode != 0) return hipErrorInvalidValue;
            else     hipLaunchKernelGGL((k_tile_lds<kLdsLarge, false>), g, b, lds_bytes, st, L, d_err);
        }
        break;
    }
    case PATH_GLOBAL: {
        const int64_t grid = L.nunits < ws_slots ? L.nunits : ws_slots;
        const dim3 g((unsigned)grid), b(kGlobalThreads);
        if (L.rank_mode != 0 && (f32 || L.rank_mode != 1)) return hipErrorInvalidValue;
        if (lds_bytes <= (size_t)kGlobalLdsSmall) {
            if (f32) hipLaunchKernelGGL((k_tile_global<true, true>), g, b, lds_bytes, st, L, ws, ws_stride, d_err);
            else if (L.rank_mode) hipLaunchKernelGGL((k_tile_global<false, true, true>), g, b, lds_bytes, st, L, ws, ws_stride, d_err);
            else     hipLaunchKernelGGL((k_tile_global<false, true>), g, b, lds_bytes, st, L, ws, ws_stride, d_err);
        } else {
            if (f32) hipLaunchKernelGGL((k_tile_global<true, false>), g, b, lds_bytes, st, L, ws, ws_stride, d_err);
            else if (L.rank_mode) hipLaunchKernelGGL((k_tile_global<false, false, true>), g, b, lds_bytes, st, L, ws, ws_stride, d_err);
            else     hipLaunchKernelGGL((k_tile_global<false, false>), g, b, lds_bytes, st, L, ws, ws_stride, d_err);
        }
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_forward_persistent(Path p, bool f32, const Launch &L, size_t lds_bytes, u32 *next,
                                    int *d_err, hipStream_t st)
{
    if (L.nunits <= 0) return hipSuccess;
    if (p != PATH_LDS_SMALL && p != PATH_LDS_LARGE) return hipErrorInvalidValue;
    const int nt = p == PATH_LDS_SMALL ? kLdsSmall : kLdsLarge;
    const void *kern = p == PATH_LDS_SMALL
                           ? (f32 ? (const void *)k_tile_lds_persistent<kLdsSmall, true> : (const void *)k_tile_lds_persistent<kLdsSmall, false>)
                           : (f32 ? (const void *)k_tile_lds_persistent<kLdsLarge, true> : (const void *)k_tile_lds_persistent<kLdsLarge, false>);
    int64_t grid = 0;
    hipError_t e = resident_workgroups(kern, nt, lds_bytes, &grid);
    if (e != hipSuccess) return e;
    if (grid > L.nunits) grid = L.nunits;
    hipLaunchKernelGGL(k_zero_counters, dim3(1), dim3(64), 0, st, next, 1);
    const dim3 g((unsigned)grid);
    if (p == PATH_LDS_SMALL) {
        if (f32) hipLaunchKernelGGL((k_tile_lds_persistent<kLdsSmall, true>), g, dim3(kLdsSmall), lds_bytes, st, L, next, d_err);
        else     hipLaunchKernelGGL((k_tile_lds_persistent<kLdsSmall, false>), g, dim3(kLdsSmall), lds_bytes, st, L, next, d_err);
    } else {
        if (f32) hipLaunchKernelGGL((k_tile_lds_persistent<kLdsLarge, true>), g, dim3(kLdsLarge), lds_bytes, st, L, next, d_err);
        else     hipLaunchKernelGGL((k_tile_lds_persistent<kLdsLarge, false>), g, dim3(kLdsLarge), lds_bytes, st, L, next, d_err);
    }
    return hipGetLastError();
}

bool bwd_seg_for(int32_t k, bool f64) { return !f64 && k <= kBwdSegMaxK; }

int64_t bwd_tiles_for(int64_t n, int32_t k, bool f64)
{
    const int64_t per = bwd_seg_for(k, f64) ? kBwdSegTargetsPerBlock : kBwdTargetsPerBlock;
    return (n + per - 1) / per;
}

hipError_t launch_backward(const BwdLaunch &L, bool f64, hipStream_t st)
{
    if (L.nunits <= 0) return hipSuccess;
    const int64_t grid = L.nunits < (1ll << 20) ? L.nunits : (1ll << 20);
    if (L.seg) {
        if (f64) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_backward_exact, dim3((unsigned)grid), dim3(kBwdThreads), 0, st, L);
        return hipGetLastError();
    }
    if (f64) hipLaunchKernelGGL(k_backward<double>, dim3((unsigned)grid), dim3(kBwdThreads), 0, st, L);
    else     hipLaunchKernelGGL(k_backward<float>, dim3((unsigned)grid), dim3(kBwdThreads), 0, st, L);
    return hipGetLastError();
}


int64_t rank64_lds_bytes_for(Path p, int32_t k)
{
    const int64_t tile = lds_bytes_for(p, k);
    const int64_t rank = 12ll * (p == PATH_LDS_SMALL ? kLdsSmall : kLdsLarge) * kRegs;
    return tile > rank ? tile : rank;
}

int64_t rank64_stride_for(Path p, int32_t k)
{
    Shape s;
    if (p == PATH_GLOBAL) {
        global_shape(1ll << 20, k, &s);
        return rank64_stride(s);
    }
    if (p != PATH_LDS_SMALL && p != PATH_LDS_LARGE) return 0;
    make_shape(1ll << 20, k, p == PATH_LDS_SMALL ? kLdsSmall : kLdsLarge, &s);
    return rank64_stride(s);
}

hipError_t launch_rank64(Path p, bool f64, const void *x, int64_t n, int32_t k, u32 *keys, int64_t stride,
                         int64_t ntiles, int64_t nunits, hipStream_t st)
{
    if (nunits <= 0) return hipSuccess;
    if (p != PATH_LDS_LARGE) return hipErrorInvalidValue;   // 512-thread tiles rank in their own LDS
    const dim3 g((unsigned)nunits);
    const size_t lds = 12u * kLdsLarge * kRegs;
    if (f64) hipLaunchKernelGGL((k_rank64<kLdsLarge, true>), g, dim3(kLdsLarge), lds, st, (const u64 *)x, n, k, keys, stride, ntiles);
    else     hipLaunchKernelGGL((k_rank64<kLdsLarge, false>), g, dim3(kLdsLarge), lds, st, (const u64 *)x, n, k, keys, stride, ntiles);
    return hipGetLastError();
}

int64_t rank64_pair_scratch(int32_t k) { return pair_rank_scratch(k); }

hipError_t launch_rank64_pair(bool f64, const void *x, int64_t n, int32_t k, u32 *keys, int64_t stride,
                              unsigned char *ws, int64_t ws_stride, int64_t slots, int64_t ntiles, int64_t nunits,
                              hipStream_t st)
{
    if (nunits <= 0) return hipSuccess;
    const dim3 g((unsigned)(slots < nunits ? slots : nunits));
    const size_t lds = 12u * kGlobalThreads * kRegs;
    if (f64) hipLaunchKernelGGL((k_rank64_pair<true>), g, dim3(kGlobalThreads), lds, st, (const u64 *)x, n, k, keys,
                                stride, ws, ws_stride, ntiles, nunits);
    else     hipLaunchKernelGGL((k_rank64_pair<false>), g, dim3(kGlobalThreads), lds, st, (const u64 *)x, n, k, keys,
                                stride, ws, ws_stride, ntiles, nunits);
    return hipGetLastError();
}

hipError_t launch_identity64(const void *x, void *y, int32_t *argmed, int64_t total, int64_t n, hipStream_t st)
{
    if (total <= 0) return hipSuccess;
    const dim3 g((unsigned)((total + 255) / 256));
    hipLaunchKernelGGL(k_identity64, g, dim3(256), 0, st, (const u64 *)x, (u64 *)y, argmed, total, n);
    return hipGetLastError();
}

}  // namespace mf

#ifdef MF_PHASE_PROBE
#include <string.h>
// Phase-probe build only (not part of libmf.so): the int32 forward on
// 512-thread tiles with every workgroup returning after tile phase `stop`
// (1 .. 17 as numbered by MF_STOP_AT; 0 runs whole tiles).  The outputs of a
// stopped launch are not written.  Returns a hipError_t.
namespace mf {
template <int S>
static hipError_t probe_launch(const Launch &L, size_t lds, int *err, hipStream_t st)
{
    hipError_t e = hipFuncSetAttribute((const void *)k_tile_lds<kLdsSmall, false, 0, S>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 156 * 1024);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tile_lds<kLdsSmall, false, 0, S>), dim3((unsigned)L.nunits), dim3(kLdsSmall), lds, st, L,
                       err);
    return hipGetLastError();
}
}  // namespace mf

extern "C" int mf_phase_probe_i32(const void *x, int64_t n, int32_t k, void *y, int32_t *argmed, int stop,
                                  void *stream)
{
    using namespace mf;
    static int *err = nullptr;
    if (path_for(k) != PATH_LDS_SMALL || n < k || n > INT32_MAX) return (int)hipErrorInvalidValue;
    if (!err && hipMalloc(&err, sizeof(int)) != hipSuccess) return (int)hipErrorOutOfMemory;
    Launch L;
    memset(&L, 0, sizeof L);
    L.x = x;
    L.y = y;
    L.argmed = argmed;
    L.one.n = n;
    L.one.k = k;
    L.rows = 1;
    L.tpr = tiles_for(PATH_LDS_SMALL, n, k);
    L.nunits = L.tpr;
    const size_t lds = (size_t)lds_bytes_for(PATH_LDS_SMALL, k);
    const hipStream_t st = (hipStream_t)stream;
    switch (stop) {
    case 0: return (int)probe_launch<0>(L, lds, err, st);
    case 1: return (int)probe_launch<1>(L, lds, err, st);
    case 2: return (int)probe_launch<2>(L, lds, err, st);
    case 3: return (int)probe_launch<3>(L, lds, err, st);
    case 4: return (int)probe_launch<4>(L, lds, err, st);
    case 5: return (int)probe_launch<5>(L, lds, err, st);
    case 6: return (int)probe_launch<6>(L, lds, err, st);
    case 7: return (int)probe_launch<7>(L, lds, err, st);
    case 8: return (int)probe_launch<8>(L, lds, err, st);
    case 9: return (int)probe_launch<9>(L, lds, err, st);
    case 10: return (int)probe_launch<10>(L, lds, err, st);
    case 11: return (int)probe_launch<11>(L, lds, err, st);
    case 12: return (int)probe_launch<12>(L, lds, err, st);
    case 13: return (int)probe_launch<13>(L, lds, err, st);
    case 14: return (int)probe_launch<14>(L, lds, err, st);
    case 15: return (int)probe_launch<15>(L, lds, err, st);
    case 16: return (int)probe_launch<16>(L, lds, err, st);
    case 17: return (int)probe_launch<17>(L, lds, err, st);
    default: return (int)hipErrorInvalidValue;
    }
}

// The float32 forward on the one-pair tiles of the workspace path (4095 <
// k <= 32767) with every tile stopping after phase `stop` (21 .. 30 as
// numbered by MF_STOP_AT; 0 runs whole tiles), in the launch configuration
// of the library (two workgroups per CU up to k = 16383).  Tiles whose
// bucket sort overflows take no part (err bit 1 is set).  Uses a workspace of
// its own.  Returns a hipError_t.
namespace mf {
template <int S>
static hipError_t gprobe_launch(const Launch &L, size_t lds, unsigned char *ws, int64_t stride, int64_t slots,
                                int *err, hipStream_t st)
{
    const dim3 g((unsigned)(L.nunits < slots ? L.nunits : slots)), b(kGlobalThreads);
    const bool two = lds <= (size_t)kGlobalLdsSmall;
    const void *kern = two ? (const void *)k_tile_global<true, true, false, S>
                           : (const void *)k_tile_global<true, false, false, S>;
    hipError_t e = hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, 152 * 1024);
    if (e != hipSuccess) return e;
    if (two) hipLaunchKernelGGL((k_tile_global<true, true, false, S>), g, b, lds, st, L, ws, stride, err);
    else hipLaunchKernelGGL((k_tile_global<true, false, false, S>), g, b, lds, st, L, ws, stride, err);
    return hipGetLastError();
}
}  // namespace mf

extern "C" int mf_phase_probe_global_f32(const void *x, int64_t n, int32_t k, void *y, int32_t *argmed, int stop,
                                         void *stream)
{
    using namespace mf;
    static int *err = nullptr;
    static unsigned char *ws = nullptr;
    static size_t wsb = 0;
    if (path_for(k) != PATH_GLOBAL || n < 2 * (int64_t)k || n > INT32_MAX) return (int)hipErrorInvalidValue;
    if (!err && hipMalloc(&err, sizeof(int)) != hipSuccess) return (int)hipErrorOutOfMemory;
    const size_t lds = (size_t)lds_bytes_for(PATH_GLOBAL, k);
    const int64_t slots = global_ws_slots(lds), stride = global_ws_stride(k);
    if (wsb < (size_t)(slots * stride)) {
        if (ws && hipFree(ws) != hipSuccess) return (int)hipErrorInvalidValue;
        ws = nullptr;
        wsb = 0;
        if (hipMalloc(&ws, (size_t)(slots * stride)) != hipSuccess) return (int)hipErrorOutOfMemory;
        wsb = (size_t)(slots * stride);
    }
    Launch L;
    memset(&L, 0, sizeof L);
    L.x = x;
    L.y = y;
    L.argmed = argmed;
    L.one.n = n;
    L.one.k = k;
    L.rows = 1;
    L.tpr = tiles_for(PATH_GLOBAL, n, k);
    L.nunits = L.tpr;
    const hipStream_t st = (hipStream_t)stream;
    switch (stop) {
    case 0: return (int)gprobe_launch<0>(L, lds, ws, stride, slots, err, st);
    case 21: return (int)gprobe_launch<21>(L, lds, ws, stride, slots, err, st);
    case 22: return (int)gprobe_launch<22>(L, lds, ws, stride, slots, err, st);
    case 23: return (int)gprobe_launch<23>(L, lds, ws, stride, slots, err, st);
    case 24: return (int)gprobe_launch<24>(L, lds, ws, stride, slots, err, st);
    case 25: return (int)gprobe_launch<25>(L, lds, ws, stride, slots, err, st);
    case 26: return (int)gprobe_launch<26>(L, lds, ws, stride, slots, err, st);
    case 27: return (int)gprobe_launch<27>(L, lds, ws, stride, slots, err, st);
    case 28: return (int)gprobe_launch<28>(L, lds, ws, stride, slots, err, st);
    case 29: return (int)gprobe_launch<29>(L, lds, ws, stride, slots, err, st);
    case 30: return (int)gprobe_launch<30>(L, lds, ws, stride, slots, err, st);
    default: return (int)hipErrorInvalidValue;
    }
}
#endif
