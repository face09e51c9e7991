// Host-side run of the tile phases (paper_1406_1717_amd/csrc/mf_tile.h),
// one work item after another, in the order the GPU kernel runs them.
// Test-only: it checks the tile logic (indexing, tables, walk) on the CPU,
// with bounds checks on every tile buffer.  It is not a fallback of the
// library and nothing in the product loads it.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <algorithm>
#include <vector>

#include "../../paper_1406_1717_amd/csrc/mf_tile.h"

using namespace mf;

static int g_force_merge = 0;
static long g_fast_tiles = 0, g_slow_tiles = 0, g_recount_tiles = 0, g_tile_order_tiles = 0, g_presorted_tiles = 0;
extern "C" void emu_set_force_merge(int v) { g_force_merge = v; }
static long g_rank_bucket_tiles = 0, g_rank_merge_tiles = 0;
extern "C" long emu_rank_bucket_tiles(void) { return g_rank_bucket_tiles; }
extern "C" long emu_rank_merge_tiles(void) { return g_rank_merge_tiles; }
extern "C" long emu_fast_tiles(void) { return g_fast_tiles; }
extern "C" long emu_slow_tiles(void) { return g_slow_tiles; }
extern "C" long emu_recount_tiles(void) { return g_recount_tiles; }
extern "C" long emu_tile_order_tiles(void) { return g_tile_order_tiles; }
extern "C" long emu_presorted_tiles(void) { return g_presorted_tiles; }

static long g_ranked_tiles = 0;
extern "C" long emu_ranked_tiles(void) { return g_ranked_tiles; }

// x: the 32-bit inputs the tile sorts; xo, yo: the elements the medians are
// copied from and to (x and y, or a 64-bit signal's elements when x holds
// its rank keys).
template <bool F32, typename E>
static int run_tile(const Shape &s, const Layout &l, int64_t t, int threads,
                    const u32 *x, const E *xo, E *yo, int32_t *argmed, std::vector<unsigned char> &lds,
                    bool ranked_keys = false, const u32 *rank_lds = nullptr)
{
    const Tile T = make_tile(s, t);
    // poison the tile memory so that reads of unwritten data show up
    memset(lds.data(), 0xA5, lds.size());
    TileMem m = tile_mem(lds.data(), l);
    bool tord = tile_order_ok(s);
    const Shape st = tile_order_shape(s);
    const int per = tile_buckets(s) / threads;   // counters per thread

    std::vector<u64> regs((size_t)threads * kRegs), tmp((size_t)threads * kRegs);
    for (int q = 0; q < threads; q++) {
        u64 v[kRegs];
        u32 raw[kRegs];
        if (rank_lds) rank_raw(s, T, rank_lds, q, raw);   // a tile that ranked its 64-bit items
        else load_raw(s, T, x, q, raw);
        if (tord) load_tile_values<F32>(s, T, m, raw, q, v);
        else load_sort_values<F32>(s, T, m, raw, q, v);
        for (int j = 0; j < kRegs; j++) regs[(size_t)q * kRegs + j] = v[j];
    }
    auto V = [&](int q, u64 (&v)[kRegs]) { for (int j = 0; j < kRegs; j++) v[j] = regs[(size_t)q * kRegs + j]; };
    int pass = 0;
    auto count = [&](std::vector<u32> &arr) {
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v); u32 a[kRegs];
            if (tord) tile_count<F32>(st, m, v, a, pass);
            else bucket_count<F32>(s, T, m, q, v, a, pass);
            for (int j = 0; j < kRegs; j++) arr[(size_t)q * kRegs + j] = a[j];
        }
    };
    // bucket path
    for (int q = 0; q < threads; q++) bucket_zero_thread(m, q, per);
    for (int b = 0; b < l.nbmax; b++) bucket_info_init(m, b);
    auto note = [&]() { for (int q = 0; q < threads; q++) { u64 v[kRegs]; V(q, v); presort_note(s, m, q, v); } };
    auto to_block = [&]() {
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v);
            tile_to_block_values(s, T, q, v);
            for (int j = 0; j < kRegs; j++) regs[(size_t)q * kRegs + j] = v[j];
        }
    };
    note();
    bool fast = s.S >= kRegs && !g_force_merge;
    bool direct = false;
    const bool ranked = tord && ranked_keys && !g_force_merge;
    std::vector<u32> arr((size_t)threads * kRegs), fin((size_t)threads * kRegs);
    const int32_t N = tile_items(s, T);
    auto attempt_counts = [&]() {
        pass = 0;
        count(arr);
        if ((m.flag[0] & 3u) != 0u) {
            g_recount_tiles++;
            for (int q = 0; q < threads; q++) bucket_zero_thread(m, q, per);
            pass = 1;
            m.flag[0] = 0u;
            count(arr);
        }
    };
    if (fast && tord && !ranked) {
        for (int q = 0; q < threads; q++) { u64 v[kRegs]; V(q, v); tile_minmax(m, v); }
        for (int q = 0; q < threads; q++) { u64 v[kRegs]; V(q, v); presort_check(s, T, m, q, threads, v, true); }
        direct = (m.flag[0] & 4u) == 0u;
        if (!direct && tile_many_ties(m, N)) {
            tord = false;
            to_block();
            for (int b = 0; b < l.nbmax; b++) bucket_info_init(m, b);
            note();
        }
    }
    if (fast && tord && !direct && !ranked) {
        attempt_counts();
        if ((m.flag[0] & 1u) != 0u) {
            tord = false;
            pass = 0;
            to_block();
            for (int q = 0; q < threads; q++) bucket_zero_thread(m, q, per);
            for (int b = 0; b < l.nbmax; b++) bucket_info_init(m, b);
            note();
        }
    }
    if (!tord && compact_tile(s)) fast = false;   // block order needs cap counters
    if (fast && !tord) {
        for (int q = 0; q < threads; q++) { u64 v[kRegs]; V(q, v); bucket_minmax(m, v); }
        for (int q = 0; q < threads; q++) { u64 v[kRegs]; V(q, v); presort_check(s, T, m, q, threads, v, false); }
        direct = (m.flag[0] & 4u) == 0u;
        if (!direct) attempt_counts();
    }
    if (fast) fast = (m.flag[0] & 1u) == 0u;
    // (key, slot) order; tile-order placement writes only the slots, whose
    // keys come from the loaded values
    std::vector<u32> slotkey((size_t)s.cap, 0u);
    auto tkey = [&](int u) {
        if (tord) {
            const u32 sl = m.sslot[u];
            return ((u64)slotkey[sl] << 32) | sl;
        }
        return ((u64)m.skey[u] << 32) | m.sslot[u];
    };
    auto check_sorted = [&]() {
        if (tord) {
            for (size_t e = 0; e < regs.size(); e++)
                if (sv_valid(regs[e])) slotkey[tv_slot(regs[e])] = tv_key(regs[e]);
            for (int u = 1; u < N; u++)
                if (tkey(u - 1) >= tkey(u)) return -13;
        } else {
            for (int b = 0; b < T.NB; b++) {
                const int len = block_len(s, T, b);
                for (int u = 1; u < len; u++)
                    if (tkey((b << s.logS) + u - 1) >= tkey((b << s.logS) + u)) return -12;
            }
        }
        return 0;
    };
    if (fast && ranked) {
        g_ranked_tiles++;
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v);
            u32 f[kRegs];
            for (int j = 0; j < kRegs; j++) f[j] = tv_key(v[j]) ^ 0x80000000u;
            tile_place(m, v, f);
        }
        const int rc = check_sorted();
        if (rc) return rc;
        g_fast_tiles++;
    } else if (fast && direct) {
        g_presorted_tiles++;
        for (int q = 0; q < threads; q++) { u64 v[kRegs]; V(q, v); presort_place(s, m, v, tord); }
        const int rc = check_sorted();
        if (rc) return rc;
        g_fast_tiles++;
    } else if (fast) {
        const int G = tord ? threads : s.S / kRegs;
        std::vector<u32> tot(threads);
        std::vector<std::vector<u32>> cl(threads, std::vector<u32>(kRegs));
        for (int q = 0; q < threads; q++) {
            u32 c[kRegs];
            tot[q] = bucket_scan_local(m, q, c, per);
            for (int j = 0; j < kRegs; j++) cl[q][j] = c[j];
        }
        for (int q = 0; q < threads; q++) {
            u32 excl = 0;
            for (int r = q & ~(G - 1); r < q; r++) excl += tot[r];
            u32 c[kRegs];
            for (int j = 0; j < kRegs; j++) c[j] = cl[q][j];
            bucket_scan_store(m, q, excl, c, per);
        }
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v); u32 a[kRegs];
            for (int j = 0; j < kRegs; j++) a[j] = arr[(size_t)q * kRegs + j];
            if (tord) tile_scatter(m, v, a, q, N);
            else bucket_scatter<F32>(s, T, m, q, v, a, pass);
        }
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v); u32 f[kRegs], a[kRegs];
            for (int j = 0; j < kRegs; j++) a[j] = arr[(size_t)q * kRegs + j];
            if (tord) tile_rank(st, m, v, N, f, a);
            else bucket_rank<F32>(s, T, m, q, v, f, pass);
            for (int j = 0; j < kRegs; j++) fin[(size_t)q * kRegs + j] = f[j];
        }
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v); u32 f[kRegs];
            for (int j = 0; j < kRegs; j++) f[j] = fin[(size_t)q * kRegs + j];
            if (tord) tile_place(m, v, f);
            else bucket_place(s, m, v, f);
        }
        const int rc = check_sorted();
        if (rc) return rc;
        g_fast_tiles++;
    } else {
        for (int q = 0; q < threads; q++) {
            u64 v[kRegs]; V(q, v);
            if (tord) tile_to_block_values(s, T, q, v);
            sort_regs(v);
            for (int j = 0; j < kRegs; j++) regs[(size_t)q * kRegs + j] = v[j];
        }
        for (int w = kRegs; w < s.S; w *= 2) {
            memcpy(m.mbuf, regs.data(), sizeof(u64) * regs.size());
            for (int q = 0; q < threads; q++) {
                u64 out[kRegs];
                merge_level(m.mbuf, w, q, out);
                for (int j = 0; j < kRegs; j++) tmp[(size_t)q * kRegs + j] = out[j];
            }
            regs.swap(tmp);
        }
        for (int b = 0; b < T.NB; b++) {
            const int len = block_len(s, T, b);
            for (int u = 1; u < len; u++)
                if (regs[(b << s.logS) + u - 1] >= regs[(b << s.logS) + u]) return -10;
        }
        for (int u = 0; u < (int)regs.size(); u++)
            if (sv_valid(regs[u])) put_block_value(s, m, u, regs[u]);
        g_slow_tiles++;
    }
    // the pair orders overwrite the bucket scratch: poison it first
    memset(m.M, 0xA5, (size_t)(l.pos - l.M) + 4 * (size_t)s.Pmax * s.Pstride);
    if (fast && tord) {
        g_tile_order_tiles++;
        std::vector<u32> w((size_t)threads * kRegs);
        std::vector<u64> cnt(threads);
        for (int q = 0; q < threads; q++) {
            u32 ww[kRegs];
            cnt[q] = tile_label_counts(s, m, q, N, ww);
            for (int j = 0; j < kRegs; j++) w[(size_t)q * kRegs + j] = ww[j];
        }
        if (s.C > 1)
            for (int q = 0; q < threads; q++) tail_table_zero(s, T, m, q, threads);
        u64 ex = 0;
        for (int q = 0; q < threads; q++) {
            u32 ww[kRegs];
            for (int j = 0; j < kRegs; j++) ww[j] = w[(size_t)q * kRegs + j];
            tile_positions(s, T, m, ex, ww, xo, yo, argmed);
            ex += cnt[q];
        }
        for (int q = 0; q < threads; q++) tile_mpad(s, T, m, q, threads);
    } else {
        for (int q = 0; q < threads; q++) tail_pair_pad(s, T, m, q, threads);
        for (int q = 0; q < threads; q++) tail_pair_merge(s, T, m, q, threads, xo, yo, argmed);
        for (int q = 0; q < threads; q++) tail_first_medians(s, T, m, q, threads);
    }
    if (s.C > 1) {
        if (!(fast && tord)) {
            for (int q = 0; q < threads; q++) tail_table_zero(s, T, m, q, threads);
            for (int q = 0; q < threads; q++) tail_table_hist(s, T, m, q, threads);
        }
        for (int q = 0; q < threads; q++) tail_table_columns(s, T, m, q, threads);
        for (int q = 0; q < threads; q++) tail_table_rows(s, T, m, q, threads);
    }
    for (int q = 0; q < threads; q++)
        if (tail_walk(s, T, m, q, threads)) return -11;
    for (int q = 0; q < threads; q++) tail_output(s, T, m, q, threads, xo, yo, argmed);
    return 0;
}

extern "C" int emu_median_filter(const void *x, int64_t n, int32_t k, int is_f32, int threads,
                                 void *y, int32_t *argmed, int32_t *out_pmax)
{
    if (k < 3 || (k & 1) == 0 || n < k) return -1;
    Shape s;
    if (make_shape(n, k, threads, &s) != 0) return -2;
    Layout l;
    make_layout(s, &l);
    if (l.total < 0) return -3;
    if (out_pmax) *out_pmax = s.Pmax;
    std::vector<unsigned char> lds((size_t)l.total + 64);
    for (int64_t t = 0; t < s.ntiles; t++) {
        const int rc = is_f32 ? run_tile<true>(s, l, t, threads, (const u32 *)x, (const u32 *)x, (u32 *)y, argmed, lds)
                              : run_tile<false>(s, l, t, threads, (const u32 *)x, (const u32 *)x, (u32 *)y, argmed, lds);
        if (rc != 0) return rc;
    }
    return 0;
}

// Ranks of the span items at xt by (key, offset), the kernels' rank_items
// with each phase as one sweep over the threads (barriers between sweeps):
// bucket sort, or the merge sort for a crowded bucket.  Checks that the
// ranks are a permutation.  Returns 0, or -20.
static int emu_rank_items(const u64 *xt, int32_t span, int threads, bool f64, std::vector<u32> &rank)
{
    const int cap = threads * kRegs;
    std::vector<u64> kr(cap), kt(cap), K(cap);
    std::vector<u32> sr(cap), st(cap), C((size_t)cap / 2), arr(cap), fin(cap), cpre(cap), tot(threads);
    std::vector<u16> S(cap);
    int lognb = 0;
    while ((1 << lognb) < cap) lognb++;
    u64 lo = ~0ull, hi = 0ull;
    for (int q = 0; q < threads; q++) {
        u64 kv[kRegs], l, h;
        u32 sv[kRegs];
        if (f64) rank64_load<true>(xt, span, q, kv, sv);
        else rank64_load<false>(xt, span, q, kv, sv);
        rank64_range(span, kv, sv, l, h);
        lo = l < lo ? l : lo;
        hi = h > hi ? h : hi;
        for (int j = 0; j < kRegs; j++) {
            kr[(size_t)q * kRegs + j] = kv[j];
            sr[(size_t)q * kRegs + j] = sv[j];
        }
    }
    auto regs = [&](int q, u64 (&kv)[kRegs], u32 (&sv)[kRegs]) {
        for (int j = 0; j < kRegs; j++) {
            kv[j] = kr[(size_t)q * kRegs + j];
            sv[j] = sr[(size_t)q * kRegs + j];
        }
    };
    const u32 sh = rank64_shift(lo, hi, lognb);
    bool full = false;
    for (int q = 0; q < threads; q++) {
        u64 kv[kRegs];
        u32 sv[kRegs], a[kRegs];
        regs(q, kv, sv);
        if (rank64_count(span, kv, sv, lo, sh, C.data(), a)) full = true;
        for (int j = 0; j < kRegs; j++) arr[(size_t)q * kRegs + j] = a[j];
    }
    rank.assign(cap, 0xFFFFFFFFu);
    if (!full && !g_force_merge) {
        for (int q = 0; q < threads; q++) {
            u32 c[kRegs];
            tot[q] = rank64_scan_local(C.data(), q, c);
            for (int j = 0; j < kRegs; j++) cpre[(size_t)q * kRegs + j] = c[j];
        }
        u32 excl = 0;
        for (int q = 0; q < threads; q++) {
            u32 c[kRegs];
            for (int j = 0; j < kRegs; j++) c[j] = cpre[(size_t)q * kRegs + j];
            rank64_scan_store(C.data(), q, excl, c);
            excl += tot[q];
        }
        std::fill(K.begin(), K.end(), 0xA5A5A5A5A5A5A5A5ull);
        for (int q = 0; q < threads; q++) {
            u64 kv[kRegs];
            u32 sv[kRegs], a[kRegs];
            regs(q, kv, sv);
            for (int j = 0; j < kRegs; j++) a[j] = arr[(size_t)q * kRegs + j];
            rank64_scatter(span, kv, sv, lo, sh, C.data(), a, K.data(), S.data());
        }
        for (int q = 0; q < threads; q++) {
            u64 kv[kRegs];
            u32 sv[kRegs], f[kRegs];
            regs(q, kv, sv);
            rank64_bucket_rank(span, kv, sv, lo, sh, C.data(), (u32)cap, K.data(), S.data(), f);
            for (int j = 0; j < kRegs; j++) fin[(size_t)q * kRegs + j] = f[j];
        }
        for (int q = 0; q < threads; q++) {
            u64 kv[kRegs];
            u32 sv[kRegs], f[kRegs];
            regs(q, kv, sv);
            for (int j = 0; j < kRegs; j++) f[j] = fin[(size_t)q * kRegs + j];
            rank64_place(span, sv, f, rank.data());
        }
        g_rank_bucket_tiles++;
    } else {
        for (int q = 0; q < threads; q++) {
            u64 kv[kRegs];
            u32 sv[kRegs];
            regs(q, kv, sv);
            sort_regs_ks(kv, sv);
            for (int j = 0; j < kRegs; j++) {
                kr[(size_t)q * kRegs + j] = kv[j];
                sr[(size_t)q * kRegs + j] = sv[j];
            }
        }
        for (int w = kRegs; w < cap; w *= 2) {
            K = kr;
            for (int i = 0; i < cap; i++) S[i] = (u16)sr[i];
            for (int q = 0; q < threads; q++) {
                u64 ko[kRegs];
                u32 so[kRegs];
                merge_level_ks(K.data(), S.data(), w, q, ko, so);
                for (int j = 0; j < kRegs; j++) {
                    kt[(size_t)q * kRegs + j] = ko[j];
                    st[(size_t)q * kRegs + j] = so[j];
                }
            }
            kr.swap(kt);
            sr.swap(st);
        }
        for (int q = 0; q < threads; q++) {
            u32 sv[kRegs];
            for (int j = 0; j < kRegs; j++) sv[j] = sr[(size_t)q * kRegs + j];
            rank64_ranks(span, q, sv, rank.data());
        }
        g_rank_merge_tiles++;
    }
    std::vector<char> seen(span, 0);
    for (int32_t i = 0; i < span; i++) {
        if (rank[i] >= (u32)span || seen[rank[i]]) return -20;
        seen[rank[i]] = 1;
    }
    return 0;
}

// 64-bit signals: each tile's ranks (emu_rank_items), then the 32-bit tiles
// on them: 512-thread tiles read their slots' ranks from the rank array
// (as from their LDS), 1024-thread tiles read the pre-pass keys at
// keys + t*k.  The medians are copied from the 64-bit x.
extern "C" int emu_median_filter64(const void *x, int64_t n, int32_t k, int is_f64, int threads,
                                   void *y, int32_t *argmed)
{
    if (k < 3 || (k & 1) == 0 || n < k) return -1;
    Shape s;
    if (make_shape(n, k, threads, &s) != 0) return -2;
    Layout l;
    make_layout(s, &l);
    if (l.total < 0) return -3;
    const int64_t stride = rank64_stride(s);
    std::vector<u32> keys((size_t)(s.ntiles * stride), 0xA5A5A5A5u), rank;
    for (int64_t t = 0; t < s.ntiles; t++) {
        const Tile T = make_tile(s, t);
        const int32_t span = tile_items(s, T);
        const int rc = emu_rank_items((const u64 *)x + T.e0, span, threads, is_f64 != 0, rank);
        if (rc != 0) return rc;
        for (int32_t i = 0; i < span; i++) keys[(size_t)(t * stride + i)] = rank[i];
    }
    std::vector<unsigned char> lds((size_t)l.total + 64);
    for (int64_t t = 0; t < s.ntiles; t++) {
        const int rc = threads == 512
                           ? run_tile<false>(s, l, t, threads, nullptr, (const u64 *)x, (u64 *)y, argmed, lds, true,
                                             keys.data() + t * stride)
                           : run_tile<false>(s, l, t, threads, keys.data() + t * k, (const u64 *)x, (u64 *)y, argmed,
                                             lds, true);
        if (rc != 0) return rc;
    }
    return 0;
}

// The pair pre-pass of 64-bit signals on the global path (k > 4095): for
// every pair tile of the shape (threads = 2S / kRegs, one pair per tile),
// chunks of 8192 items ranked (emu_rank_items, 1024 threads), written in
// sorted (key, offset) order, merged level by level in output tiles of 8192
// staged as the kernel stages them in LDS (merge_split_ko, merge_local_ko
// for each of the 1024 threads), then
// keys[t * stride + offset] = rank.
extern "C" int emu_rank_pairs64(const void *x, int64_t n, int32_t k, int is_f64, uint32_t *keys, int64_t *out_stride,
                                int64_t *out_tiles)
{
    int32_t S = 1;
    while (S < k) S <<= 1;
    Shape s;
    if (make_shape(n, k, 2 * S / kRegs, &s) != 0) return -2;
    const int64_t stride = rank64_stride(s);
    *out_stride = stride;
    *out_tiles = s.ntiles;
    if (!keys) return 0;
    const int32_t C = 1024 * kRegs;
    std::vector<u64> K0(2 * (size_t)k), K1(2 * (size_t)k);
    std::vector<u32> O0(2 * (size_t)k), O1(2 * (size_t)k), rank;
    for (int64_t t = 0; t < s.ntiles; t++) {
        const Tile T = make_tile(s, t);
        const int32_t span = tile_items(s, T);
        const u64 *xt = (const u64 *)x + T.e0;
        for (int32_t c0 = 0; c0 < span; c0 += C) {
            const int32_t len = span - c0 < C ? span - c0 : C;
            const int rc = emu_rank_items(xt + c0, len, 1024, is_f64 != 0, rank);
            if (rc != 0) return rc;
            for (int32_t i = 0; i < len; i++) {
                K0[c0 + rank[i]] = is_f64 ? key_of_f64(xt[c0 + i]) : key_of_i64(xt[c0 + i]);
                O0[c0 + rank[i]] = (u32)(c0 + i);
            }
        }
        u64 *Kin = K0.data(), *Kout = K1.data();
        u32 *Oin = O0.data(), *Oout = O1.data();
        std::vector<u64> LK(C);
        std::vector<u32> LO(C);
        for (int32_t w = C; w < span; w <<= 1) {
            for (int32_t ob = 0; ob < span; ob += C) {
                int32_t s0, lenA, lenB;
                merge_runs(span, w, ob, s0, lenA, lenB);
                const int32_t d0 = ob - s0;
                const int32_t d1 = d0 + C < lenA + lenB ? d0 + C : lenA + lenB;
                const int32_t a0 = merge_split_ko(Kin + s0, Oin + s0, lenA, Kin + s0 + w, Oin + s0 + w, lenB, d0);
                const int32_t a1 = merge_split_ko(Kin + s0, Oin + s0, lenA, Kin + s0 + w, Oin + s0 + w, lenB, d1);
                const int32_t na = a1 - a0, b0 = d0 - a0, nb = (d1 - d0) - na;
                if (na < 0 || nb < 0 || na + nb > C) return -21;
                std::fill(LK.begin(), LK.end(), 0xA5A5A5A5A5A5A5A5ull);
                for (int32_t i = 0; i < na + nb; i++) {
                    const int32_t src = i < na ? s0 + a0 + i : s0 + w + b0 + (i - na);
                    LK[i] = Kin[src];
                    LO[i] = Oin[src];
                }
                for (int q = 0; q < 1024; q++) {
                    u64 kv[kRegs];
                    u32 ov[kRegs];
                    const int32_t cnt = merge_local_ko(LK.data(), LO.data(), na, nb, q * kRegs, kv, ov);
                    for (int j = 0; j < cnt; j++) {
                        Kout[ob + q * kRegs + j] = kv[j];
                        Oout[ob + q * kRegs + j] = ov[j];
                    }
                }
            }
            std::swap(Kin, Kout);
            std::swap(Oin, Oout);
        }
        for (int32_t p = 0; p < span; p++) keys[t * stride + Oin[p]] = (u32)p;
    }
    return 0;
}

// Tiles [t0, t1) of a signal of length n (a check of the index arithmetic
// near the end of long signals): x, y and argmed point at element `base` of
// the signal, input and outputs, so that only x[base ..], y[base ..] and
// argmed[base ..] need to exist.
extern "C" int emu_tile_range(const float *x_at_base, int64_t base, int64_t n, int32_t k, int threads,
                              int64_t t0, int64_t t1, float *y_at_base, int32_t *argmed_at_base)
{
    Shape s;
    if (make_shape(n, k, threads, &s) != 0) return -2;
    Layout l;
    make_layout(s, &l);
    if (l.total < 0) return -3;
    if (t1 > s.ntiles) t1 = s.ntiles;
    std::vector<unsigned char> lds((size_t)l.total + 64);
    const u32 *x = (const u32 *)x_at_base - base;
    u32 *y = (u32 *)y_at_base - base;
    int32_t *am = argmed_at_base - base;
    for (int64_t t = t0; t < t1; t++) {
        const int rc = run_tile<true>(s, l, t, threads, x, x, y, am, lds);
        if (rc != 0) return rc;
    }
    return 0;
}

extern "C" int64_t emu_ntiles(int64_t n, int32_t k, int threads)
{
    Shape s;
    if (make_shape(n, k, threads, &s) != 0) return -1;
    return s.ntiles;
}

// The order-preserving keys of the tile phases, element by element: kind 0
// float32, 1 int32 (32-bit keys into out32), 2 float64, 3 int64 (64-bit keys
// into out64).
extern "C" void emu_keys(const void *x, int64_t n, int kind, uint32_t *out32, uint64_t *out64)
{
    for (int64_t i = 0; i < n; i++) {
        if (kind == 0) out32[i] = key_of_f32(((const u32 *)x)[i]);
        else if (kind == 1) out32[i] = key_of_i32(((const u32 *)x)[i]);
        else if (kind == 2) out64[i] = key_of_f64(((const u64 *)x)[i]);
        else out64[i] = key_of_i64(((const u64 *)x)[i]);
    }
}

// The kernels' exact division by a per-launch reciprocal (udiv16 with
// recip32) against the hardware divide: every dividend for divisors up to
// 300, and the dividends next to each multiple plus a stride for every
// divisor below 2^16.  Returns the number of mismatches.
extern "C" long emu_check_udiv16(void)
{
    long bad = 0;
    for (uint32_t d = 1; d < 65536u; d++) {
        const uint32_t r = recip32((int32_t)d);
        for (uint32_t q = 0; q * d < 65536u; q++)
            for (int e = -1; e <= 1; e++) {
                const int64_t a = (int64_t)q * d + e;
                if (a >= 0 && a < 65536 && udiv16((uint32_t)a, r) != (uint32_t)a / d) bad++;
            }
        for (uint32_t a = 0; a < 65536u; a += (d < 300u ? 1u : 977u))
            if (udiv16(a, r) != a / d) bad++;
    }
    return bad;
}

// The tail of the one-pair tiles (k > 4095) that keep their merged order in
// global memory: the pair's merged order and position maps made here by a
// plain sort of (key, block, t), then the kernels' coarse count table, walk
// and output phases, each as one sweep over the threads.  lds: the
// workgroup's dynamic LDS bytes, which set the walk chunks.  Returns 0, or
// a negative code.
extern "C" int emu_global_tail(const void *x, int64_t n, int32_t k, int is_f32, int32_t lds, void *y,
                               int32_t *argmed, int32_t *out_L)
{
    if (k < 3 || (k & 1) == 0 || n < 2 * (int64_t)k) return -1;
    int32_t S = 1;
    while (S < k) S <<= 1;
    Shape s;
    if (make_shape(n, k, 2 * S / kRegs, &s) != 0) return -2;
    if (s.Pmax != 1) return -3;
    global_chunks(&s, lds);
    if (out_L) *out_L = s.L;
    const int32_t G = gcols(s);
    if (4 * G * (s.C + kGcolGroups) > lds || 2 * s.Mstride > lds) return -4;
    const u32 *xu = (const u32 *)x;
    std::vector<u16> M((size_t)s.Mstride);
    std::vector<u32> pos((size_t)s.Pstride + 1);
    std::vector<u16> stage((size_t)k);
    std::vector<u32> tbuf((size_t)lds / 4);
    for (int64_t t = 0; t < s.ntiles; t++) {
        const Tile T = make_tile(s, t);
        if (T.P != 1) return -5;
        const int32_t lenB = block_len(s, T, 1), N = k + lenB;
        std::vector<u64> v((size_t)N);
        for (int32_t i = 0; i < N; i++) {
            const int32_t b = i < k ? 0 : 1, tt = i < k ? i : i - k;
            const u32 raw = xu[T.e0 + i];
            const u32 key = is_f32 ? key_of_f32(raw) : key_of_i32(raw);
            v[i] = ((u64)key << 32) | ((u64)b << 16) | (u64)tt;
        }
        std::sort(v.begin(), v.end());
        for (int32_t r = 0; r < s.Mstride; r++) M[mslot(r)] = (u16)kMPad;
        for (int32_t r = 0; r < N; r++) {
            const u32 b = (u32)(v[r] >> 16) & 1u, tt = (u32)v[r] & 0xFFFFu;
            M[mslot(r)] = (u16)((b << 15) | tt);
            if (b) pos[tt] = (pos[tt] & 0xFFFFu) | ((u32)r << 16);
            else pos[tt] = (pos[tt] & 0xFFFF0000u) | (u32)r;
        }
        TileMem m = {};
        m.M = M.data();
        m.pos = pos.data();
        m.stage = stage.data();
        u32 *tb = tbuf.data(), *gt = tb + s.C * G;
        gtab_zero(s, tb, 0, 1);
        gtab_hist(s, T, m, tb, 0, 1);
        gtab_col_sums(s, tb, gt, 0, 1);
        gtab_col_apply(s, tb, gt, 0, 1);
        if (s.C > kGchunkMax) return -6;
        std::vector<u32> info((size_t)s.C);
        gtab_rows(s, tb, info.data(), 0, 1);
        const int bad = lds > 65536 ? gtail_walk<8, u32>(s, T, m, info.data(), 0, 1, xu, (u32 *)y, argmed)
                                    : gtail_walk<2, u32>(s, T, m, info.data(), 0, 1, xu, (u32 *)y, argmed);
        if (bad) return -11;
        gtail_output<u32>(s, T, m, 0, 1, xu, (u32 *)y, argmed);
    }
    return 0;
}
