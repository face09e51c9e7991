// Host-side run of the tile phases (paper_1406_1717_amd/csrc/mf_tile.h),
// one work item after another, in the order the GPU kernel runs them.
// Test-only: it checks the tile logic (indexing, tables, walk) on the CPU,
// with bounds checks on every tile buffer.  It is not a fallback of the
// library and nothing in the product loads it.
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <vector>

#include "../../paper_1406_1717_amd/csrc/mf_tile.h"

using namespace mf;

template <bool F32>
static int run_tile(const Shape &s, const Layout &l, int64_t t, int threads,
                    const u32 *x, u32 *y, int32_t *argmed, std::vector<unsigned char> &lds)
{
    const Tile T = make_tile(s, t);
    // poison the tile memory so that reads of unwritten data show up
    memset(lds.data(), 0xA5, lds.size());
    TileMem m = tile_mem(lds.data(), l);

    for (int b = 0; b < T.NB; b++)
        for (int u = 0; u < block_len(s, T, b); u++) load_item(s, T, m, x, b, u);

    std::vector<u64> regs((size_t)threads * kRegs), tmp((size_t)threads * kRegs);
    for (int q = 0; q < threads; q++) {
        u64 v[kRegs];
        for (int j = 0; j < kRegs; j++) v[j] = sort_value<F32>(s, T, m, q * kRegs + j);
        sort_regs(v);
        for (int j = 0; j < kRegs; j++) regs[(size_t)q * kRegs + j] = v[j];
    }
    for (int w = kRegs; w < s.S; w *= 2) {
        memcpy(m.srt, regs.data(), sizeof(u64) * regs.size());
        for (int q = 0; q < threads; q++) {
            u64 out[kRegs];
            merge_level(m.srt, w, q, out);
            for (int j = 0; j < kRegs; j++) tmp[(size_t)q * kRegs + j] = out[j];
        }
        regs.swap(tmp);
    }
    memcpy(m.srt, regs.data(), sizeof(u64) * regs.size());

    // sortedness check of every block
    for (int b = 0; b < T.NB; b++) {
        const int len = block_len(s, T, b);
        for (int u = 1; u < len; u++)
            if (m.srt[(b << s.logS) + u - 1] >= m.srt[(b << s.logS) + u]) return -10;
    }

    const int ipp = merge_items_per_pair(s);
    for (int p = 0; p < T.P; p++)
        for (int g = 0; g < ipp; g++) pair_merge_item(s, T, m, p, g);
    if (T.j0 == 1) output_first(s, T, m, y, argmed);

    for (int p = 0; p < T.P; p++)
        for (int w = 0; w < s.Wn; w++) table_init_item(s, m, p, w);
    for (int p = 0; p < T.P; p++)
        for (int i = 0; i < block_len(s, T, p + 1); i++) table_flip_item(s, T, m, p, i);
    for (int p = 0; p < T.P; p++)
        for (int w = 0; w < s.Wn; w++) table_prefix_item(s, T, m, p, w);
    for (int p = 0; p < T.P; p++)
        for (int c = 0; c < pair_chunks(s, T, p); c++) table_count_item(s, m, p, c);
    for (int p = 0; p < T.P; p++)
        for (int c = 0; c < pair_chunks(s, T, p); c++)
            if (walk_item(s, T, m, p, c) != 0) return -11;
    const int64_t no = tile_outputs(s, T);
    for (int64_t u = 0; u < no; u++) output_item(s, T, m, u, y, argmed);
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
        const int rc = is_f32 ? run_tile<true>(s, l, t, threads, (const u32 *)x, (u32 *)y, argmed, lds)
                              : run_tile<false>(s, l, t, threads, (const u32 *)x, (u32 *)y, argmed, lds);
        if (rc != 0) return rc;
    }
    return 0;
}
