// HIP kernels of the sorting-based median filter (arXiv:1406.1717) for
// gfx950.  The per-tile phases live in mf_tile.h; this file runs them:
//
//   k_tile_lds<NT>   k <= 4096: one workgroup per tile, every tile buffer
//                    in LDS (NT = 256 threads for blocks up to 2048 slots,
//                    512 above).
//   k_tile_global    4096 < k <= 32767: one pair per tile, the first sort
//                    levels in LDS and the tile buffers in a per-workgroup
//                    global workspace; workgroups loop over tiles.
//   k_identity       k = 1.
//   k_backward       deterministic scatter of the upstream gradient.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_tile.h"
#include "mf_launch.h"

namespace mf {

// ------------------------------------------------------------------ helpers

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

// Resolves work unit uidx of a launch into its signal and tile.
struct Resolved {
    const u32 *x;
    u32 *y;
    int32_t *argmed;
    int64_t n;
    int32_t k;
    int64_t tile;
};

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
        d.x_off += row * d.n;
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
// filled m.xv and m.srt.  NT threads, barriers between phases.
template <int NT>
__device__ void tile_tail(const Shape &s, const Tile &T, const TileMem &m, const Resolved &d,
                          int *err)
{
    const int tid = threadIdx.x;
    const int ipp = merge_items_per_pair(s);
    for (int it = tid; it < T.P * ipp; it += NT) pair_merge_item(s, T, m, it / ipp, it % ipp);
    if (T.j0 == 1 && tid == 0) output_first(s, T, m, (u32 *)d.y, d.argmed);
    __syncthreads();

    for (int it = tid; it < T.P * s.Wn; it += NT) table_init_item(s, m, it / s.Wn, it % s.Wn);
    __syncthreads();
    for (int it = tid; it < T.P * s.k; it += NT) {
        const int p = it / s.k, i = it - p * s.k;
        if (i < block_len(s, T, p + 1)) table_flip_item(s, T, m, p, i);
    }
    __syncthreads();
    for (int it = tid; it < T.P * s.Wn; it += NT) table_prefix_item(s, T, m, it / s.Wn, it % s.Wn);
    __syncthreads();
    for (int it = tid; it < T.P * s.C; it += NT) {
        const int p = it / s.C, c = it - p * s.C;
        if (c < pair_chunks(s, T, p)) table_count_item(s, m, p, c);
    }
    __syncthreads();

    for (int it = tid; it < T.P * s.C; it += NT) {
        const int p = it / s.C, c = it - p * s.C;
        if (c < pair_chunks(s, T, p))
            if (walk_item(s, T, m, p, c) != 0) atomicOr(err, 1);
    }
    __syncthreads();

    const int64_t no = tile_outputs(s, T);
    for (int64_t u = tid; u < no; u += NT) output_item(s, T, m, u, (u32 *)d.y, d.argmed);
}

// ------------------------------------------------------------------ LDS path

template <int NT, bool F32>
__global__ __launch_bounds__(NT) void k_tile_lds(Launch L, int *err)
{
    extern __shared__ __align__(16) unsigned char lds[];
    const Resolved d = unit_of(L, blockIdx.x);
    const int64_t tile = d.tile;
    const int tid = threadIdx.x;

    Shape s;
    make_shape(d.n, d.k, NT, &s);
    Layout l;
    make_layout(s, &l);
    const TileMem m = tile_mem(lds, l);
    const Tile T = make_tile(s, tile);
    const u32 *x = d.x;

    // 1. load (coalesced within each block)
    for (int b = 0; b < T.NB; b++) {
        const int len = block_len(s, T, b);
        for (int t = tid; t < len; t += NT) load_item(s, T, m, x, b, t);
    }
    __syncthreads();

    // 2. sort: registers, then merge-path levels up to the block slot size
    u64 v[kRegs];
#pragma unroll
    for (int j = 0; j < kRegs; j++) v[j] = sort_value<F32>(s, T, m, tid * kRegs + j);
    sort_regs(v);
    for (int w = kRegs; w < s.S; w <<= 1) {
        store_regs(m.srt + tid * kRegs, v);
        __syncthreads();
        merge_level(m.srt, w, tid, v);
        __syncthreads();
    }
    store_regs(m.srt + tid * kRegs, v);
    __syncthreads();

    tile_tail<NT>(s, T, m, d, err);
}

// ------------------------------------------------------------------ global path

struct GLayout {
    int64_t xv, srt, srt2, M, pos, words, pc, stage, total;
};

__host__ __device__ inline void make_glayout(const Shape &s, GLayout *g)
{
    int64_t off = 0;
    g->xv = off;   off += 4ll * s.cap;
    g->srt = off;  off += 8ll * s.cap;
    g->srt2 = off; off += 8ll * s.cap;
    g->M = off;    off += 2ll * s.Pmax * s.Mstride;
    off = (off + 255) & ~255ll;
    g->pos = off;  off += 4ll * s.Pmax * s.k;
    off = (off + 255) & ~255ll;
    g->total = off;
    int64_t a = g->srt2;
    g->words = a;  a += 8ll * s.Pmax * s.C * s.Wn;
    g->pc = a;     a += 2ll * s.Pmax * s.C * (s.Wn + 1);
    a = (a + 15) & ~15ll;
    g->stage = a;
}

__host__ __device__ inline int global_shape(int64_t n, int32_t k, Shape *s)
{
    int32_t S = 1;
    while (S < k) S <<= 1;
    return make_shape(n, k, 2 * S / kRegs, s);
}

template <bool F32>
__global__ __launch_bounds__(kGlobalThreads) void k_tile_global(Launch L, unsigned char *ws,
                                                                int64_t ws_stride, int *err)
{
    extern __shared__ __align__(16) unsigned char lds[];
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
        TileMem m;
        m.xv = (u32 *)(base + g.xv);
        m.srt = (u64 *)(base + g.srt);
        m.M = (u16 *)(base + g.M);
        m.pos = (u32 *)(base + g.pos);
        m.words = (u64 *)(base + g.words);
        m.pc = (u16 *)(base + g.pc);
        m.stage = (u16 *)(base + g.stage);
        u64 *srt2 = (u64 *)(base + g.srt2);
        const Tile T = make_tile(s, tile);
        const u32 *x = d.x;

        __syncthreads();   // the previous tile is done with the workspace
        for (int b = 0; b < T.NB; b++) {
            const int len = block_len(s, T, b);
            for (int t = tid; t < len; t += kGlobalThreads) load_item(s, T, m, x, b, t);
        }
        __syncthreads();

        // sort chunks of `chunk` slots in LDS; blocks larger than a chunk
        // get their last merge level from srt2 into srt
        const bool glevel = s.S > chunk;
        u64 *dst0 = glevel ? srt2 : m.srt;
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
            store_regs(dst0 + (int64_t)vt * kRegs, v);
        }
        __syncthreads();
        if (glevel) {
            const int vthreads = s.cap / kRegs;
            for (int vt = tid; vt < vthreads; vt += kGlobalThreads) {
                u64 v[kRegs];
                merge_level(srt2, chunk, vt, v);
                store_regs(m.srt + (int64_t)vt * kRegs, v);
            }
            __syncthreads();
        }
        tile_tail<kGlobalThreads>(s, T, m, d, err);
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
// increasing order; lanes that hit the same target take turns in lane
// order (lowest lane first, settled by an LDS atomic minimum), so every
// accumulator receives its terms in increasing o.
__global__ __launch_bounds__(kBwdThreads) void k_backward(BwdLaunch L)
{
    __shared__ double acc[kBwdThreads / 64][kBwdTargetsPerWave];
    __shared__ int owner[kBwdThreads / 64][kBwdTargetsPerWave];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    double *A = acc[wave];
    int *own = owner[wave];

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
            const float *grad_y;
            const int32_t *argmed;
            float *grad_x;
            int64_t n;
            int32_t k;
        } d = {L.grad_y + sd.y_off, L.argmed + sd.y_off, L.grad_x + sd.x_off, sd.n, sd.k};
        const int64_t nout = d.n - d.k + 1;
        const int64_t j0 = tile * kBwdTargetsPerBlock + (int64_t)wave * kBwdTargetsPerWave;
        for (int t = lane; t < kBwdTargetsPerWave; t += 64) {
            A[t] = 0.0;
            own[t] = 64;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (j0 < d.n) {
            const int64_t olo = (j0 - d.k + 1) > 0 ? (j0 - d.k + 1) : 0;
            int64_t ohi = j0 + kBwdTargetsPerWave;
            if (ohi > nout) ohi = nout;
            for (int64_t b0 = olo; b0 < ohi; b0 += 64) {
                const int64_t o = b0 + lane;
                int tgt = -1;
                float g = 0.f;
                if (o < ohi) {
                    const int64_t j = d.argmed[o];
                    if (j >= j0 && j < j0 + kBwdTargetsPerWave) {
                        tgt = (int)(j - j0);
                        g = d.grad_y[o];
                    }
                }
                bool pend = tgt >= 0;
                // each round retires the lowest pending lane of every target,
                // so 64 rounds always suffice
                for (int round = 0; round < 64 && __ballot(pend) != 0ull; round++) {
                    if (pend) atomicMin(&own[tgt], lane);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    const bool win = pend && (__atomic_load_n(&own[tgt], __ATOMIC_RELAXED) == lane);
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                    if (win) {
                        A[tgt] += (double)g;
                        own[tgt] = 64;
                        pend = false;
                    }
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                }
            }
            for (int t = lane; t < kBwdTargetsPerWave; t += 64)
                if (j0 + t < d.n) d.grad_x[j0 + t] = (float)A[t];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ host side

Path path_for(int32_t k)
{
    if (k == 1) return PATH_IDENTITY;
    int32_t S = 1;
    while (S < k) S <<= 1;
    if (2 * S <= 256 * kRegs) return PATH_LDS256;
    if (2 * S <= 512 * kRegs) return PATH_LDS512;
    if (k <= 32767) return PATH_GLOBAL;
    return PATH_NONE;
}

int64_t tiles_for(Path p, int64_t n, int32_t k)
{
    Shape s;
    switch (p) {
    case PATH_IDENTITY: return (n + 65535) / 65536;
    case PATH_LDS256: make_shape(n, k, 256, &s); return s.ntiles;
    case PATH_LDS512: make_shape(n, k, 512, &s); return s.ntiles;
    case PATH_GLOBAL: global_shape(n, k, &s); return s.ntiles;
    default: return 0;
    }
}

int64_t lds_bytes_for(Path p, int32_t k)
{
    Shape s;
    Layout l;
    switch (p) {
    case PATH_LDS256: make_shape(1ll << 20, k, 256, &s); make_layout(s, &l); return l.total;
    case PATH_LDS512: make_shape(1ll << 20, k, 512, &s); make_layout(s, &l); return l.total;
    case PATH_GLOBAL: return 8ll * kGlobalThreads * kRegs;
    default: return 0;
    }
}

int64_t global_ws_stride(int32_t k)
{
    Shape s;
    global_shape(1ll << 30, k, &s);
    GLayout g;
    make_glayout(s, &g);
    return (g.total + 255) & ~255ll;
}

hipError_t prepare_kernels()
{
    hipError_t e = hipSuccess;
    const int big = 160 * 1024;
#define MF_ATTR(kern)                                                                        \
    if (e == hipSuccess)                                                                     \
        e = hipFuncSetAttribute((const void *)(kern), hipFuncAttributeMaxDynamicSharedMemorySize, big);
    MF_ATTR((k_tile_lds<256, true>))
    MF_ATTR((k_tile_lds<256, false>))
    MF_ATTR((k_tile_lds<512, true>))
    MF_ATTR((k_tile_lds<512, false>))
    MF_ATTR((k_tile_global<true>))
    MF_ATTR((k_tile_global<false>))
#undef MF_ATTR
    return e;
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
    case PATH_LDS256:
        if (f32) hipLaunchKernelGGL((k_tile_lds<256, true>), dim3((unsigned)L.nunits), dim3(256), lds_bytes, st, L, d_err);
        else     hipLaunchKernelGGL((k_tile_lds<256, false>), dim3((unsigned)L.nunits), dim3(256), lds_bytes, st, L, d_err);
        break;
    case PATH_LDS512:
        if (f32) hipLaunchKernelGGL((k_tile_lds<512, true>), dim3((unsigned)L.nunits), dim3(512), lds_bytes, st, L, d_err);
        else     hipLaunchKernelGGL((k_tile_lds<512, false>), dim3((unsigned)L.nunits), dim3(512), lds_bytes, st, L, d_err);
        break;
    case PATH_GLOBAL: {
        const int64_t grid = L.nunits < ws_slots ? L.nunits : ws_slots;
        if (f32) hipLaunchKernelGGL((k_tile_global<true>), dim3((unsigned)grid), dim3(kGlobalThreads), lds_bytes, st, L, ws, ws_stride, d_err);
        else     hipLaunchKernelGGL((k_tile_global<false>), dim3((unsigned)grid), dim3(kGlobalThreads), lds_bytes, st, L, ws, ws_stride, d_err);
        break;
    }
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t bwd_tiles_for(int64_t n) { return (n + kBwdTargetsPerBlock - 1) / kBwdTargetsPerBlock; }

hipError_t launch_backward(const BwdLaunch &L, hipStream_t st)
{
    if (L.nunits <= 0) return hipSuccess;
    const int64_t grid = L.nunits < (1ll << 20) ? L.nunits : (1ll << 20);
    hipLaunchKernelGGL(k_backward, dim3((unsigned)grid), dim3(kBwdThreads), 0, st, L);
    return hipGetLastError();
}

}  // namespace mf
