// Tile phases of the sorting-based median filter (arXiv:1406.1717).
//
// A tile is a run of consecutive block pairs of one signal.  With blocks of
// length k (Section 3; the signal's last block may be shorter), pair j has
// left block A = X_{j-1} and right block B = X_j and produces the outputs
// o = (j-1)k + i + 1 for steps i = 0 .. len(B)-1.  A tile of P pairs covers
// the P+1 blocks j0-1 .. j0+P-1.
//
// The phases below run one after another inside one workgroup (separated by
// barriers on the GPU).  Each phase is a loop over independent work items,
// so the same functions also run on the host, one item after another, for
// checking the tile logic without a GPU.
//
//   1. load      x -> registers (8 slots per thread; block b at slot b*S).
//   2. sort      bucket sort (a monotone map of the key onto buckets, LDS
//                atomic counts, scan, scatter, rank within the bucket by
//                the full value).  Tiles of at most four blocks sort all
//                their items at once by (key, block, t) ("tile order");
//                others sort each block by (key, t).  Packing the index
//                into the value makes every value distinct, so the sort is
//                stable in the sense of Section 5.2.  Heavy ties fall back
//                to a merge sort (bitonic in registers, merge-path levels).
//   3. pair orders  for each pair, the merged order of A and B by
//                (key, A-before-B, t) -> M[r] = isB << 15 | t (stored at
//                mslot(r)), and the merged positions posA[t], posB[t]:
//                from a prefix count of each block's items along the tile
//                order, or by merge path.
//   4. tables    for every walk chunk (steps c*L ..), the number of window
//                members below each 64-position word of the merged order at
//                the chunk's start: a packed histogram over (t/L, word) of
//                A and B items, then prefix sums.
//   5. walk      one lane per chunk of L steps (short chunks, so that many
//                lanes walk at once): the window of step i is
//                A[i+1..] u B[..i] (Section 3, postprocessing).  In merged order,
//                position r is a member after step i iff (isA and t > i) or (isB and
//                t <= i).  Step i removes A[i] and adds B[i]; the rank-h
//                member then moves to the next or previous member, or stays:
//                this is the block structures' cursor update (Section 5.3)
//                and rebalancing (Section 6.2) with both cursors folded into
//                one position of the merged order.  A 64-bit register window
//                of membership bits around the median is kept up to date.
//   6. output    y[o] = x[argmed[o]] (bit copy, gathered from x, which the
//                tile has just read; for a 64-bit signal from its 64-bit
//                elements), argmed[o] global index.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MF_HD __host__ __device__ __forceinline__
#else
#define MF_HD static inline
struct uint4 { uint32_t x, y, z, w; };
#endif

#if defined(__HIPCC__)
// Wave-wide reductions and exclusive scans of the ROCm device library (row
// and wave shifts between lanes; every lane of the wave must be active).
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_min_u32(unsigned int);
extern "C" __device__ __attribute__((const)) unsigned int __ockl_wfred_max_u32(unsigned int);
extern "C" __device__ unsigned int __ockl_wfscan_add_u32(unsigned int, bool);
extern "C" __device__ unsigned long __ockl_wfscan_add_u64(unsigned long, bool);
#endif

namespace mf {

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint16_t u16;

static const u64 kPadAll = ~0ull;          // slot beyond the tile's blocks
static const u32 kMPad = 0xFFFFu;          // merged-order padding: never a member

// Slot of merged position r in a pair's M row: within each group of 32
// positions, dword j holds positions j and j + 16, so that the membership
// bits of a group come out of its 16 dwords in position order.
MF_HD int32_t mslot(int32_t r)
{
    const u32 u = (u32)r, rot = (u << 1) | ((u >> 4) & 1u);   // low five bits rotated left by one
    return (int32_t)((rot & 31u) | (u & ~31u));
}

// Byte offset of merged position r in a pair's M row, 2 * mslot(r): bits
// 2..5 take bits 0..3 of r, bit 1 takes bit 4, bits 6.. take bits 5.. (two
// bit-field inserts on the GPU, written out so that the compiler keeps them).
MF_HD u32 mslot_bytes(u32 r)
{
#if defined(__HIP_DEVICE_COMPILE__)
    u32 z, w;
    asm("v_bfi_b32 %0, 60, %1, %2" : "=v"(z) : "v"(r << 2), "v"(r << 1));
    asm("v_bfi_b32 %0, 2, %1, %2" : "=v"(w) : "v"(r >> 3), "v"(z));
    return w;
#else
    return 2u * (u32)mslot((int32_t)r);
#endif
}

// Entry of merged position r in the M row starting at Mp.
MF_HD u16 &m_entry(u16 *Mp, u32 r) { return *(u16 *)((unsigned char *)Mp + mslot_bytes(r)); }
MF_HD u16 m_entry(const u16 *Mp, u32 r) { return *(const u16 *)((const unsigned char *)Mp + mslot_bytes(r)); }

// Lane-wise 16-bit difference a - b of two packed halves.
MF_HD uint32_t psub16(uint32_t a, uint32_t b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    typedef unsigned short v2u16 __attribute__((ext_vector_type(2)));
    const v2u16 d = __builtin_bit_cast(v2u16, a) - __builtin_bit_cast(v2u16, b);
    return __builtin_bit_cast(uint32_t, d);
#else
    return (((a & 0xFFFFu) - (b & 0xFFFFu)) & 0xFFFFu) | ((((a >> 16) - (b >> 16)) & 0xFFFFu) << 16);
#endif
}
static const int kRegs = 8;                // sort values per thread
static const int kRankPad = 4;             // entries past the scattered values that
                                           // the tile-order rank reads unchecked
static const int32_t kPairBudget = 48 * 1024; // bytes of M + pos per tile
static const int kColGroups = 8;           // row groups per count-table column

// ---------------------------------------------------------------- keys

// Unsigned 32-bit key whose order is the value order.  Floats: -0.0 maps
// to +0.0, every NaN maps to the top key (NaN above +inf, NaNs equal).
MF_HD u32 key_of_f32(u32 u)
{
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0xFFFFFFFFu;
    if (u == 0x80000000u) u = 0u;
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

MF_HD u32 key_of_i32(u32 u) { return u ^ 0x80000000u; }

MF_HD int popc64(u64 v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __popcll(v);
#else
    return __builtin_popcountll(v);
#endif
}

MF_HD int ctz64(u64 v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __ffsll((unsigned long long)v) - 1;
#else
    return __builtin_ctzll(v);
#endif
}

MF_HD int hibit64(u64 v)   // index of the highest set bit, v != 0
{
#if defined(__HIP_DEVICE_COMPILE__)
    return 63 - __clzll((long long)v);
#else
    return 63 - __builtin_clzll(v);
#endif
}

// Number of significant bits of v (0 for v = 0).
MF_HD int32_t bitlen32(u32 v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return v ? 32 - __clz((int)v) : 0;
#else
    return v ? 32 - __builtin_clz(v) : 0;
#endif
}

// Position of the q-th (0-based) set bit of w; w must have more than q bits.
MF_HD int select64(u64 w, int q)
{
    int pos = 0;
    int c = popc64(w & 0xFFFFFFFFull);
    if (q >= c) { q -= c; w >>= 32; pos += 32; }
    c = popc64(w & 0xFFFFull);
    if (q >= c) { q -= c; w >>= 16; pos += 16; }
    c = popc64(w & 0xFFull);
    if (q >= c) { q -= c; w >>= 8; pos += 8; }
    c = popc64(w & 0xFull);
    if (q >= c) { q -= c; w >>= 4; pos += 4; }
    c = popc64(w & 0x3ull);
    if (q >= c) { q -= c; w >>= 2; pos += 2; }
    c = (int)(w & 1ull);
    if (q >= c) { pos += 1; }
    return pos;
}

// ---------------------------------------------------------------- geometry

// Shape of the tiles of one signal (fixed n, k) for a given sort capacity.
struct Shape {
    int64_t n;       // signal length
    int32_t k, h;    // window, half-window
    int32_t S;       // slot stride of a block in the sort buffer (pow2 >= k)
    int32_t logS;
    int32_t cap;     // sort capacity of a tile (threads * kRegs)
    int32_t Pmax;    // pairs per full tile
    int64_t nblocks; // ceil(n / k)
    int64_t npairs;  // nblocks - 1
    int64_t ntiles;  // tiles covering all pairs (1 when there is no pair)
    int32_t L;       // walk chunk length (odd)
    int32_t C;       // chunks of a full pair, ceil(k / L)
    int32_t Wn;      // 64-position words of a pair's merged order, ceil(2k/64)
    int32_t Wrow;    // cells per count-table row: even, an odd number of dwords
    int32_t Mstride; // u16 entries per pair in M (Wn * 64; 32 when 2k <= 32)
    int32_t Pstride; // u32 entries per pair in pos (k rounded up to 4)
    int32_t seg;     // merged outputs per pair-merge item (odd)
};

// LDS (or scratch) layout of a tile, in bytes from the base.  The sorted
// blocks are kept as keys and slot indices in two arrays (6 bytes per slot).
struct Layout {
    int32_t xv;      // unused in LDS (-1): the output gathers from x
    int32_t skey;    // u32[cap]  sorted keys
    int32_t sslot;   // u16[cap]  their slots (block << logS | t)
    int32_t mbuf;    // u64[cap]  merge-sort buffer, and the bucket sort's
                     //           scattered values (aliases skey, sslot, M)
    int32_t M;       // u16[Pmax * Mstride]
    int32_t pos;     // u32[Pmax * k]     posA | posB << 16
    int32_t cnt;     // u16[Pmax * C * Wrow]       (aliases skey, sslot)
    int32_t bk;      // u32[cap] bucket counters, after mbuf (aliases M, pos)
    int32_t info;    // u32[2 * nbmax + 1]         (aliases M, pos)
    int32_t nbmax;   // blocks of a full tile
    int32_t stage;   // u16[Pmax * k]              (aliases skey, sslot)
    int32_t total;   // bytes
};

// Largest window walked as a single chunk per pair (no count tables).
static const int32_t kOneChunkMax = 31;

MF_HD int32_t ceil_div32(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

// ceil(2^32 / d) for 2 <= d < 2^16; 0 stands for d = 1.
MF_HD u32 recip32(int32_t d) { return d <= 1 ? 0u : 0xFFFFFFFFu / (u32)d + 1u; }

// a / d for a, d < 2^16 with dr = recip32(d): a high multiply, exact (the
// reciprocal's rounding adds less than a * 2^-32 < 1/d to a/d).
MF_HD u32 udiv16(u32 a, u32 dr)
{
    if (dr == 0u) return a;
#if defined(__HIP_DEVICE_COMPILE__)
    return __umulhi(a, dr);
#else
    return (u32)(((u64)a * dr) >> 32);
#endif
}

// a * b for operands below 2^24 (one 24-bit multiply on the GPU).
MF_HD u32 mul24(u32 a, u32 b)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __umul24(a, b);
#else
    return a * b;
#endif
}

// Fills s for window k over n items with `threads` threads per tile.
// Returns 0, or -1 when k does not fit this capacity (two blocks needed).
// All arithmetic is 32-bit (n < 2^31): the kernels evaluate this per tile.
MF_HD int make_shape(int64_t n, int32_t k, int32_t threads, Shape *s)
{
    const u32 uk = (u32)k, ut = (u32)threads;
    s->n = n;
    s->k = k;
    s->h = (k - 1) >> 1;
    int32_t S = 1, logS = 0;
    while (S < k) { S <<= 1; logS++; }
    s->S = S;
    s->logS = logS;
    s->cap = threads * kRegs;
    if (2 * S > s->cap) return -1;
    s->Wn = (int32_t)((2u * uk + 63u) >> 6);
    // an odd dword stride spreads a column's cells over the LDS banks
    s->Wrow = 2 * (((s->Wn + 1) >> 1) | 1);
    // a pair of k <= 15 fits one 32-position group of membership bits
    s->Mstride = 2 * k <= 32 ? 32 : s->Wn * 64;
    s->Pstride = (k + 3) & ~3;
    // pairs per tile: as many blocks as the sort holds, but the merged
    // orders and position maps of all pairs stay within kPairBudget bytes
    int32_t P = (s->cap >> logS) - 1;
    const int32_t per_pair = 2 * s->Mstride + 4 * s->Pstride + 16;
    if (P * per_pair > kPairBudget) P = (int32_t)((u32)kPairBudget / (u32)per_pair);
    if (P < 1) P = 1;
    s->Pmax = P;
    // pair-merge segments: odd (the lanes of a wave, which take consecutive
    // segments, then read LDS words on distinct banks), long enough that no
    // thread has more than one search chain, but not much longer than the
    // search itself (short blocks: many short segments)
    int32_t seg = (int32_t)(((u32)P * (u32)s->Mstride + ut - 1u) / ut);
    const int32_t seg_max = 2 * logS + 5;
    if (seg > seg_max) seg = seg_max;
    if (seg < 9) seg = 9;
    s->seg = seg | 1;
    // chunk length: odd (lanes walking neighbouring chunks then read the
    // position maps on distinct LDS banks), at least 11, large enough that
    // the tile has no more chunks than threads and that the count tables,
    // their column-group totals and the staged medians of all pairs fit in
    // the sort buffer they reuse.  Windows up to 31 walk a pair in one chunk:
    // the count tables cost more than the longer walk saves.  Otherwise the
    // walk's steps are serial per lane, so shorter chunks pay until the 64
    // further chunks that add a wave to the walk (and to the tables) cost
    // about two steps (the buffer check below lengthens the chunks again
    // where the tables' rows are wide).
    int32_t L = 15;
    {
        int32_t best = 1 << 30;
        for (int32_t l = 15; l >= 11; l -= 2) {
            const u32 c = (uk + (u32)l - 1u) / (u32)l;
            const int32_t cost = l + 2 * (int32_t)(((u32)P * c + 63u) >> 6);
            if (cost < best) { best = cost; L = l; }
        }
    }
    const int32_t per_thread = (int32_t)(((u32)P * uk + ut - 1u) / ut);
    if (L < per_thread) L = per_thread | 1;
    if (k <= kOneChunkMax) L = k;
    u32 C = (uk + (u32)L - 1u) / (u32)L;
    for (;;) {
        const u32 need = (u32)P * (2u * C * (u32)s->Wrow + 2u * uk + 48u);
        if (need <= 6u * (u32)s->cap || L >= k) break;
        L += 2;
        C = (uk + (u32)L - 1u) / (u32)L;
    }
    s->L = L;
    s->C = (int32_t)C;
    s->nblocks = (int64_t)(((u32)n + uk - 1u) / uk);
    s->npairs = s->nblocks - 1;
    s->ntiles = s->npairs > 0 ? (int64_t)(((u32)s->npairs + (u32)P - 1u) / (u32)P) : 1;
    return 0;
}

// Tiles of one pair with 1024 threads (cap >= 8192 slots, two blocks of
// 2048 < k <= 4096) keep their LDS near 80 KB, so that (up to k of about
// 3900) two workgroups share a CU: the tile order counts into cap/2 buckets
// placed right after the scattered values (2k of them), and block order,
// which needs cap counters, is not used (such tiles take the merge sort).
MF_HD bool compact_tile(const Shape &s) { return s.cap >= 8192 && s.Pmax == 1; }
MF_HD int32_t tile_buckets(const Shape &s) { return compact_tile(s) ? s.cap / 2 : s.cap; }

// Row dwords of a count table that hold real cells (two cells each).
MF_HD int32_t col_dwords(const Shape &s) { return (s.Wn + 1) >> 1; }

// 32-position membership dwords of a pair's merged order.
MF_HD int32_t m_dwords(const Shape &s) { return s.Mstride >> 5; }

MF_HD void make_layout(const Shape &s, Layout *l)
{
    int32_t off = 0;
    l->xv = -1;
    l->skey = off;   off += 4 * s.cap;
    l->sslot = off;  off += 2 * s.cap;
    off = (off + 15) & ~15;
    l->mbuf = 0;
    l->M = off;      off += 2 * s.Pmax * s.Mstride;
    off = (off + 15) & ~15;
    l->pos = off;    off += 4 * s.Pmax * s.Pstride;
    off = (off + 15) & ~15;
    // bucket sort scratch, used before the pair orders are written: after the
    // 64-bit scatter buffer (slot-indexed in block order, at most 2k values in
    // the tile order of a compact tile) and the kRankPad entries past it
    l->bk = compact_tile(s) ? ((16 * s.k + 8 * kRankPad + 15) & ~15) : 8 * (s.cap + kRankPad);
    l->info = l->bk + 4 * tile_buckets(s);
    l->nbmax = s.Pmax + 1;
    const int32_t bend = l->info + 4 * (2 * (s.Pmax + 1) + 1);
    if (off < bend) off = (bend + 15) & ~15;
    if (off < 8 * s.cap) off = 8 * s.cap;
    l->total = off;
    int32_t a = 0;
    l->cnt = a;      a += 2 * s.Pmax * s.C * s.Wrow;
    a = (a + 15) & ~15;
    l->stage = a;    a += 2 * s.Pmax * s.k;
    if (a > l->M) l->total = -1;   // aliased region overflows
}

// The tile of pairs [j0, j0 + P).
struct Tile {
    int64_t j0;      // first pair (>= 1)
    int32_t P;       // pairs (0 only for a single-block signal)
    int32_t NB;      // blocks = P + 1
    int64_t e0;      // global index of the first element of the tile
    int64_t o0;      // first output index written by the pairs: (j0-1)k + 1
    int32_t lenLast; // length of block NB-1 (every other block has k items)
    int32_t Clast;   // walk chunks of pair P-1 (every other pair has C)
};

MF_HD Tile make_tile(const Shape &s, int64_t t)
{
    Tile T;
    T.j0 = 1 + t * (int64_t)s.Pmax;
    int64_t left = s.npairs - (T.j0 - 1);
    T.P = (int32_t)(left < s.Pmax ? (left > 0 ? left : 0) : s.Pmax);
    T.NB = T.P + 1;
    T.e0 = (T.j0 - 1) * (int64_t)s.k;
    T.o0 = T.e0 + 1;
    // only the signal's last block can be short, and it ends the last tile
    const int64_t rem = s.n - (T.e0 + (int64_t)(T.NB - 1) * s.k);
    T.lenLast = (int32_t)(rem < s.k ? rem : s.k);
    T.Clast = (T.lenLast + s.L - 1) / s.L;
    return T;
}

// Items of block b of the tile (0 <= b < NB).
MF_HD int32_t block_len(const Shape &s, const Tile &T, int32_t b)
{
    return b == T.NB - 1 ? T.lenLast : s.k;
}

// ---------------------------------------------------------------- views

struct TileMem {
    u32 *bk;         // bucket counters / starts, slot-indexed like skey
    u32 *bmin;       // per block: smallest key
    u32 *bmax;       // per block: largest key
    u32 *flag;       // bit 0: a bucket passed kBucketMax; bit 1: kBucketSoft;
                     // bit 2: the items are not already in sort order
    u32 *xv;
    u32 *skey;
    u16 *sslot;
    u64 *mbuf;
    u16 *M;
    u32 *pos;
    u16 *cnt;
    u16 *stage;
};

MF_HD TileMem tile_mem(unsigned char *base, const Layout &l)
{
    TileMem m;
    m.bk = (u32 *)(base + l.bk);
    m.bmin = (u32 *)(base + l.info);
    m.bmax = m.bmin + l.nbmax;
    m.flag = m.bmax + l.nbmax;
    m.xv = nullptr;
    m.skey = (u32 *)(base + l.skey);
    m.sslot = (u16 *)(base + l.sslot);
    m.mbuf = (u64 *)(base + l.mbuf);
    m.M = (u16 *)(base + l.M);
    m.pos = (u32 *)(base + l.pos);
    m.cnt = (u16 *)(base + l.cnt);
    m.stage = (u16 *)(base + l.stage);
    return m;
}

// ---------------------------------------------------------------- 1. load

// Item = element u of block b (0 <= u < len(b)); items enumerated per block.
MF_HD void load_item(const Shape &s, const Tile &T, const TileMem &m,
                     const u32 *x, int32_t b, int32_t t)
{
    m.xv[((int32_t)b << s.logS) + t] = x[T.e0 + (int64_t)b * s.k + t];
}

// ---------------------------------------------------------------- 2. sort

// Packed sort value of slot u.
template <bool F32>
MF_HD u64 sort_value(const Shape &s, const Tile &T, const TileMem &m, int32_t u)
{
    const int32_t b = u >> s.logS;
    const int32_t t = u & (s.S - 1);
    if (b >= T.NB) return kPadAll;
    const u64 hb = (u64)b << 48;
    if (t >= block_len(s, T, b)) return hb | 0x0000FFFFFFFFFFFFull;   // block padding
    const u32 raw = m.xv[u];
    const u32 key = F32 ? key_of_f32(raw) : key_of_i32(raw);
    return hb | ((u64)key << 16) | (u64)t;
}

// Phase 1, global part: thread `tid` loads the inputs of its kRegs slots
// (block b = slot >> logS, t = slot & (S-1); 0 past a block's end) into
// registers, all loads in flight at once.  Separate from the rest of the
// tile so that a workgroup can issue the next tile's loads early.
MF_HD void load_raw(const Shape &s, const Tile &T, const u32 *x, int32_t tid, u32 (&raw)[kRegs])
{
    if (s.S >= kRegs) {
        // the thread's slots are consecutive items of one block
        const int32_t u = tid * kRegs;
        const int32_t b = u >> s.logS, t0 = u & (s.S - 1);
        const int32_t len = b < T.NB ? block_len(s, T, b) : 0;
        const u32 *src = x + T.e0 + (int64_t)b * s.k + t0;
        if (t0 + kRegs <= len) {
#pragma unroll
            for (int j = 0; j < kRegs; j++) raw[j] = src[j];
        } else {
#pragma unroll
            for (int j = 0; j < kRegs; j++) raw[j] = (t0 + j < len) ? src[j] : 0u;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const int32_t u = tid * kRegs + j;
        const int32_t b = u >> s.logS;
        const int32_t t = u & (s.S - 1);
        const int32_t len = (b < T.NB) ? block_len(s, T, b) : 0;
        raw[j] = (t < len) ? x[T.e0 + (int64_t)b * s.k + t] : 0u;
    }
}

// Phases 1 and 2 together: the packed sort values of the thread's slots.
template <bool F32>
MF_HD void load_sort_values(const Shape &s, const Tile &T, const TileMem &m, const u32 (&raw)[kRegs],
                            int32_t tid, u64 (&v)[kRegs])
{
    if (s.S >= kRegs) {
        const int32_t u = tid * kRegs;
        const int32_t b = u >> s.logS, t0 = u & (s.S - 1);
        const bool inb = b < T.NB;
        const int32_t nv = inb ? block_len(s, T, b) - t0 : 0;
        const u64 hb = (u64)b << 48;
        const u64 pad = inb ? (hb | 0x0000FFFFFFFFFFFFull) : kPadAll;
#pragma unroll
        for (int j = 0; j < kRegs; j++) {
            const u32 key = F32 ? key_of_f32(raw[j]) : key_of_i32(raw[j]);
            v[j] = j < nv ? (hb | ((u64)key << 16) | (u64)(t0 + j)) : pad;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const int32_t u = tid * kRegs + j;
        const int32_t b = u >> s.logS;
        const int32_t t = u & (s.S - 1);
        if (b >= T.NB) { v[j] = kPadAll; continue; }
        const u64 hb = (u64)b << 48;
        if (t >= block_len(s, T, b)) { v[j] = hb | 0x0000FFFFFFFFFFFFull; continue; }
        const u32 key = F32 ? key_of_f32(raw[j]) : key_of_i32(raw[j]);
        v[j] = hb | ((u64)key << 16) | (u64)t;
    }
}

MF_HD void cswap(u64 &a, u64 &b, bool up)
{
    const bool sw = up ? (a > b) : (a < b);
    const u64 lo = sw ? b : a;
    const u64 hi = sw ? a : b;
    a = lo;
    b = hi;
}

// Bitonic sort of kRegs values, ascending.
MF_HD void sort_regs(u64 (&v)[kRegs])
{
#pragma unroll
    for (int size = 2; size <= kRegs; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < kRegs; i++) {
                const int j = i ^ stride;
                if (j > i) cswap(v[i], v[j], (i & size) == 0);
            }
        }
    }
}

// One merge-path level: runs of length w in buf (sorted) are merged pairwise;
// thread `tid` produces outputs [tid*kRegs, tid*kRegs + kRegs) into out.
MF_HD void merge_level(const u64 *buf, int32_t w, int32_t tid, u64 (&out)[kRegs])
{
    const int32_t first = tid * kRegs;
    const int32_t s0 = first & ~(2 * w - 1);
    const u64 *A = buf + s0;
    const u64 *B = buf + s0 + w;
    const int32_t d = first - s0;
    int32_t lo = d > w ? d - w : 0;
    int32_t hi = d < w ? d : w;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (A[mid] < B[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    int32_t a = lo, b = d - lo;
    u64 va = a < w ? A[a] : kPadAll;
    u64 vb = b < w ? B[b] : kPadAll;
#pragma unroll
    for (int q = 0; q < kRegs; q++) {
        const bool takeA = (b >= w) || (a < w && va < vb);
        out[q] = takeA ? va : vb;
        if (takeA) { a++; va = a < w ? A[a] : kPadAll; }
        else       { b++; vb = b < w ? B[b] : kPadAll; }
    }
}

// Sort values carry the block in bits 48..63, the key in bits 16..47 and
// t in bits 0..15.
MF_HD u32 sv_key(u64 v) { return (u32)(v >> 16); }
MF_HD u32 sv_t(u64 v) { return (u32)(v & 0xFFFFu); }

// ---------------------------------------------------------------- 2'. bucket sort
//
// The common path of phase 2 (any sort may serve as the piecewise sort,
// Section 1 "Contribution"): each block's keys are spread over S buckets by
// a monotone map of the value onto [0, S); an item's arrival number in its
// bucket, the bucket starts (a scan of the counts) and its rank among the
// bucket's items by the full (key, t) value give its sorted position.
//
// Maps: the first count uses one linear in the value (integers: the key;
// floats with a finite range: (v - min) * S / (max - min)).  If a bucket
// then holds kBucketSoft or more items (values clustered against the
// block's range, as with rare outliers), the tile counts again with a
// clamped logarithmic map: the float bit pattern of |v| (integers are
// converted to float first), with magnitudes more than kLogSpan binades
// below the block's largest collapsed to zero, signed back; it spreads
// values evenly over orders of magnitude without spending buckets on the
// tiny ones.  A tile whose buckets still hold more than kBucketMax items
// (heavy ties) takes the merge sort above instead.
// Needs S >= kRegs, so that the kRegs slots of a thread lie in one block.

static const int kBucketMax = 32;
static const int kBucketSoft = 12;
static const u32 kLogSpan = 16;
enum { BK_KEY = 0, BK_FLIN = 1, BK_CLOG = 2 };

MF_HD u32 f32_bits(float f)
{
    union { float f; u32 u; } c;
    c.f = f;
    return c.u;
}

MF_HD float bits_f32(u32 u)
{
    union { float f; u32 u; } c;
    c.u = u;
    return c.f;
}

// Float value of a float key (finite keys; -0.0 comes back as +0.0).
MF_HD float f32_of_key(u32 key) { return bits_f32((key & 0x80000000u) ? (key & 0x7FFFFFFFu) : ~key); }

// Key of the float nearest to the integer of an integer key (monotone).
MF_HD u32 ilog_key(u32 key) { return key_of_f32(f32_bits((float)(int32_t)(key ^ 0x80000000u))); }

// Magnitude bits |v| of a float key.
MF_HD u32 key_mag(u32 fk) { return (fk & 0x80000000u) ? (fk & 0x7FFFFFFFu) : (~fk & 0x7FFFFFFFu); }

// Clamped logarithmic code of a float key: monotone in the key.
MF_HD u32 clog_code(u32 fk, u32 floor_mag)
{
    const u32 mag = key_mag(fk);
    const u32 c = mag > floor_mag ? mag - floor_mag : 0u;
    return (fk & 0x80000000u) ? 0x40000000u + c : 0x40000000u - c;
}

// A block's bucket map.
struct BucketFn {
    u32 mode, lo, sh;
    float fmin, scale;   // BK_FLIN
    u32 floor_mag;       // BK_CLOG
    u32 top;             // S - 1
};

template <bool F32>
MF_HD u32 bucket_of(const BucketFn &f, u32 key)
{
    if (F32 && f.mode == BK_FLIN) {
        const u32 q = (u32)((f32_of_key(key) - f.fmin) * f.scale);
        return q < f.top ? q : f.top;
    }
    if (f.mode == BK_CLOG) return (clog_code(F32 ? key : ilog_key(key), f.floor_mag) - f.lo) >> f.sh;
    return (key - f.lo) >> f.sh;
}

MF_HD bool sv_valid(u64 v) { return (v & 0xFFFFu) != 0xFFFFu; }
MF_HD int32_t sv_block(u64 v) { return (int32_t)(v >> 48); }

// Sorted item at slot q: key and slot index (block << logS | t).
MF_HD void put_sorted(const TileMem &m, int32_t q, u32 key, u32 slot)
{
    m.skey[q] = key;
    m.sslot[q] = (u16)slot;
}

// The sorted item at q as a block-order value of block 0 (key << 16 | t),
// for comparisons within a block and for merge path.
MF_HD u64 sorted_kt(const Shape &s, const TileMem &m, int32_t q)
{
    return ((u64)m.skey[q] << 16) | (u64)(m.sslot[q] & (u32)(s.S - 1));
}

MF_HD void put_block_value(const Shape &s, const TileMem &m, int32_t q, u64 v)
{
    put_sorted(m, q, sv_key(v), ((u32)sv_block(v) << s.logS) | sv_t(v));
}

// Thread tid's `per` consecutive counters (per = 8, or 4 in a compact
// tile: tile_buckets / threads).
MF_HD void bucket_zero_thread(const TileMem &m, int32_t tid, int32_t per)
{
    uint4 *p = (uint4 *)(m.bk + tid * per);
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int j = 0; j < per / 4; j++) p[j] = z;
}
// Block info entry b < nbmax.
MF_HD void bucket_info_init(const TileMem &m, int32_t b)
{
    m.bmin[b] = 0xFFFFFFFFu;
    m.bmax[b] = 0u;
    if (b == 0) m.flag[0] = 0u;
}

#if defined(__HIP_DEVICE_COMPILE__)
#define MF_MIN32(ptr, v) atomicMin((unsigned int *)(ptr), (unsigned int)(v))
#define MF_MAX32(ptr, v) atomicMax((unsigned int *)(ptr), (unsigned int)(v))
#define MF_ADDRTN32(ptr, v) atomicAdd((unsigned int *)(ptr), (unsigned int)(v))
#define MF_OR32(ptr, v) atomicOr((unsigned int *)(ptr), (unsigned int)(v))
#else
#define MF_OR32(ptr, v) (*(ptr) |= (v))
#define MF_MIN32(ptr, v) (*(ptr) = (*(ptr) < (v) ? *(ptr) : (v)))
#define MF_MAX32(ptr, v) (*(ptr) = (*(ptr) > (v) ? *(ptr) : (v)))
static inline u32 mf_addrtn32(u32 *p, u32 v) { u32 o = *p; *p += v; return o; }
#define MF_ADDRTN32(ptr, v) mf_addrtn32((ptr), (v))
#endif

// Per thread: the thread's keys' minimum and maximum into its block's info.
MF_HD void bucket_minmax(const TileMem &m, const u64 (&v)[kRegs])
{
    u32 mn = 0xFFFFFFFFu, mx = 0u;
    int32_t b = -1;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        if (sv_valid(v[j])) {
            const u32 key = sv_key(v[j]);
            mn = key < mn ? key : mn;
            mx = key > mx ? key : mx;
            b = sv_block(v[j]);
        }
    }
    if (b >= 0) {
        MF_MIN32(m.bmin + b, mn);
        MF_MAX32(m.bmax + b, mx);
    }
}

// The bucket map of `pass` (0: linear in the value, 1: clamped
// logarithmic) for keys in [mn, mx], landing in [0, S).  Every thread that
// needs a block's map builds it from the block's key range (the same
// arithmetic everywhere, so the same map).
template <bool F32>
MF_HD BucketFn make_bucket_fn(int32_t S, int32_t logS, u32 mn, u32 mx, int pass)
{
    BucketFn f;
    f.mode = BK_KEY;
    f.lo = mn;
    f.fmin = f.scale = 0.f;
    f.floor_mag = 0u;
    f.top = (u32)S - 1u;
    u32 hi = mx;
    if (F32 && pass == 0 && mn > 0x007FFFFFu && mx < 0xFF800000u) {   // finite range
        const float a = f32_of_key(mn), r = f32_of_key(mx) - a;
        if (r > 0.f && r <= 3.0e38f) {
            const float sc = (float)S / r;
            if (sc <= 3.0e38f) {
                f.mode = BK_FLIN;
                f.fmin = a;
                f.scale = sc;
            }
        }
    }
    if (pass == 1) {
        const u32 a = F32 ? mn : ilog_key(mn), z = F32 ? mx : ilog_key(mx);
        const u32 ma = key_mag(a), mz = key_mag(z);
        const u32 top = ma > mz ? ma : mz, span = kLogSpan << 23;
        f.mode = BK_CLOG;
        f.floor_mag = top > span ? top - span : 0u;
        f.lo = clog_code(a, f.floor_mag);
        hi = clog_code(z, f.floor_mag);
    }
    const int32_t bits = bitlen32(hi - f.lo);
    f.sh = (u32)(bits > logS ? bits - logS : 0);
    return f;
}

template <bool F32>
MF_HD BucketFn bucket_fn(const Shape &s, const TileMem &m, int32_t b, int pass)
{
    return make_bucket_fn<F32>(s.S, s.logS, m.bmin[b], m.bmax[b], pass);
}

// A block's bucket parameters, read once per thread.
struct BlockView {
    u32 mn, mx, len;
    BucketFn f;
    const u32 *start;      // bucket starts (after the scan)
    int32_t base;          // the block's first slot
};

template <bool F32>
MF_HD BlockView block_view(const Shape &s, const Tile &T, const TileMem &m, int32_t b, int pass)
{
    BlockView V;
    V.mn = m.bmin[b];
    V.mx = m.bmax[b];
    V.f = bucket_fn<F32>(s, m, b, pass);
    V.len = (u32)block_len(s, T, b);
    V.start = m.bk + (b << s.logS);
    V.base = b << s.logS;
    return V;
}

// Block of thread tid's slots (S >= kRegs), or -1 if they lie past the tile.
MF_HD int32_t thread_block(const Shape &s, const Tile &T, int32_t tid)
{
    const int32_t b = (tid * kRegs) >> s.logS;
    return b < T.NB ? b : -1;
}

// Per thread: count each item in its bucket; the old count is its arrival
// number.  Sets the flag when a bucket passes kBucketMax.
template <bool F32>
MF_HD void bucket_count(const Shape &s, const Tile &T, const TileMem &m, int32_t tid,
                        const u64 (&v)[kRegs], u32 (&arr)[kRegs], int pass)
{
    const int32_t b = thread_block(s, T, tid);
    BucketFn f;
    f.mode = BK_KEY;
    f.lo = f.sh = 0u;
    f.fmin = f.scale = 0.f;
    f.floor_mag = f.top = 0u;
    if (b >= 0) f = bucket_fn<F32>(s, m, b, pass);
    u32 *cnt = m.bk + (b >= 0 ? (b << s.logS) : 0);
    u32 mx = 0u;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        arr[j] = 0u;
        if (sv_valid(v[j])) {
            arr[j] = MF_ADDRTN32(cnt + bucket_of<F32>(f, sv_key(v[j])), 1u);
            mx = arr[j] > mx ? arr[j] : mx;
        }
    }
    if (mx >= (u32)kBucketSoft) MF_OR32(m.flag, mx >= (u32)kBucketMax ? 3u : 2u);
}

// Per thread: the local part of the bucket scan.  Thread tid owns counters
// [tid*per, tid*per + per) (per = 8, or 4 in a compact tile); on return c
// holds their exclusive prefix within the thread and the thread total is
// returned.
MF_HD u32 bucket_scan_local(const TileMem &m, int32_t tid, u32 (&c)[kRegs], int32_t per)
{
    const uint4 *src = (const uint4 *)(m.bk + tid * per);
    u32 acc = 0u;
    for (int g = 0; g < per / 4; g++) {
        const uint4 q = src[g];
        c[4 * g + 0] = acc; acc += q.x;
        c[4 * g + 1] = acc; acc += q.y;
        c[4 * g + 2] = acc; acc += q.z;
        c[4 * g + 3] = acc; acc += q.w;
    }
    return acc;
}

// Per thread: bucket starts = prefix of earlier threads of the block (excl)
// plus the local prefix.
MF_HD void bucket_scan_store(const TileMem &m, int32_t tid, u32 excl, const u32 (&c)[kRegs], int32_t per)
{
    uint4 *dst = (uint4 *)(m.bk + tid * per);
    for (int g = 0; g < per / 4; g++) {
        uint4 q;
        q.x = excl + c[4 * g + 0];
        q.y = excl + c[4 * g + 1];
        q.z = excl + c[4 * g + 2];
        q.w = excl + c[4 * g + 3];
        dst[g] = q;
    }
}

// Entries of the scattered bucket [x, hi) of buf below v.  The first four
// are read by every lane without a loop (an entry past the bucket is read
// at x and not counted); longer buckets loop over the rest.
template <typename P>
MF_HD u32 bucket_below(P buf, u32 x, u32 hi, u64 v)
{
    const u32 n = hi - x;
    u32 f = 0u;
#pragma unroll
    for (u32 u = 0; u < 4u; u++) {
        const u64 e = buf[x + (u < n ? u : 0u)];
        f += (u < n && e < v) ? 1u : 0u;
    }
    for (u32 q = x + 4u; q < hi; q++) f += (buf[q] < v) ? 1u : 0u;
    return f;
}

// Bucket [lo, hi) of key in block view V (key within the block's range).
template <bool F32>
MF_HD void view_bucket(const Shape &s, const BlockView &V, u32 key, u32 &lo, u32 &hi)
{
    const u32 bk = bucket_of<F32>(V.f, key);
    lo = V.start[bk];
    hi = (bk + 1u < (u32)s.S) ? V.start[bk + 1] : V.len;
}

// Per thread: place each item at bucket start + arrival number.
template <bool F32>
MF_HD void bucket_scatter(const Shape &s, const Tile &T, const TileMem &m, int32_t tid,
                          const u64 (&v)[kRegs], const u32 (&arr)[kRegs], int pass)
{
    const int32_t b = thread_block(s, T, tid);
    if (b < 0) return;
    const BlockView V = block_view<F32>(s, T, m, b, pass);
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if (sv_valid(v[j])) m.mbuf[V.base + (int32_t)(V.start[bucket_of<F32>(V.f, sv_key(v[j]))] + arr[j])] = v[j];
}

// Per thread: final position = bucket start + rank among the bucket's items
// by the full value.
template <bool F32>
MF_HD void bucket_rank(const Shape &s, const Tile &T, const TileMem &m, int32_t tid,
                       const u64 (&v)[kRegs], u32 (&fin)[kRegs], int pass)
{
    const int32_t b = thread_block(s, T, tid);
    u32 x[kRegs], hi[kRegs];
    BlockView V;
    V.base = 0;
    if (b >= 0) V = block_view<F32>(s, T, m, b, pass);
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        x[j] = 0u;
        hi[j] = 0u;
        if (b >= 0 && sv_valid(v[j])) view_bucket<F32>(s, V, sv_key(v[j]), x[j], hi[j]);
        fin[j] = x[j];
    }
    // one bucket scan per item: a wave pays, per item slot, for the largest
    // of its lanes' buckets (rather than for the largest of all its items)
#pragma unroll
    for (int j = 0; j < kRegs; j++) fin[j] += bucket_below(m.mbuf + V.base, x[j], hi[j], v[j]);
}

// Per thread: write the sorted blocks (after every rank has been read).
MF_HD void bucket_place(const Shape &s, const TileMem &m, const u64 (&v)[kRegs], const u32 (&fin)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if (sv_valid(v[j])) put_block_value(s, m, (sv_block(v[j]) << s.logS) + (int32_t)fin[j], v[j]);
}

// Walk chunks of pair p (phase 4), and row c of its count table.
MF_HD int32_t pair_chunks(const Shape &s, const Tile &T, int32_t p)
{
    return p == T.P - 1 ? T.Clast : s.C;
}

#if defined(__HIP_DEVICE_COMPILE__)
#define MF_ADD32(ptr, v) atomicAdd((unsigned int *)(ptr), (unsigned int)(v))
#else
#define MF_ADD32(ptr, v) (*(ptr) += (v))
#endif

// Row c of pair p's count table: 16-bit cells.  While the histogram is
// built, a cell holds its word's A items in the low byte and B items in the
// high byte (each at most 64); after the column pass, a member count.
MF_HD int32_t cnt_row_idx(const Shape &s, int32_t p, int32_t c)
{
    return (int32_t)mul24(mul24((u32)p, (u32)s.C) + (u32)c, (u32)s.Wrow);
}

MF_HD u16 *cnt_row(const Shape &s, const TileMem &m, int32_t p, int32_t c)
{
    return m.cnt + cnt_row_idx(s, p, c);
}

// Adds v (1 for an A item, 0x100 for a B item) to cell e, through an atomic
// add on the 32-bit word that holds it (the other cell's bytes never carry).
MF_HD void cnt_add(const TileMem &m, int32_t e, u32 v)
{
    MF_ADD32((u32 *)((unsigned char *)m.cnt + 2 * (e & ~1)), v << (16 * (e & 1)));
}


// ---------------------------------------------------------------- 2''. tile-order sort
//
// Tiles of at most four blocks sort all their items at once by (key, block,
// t).  Restricted to blocks b and b + 1 that order is pair b's merged order
// (on equal keys A = block b comes first, then t), so counting, along it,
// the items of each block gives every item its merged position in both of
// its pairs: phase 3 without a merge.  The counts of the four blocks are
// packed in one 64-bit word (16 bits each), so the count is one prefix scan.
// The sort is the bucket sort above over a single segment: cap buckets
// spanning the tile's value range.  Values: key << 32 | slot, where the
// slot (block << logS | t) orders like (block, t); padding ~0 (slot field
// 0xFFFF, so sv_valid still applies).

static const int kTileOrderBlocks = 4;

MF_HD bool tile_order_ok(const Shape &s) { return s.Pmax + 1 <= kTileOrderBlocks && s.S >= kRegs; }

MF_HD u32 tv_key(u64 v) { return (u32)(v >> 32); }
MF_HD u32 tv_slot(u64 v) { return (u32)(v & 0xFFFFu); }

// The bucket sort's shape for the tile-wide segment (tile_buckets buckets).
MF_HD Shape tile_order_shape(const Shape &s)
{
    Shape st = s;
    st.S = tile_buckets(s);
    int32_t l = 0;
    while ((1 << l) < st.S) l++;
    st.logS = l;
    return st;
}

// Valid items of the tile.
MF_HD int32_t tile_items(const Shape &s, const Tile &T)
{
    int32_t N = 0;
    for (int32_t b = 0; b < T.NB; b++) N += block_len(s, T, b);
    return N;
}

// Phase 1 for tile order: as load_sort_values, with tile-order values.
template <bool F32>
MF_HD void load_tile_values(const Shape &s, const Tile &T, const TileMem &m, const u32 (&raw)[kRegs],
                            int32_t tid, u64 (&v)[kRegs])
{
    if (s.S >= kRegs) {
        const int32_t u = tid * kRegs;
        const int32_t b = u >> s.logS, t0 = u & (s.S - 1);
        const int32_t nv = b < T.NB ? block_len(s, T, b) - t0 : 0;
#pragma unroll
        for (int j = 0; j < kRegs; j++) {
            const u32 key = F32 ? key_of_f32(raw[j]) : key_of_i32(raw[j]);
            v[j] = j < nv ? (((u64)key << 32) | (u64)(u + j)) : kPadAll;
        }
        return;
    }
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const int32_t u = tid * kRegs + j;
        const int32_t b = u >> s.logS;
        const int32_t t = u & (s.S - 1);
        if (b >= T.NB || t >= block_len(s, T, b)) { v[j] = kPadAll; continue; }
        const u32 key = F32 ? key_of_f32(raw[j]) : key_of_i32(raw[j]);
        v[j] = ((u64)key << 32) | (u64)u;
    }
}

// The same slots as block-first sort values (for the merge-sort fallback).
MF_HD void tile_to_block_values(const Shape &s, const Tile &T, int32_t tid, u64 (&v)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const int32_t b = (tid * kRegs + j) >> s.logS;
        if (sv_valid(v[j])) v[j] = ((u64)b << 48) | ((u64)tv_key(v[j]) << 16) | (u64)(tv_slot(v[j]) & (u32)(s.S - 1));
        else v[j] = (b >= T.NB) ? kPadAll : (((u64)b << 48) | 0x0000FFFFFFFFFFFFull);
    }
}

// Per thread: the tile's key range into block info entry 0 (reduced over
// the wave first, so that one lane per wave updates the shared words).
MF_HD void tile_minmax(const TileMem &m, const u64 (&v)[kRegs])
{
    // padding (kPadAll, never a real value: its slot field is past every
    // slot) has the largest key, which leaves the minimum alone
    u32 mn = 0xFFFFFFFFu, mx = 0u;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const u32 key = tv_key(v[j]);
        const u32 kx = v[j] == kPadAll ? 0u : key;
        mn = key < mn ? key : mn;
        mx = kx > mx ? kx : mx;
    }
#if defined(__HIP_DEVICE_COMPILE__)
    mn = __ockl_wfred_min_u32(mn);
    mx = __ockl_wfred_max_u32(mx);
    const bool lead = (threadIdx.x & 63) == 0;
#else
    const bool lead = true;
#endif
    if (lead && mn <= mx) {
        MF_MIN32(m.bmin, mn);
        MF_MAX32(m.bmax, mx);
    }
}

// After tile_minmax: true when the tile's values are so few (range under a
// quarter of the item count) that equal keys would crowd its buckets; such
// tiles sort block by block.
MF_HD bool tile_many_ties(const TileMem &m, int32_t N)
{
    const u32 range = m.bmax[0] - m.bmin[0];
    return (u64)range * 4u < (u64)N;
}

// Per thread: each item's bucket and arrival number in it (st =
// tile_order_shape), packed as bucket << 8 | arrival (arrivals stay below
// kBucketMax, or the tile leaves the tile order), for scatter and rank.
template <bool F32>
MF_HD void tile_count(const Shape &st, const TileMem &m, const u64 (&v)[kRegs], u32 (&ab)[kRegs], int pass)
{
    const BucketFn f = bucket_fn<F32>(st, m, 0, pass);
    u32 mx = 0u;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        ab[j] = 0u;
        if (sv_valid(v[j])) {
            const u32 bk = bucket_of<F32>(f, tv_key(v[j]));
            const u32 a = MF_ADDRTN32(m.bk + bk, 1u);
            mx = a > mx ? a : mx;
            ab[j] = (bk << 8) | (a & 0xFFu);
        }
    }
    if (mx >= (u32)kBucketSoft) MF_OR32(m.flag, mx >= (u32)kBucketMax ? 3u : 2u);
}

MF_HD void tile_scatter(const TileMem &m, const u64 (&v)[kRegs], const u32 (&ab)[kRegs], int32_t tid, int32_t N)
{
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if (sv_valid(v[j])) m.mbuf[m.bk[ab[j] >> 8] + (ab[j] & 0xFFu)] = v[j];
    if (tid < kRankPad) m.mbuf[N + tid] = kPadAll;
}

// Per thread: sorted position = bucket start + rank by the full value among
// the bucket's items (as in bucket_rank).  N: valid items.
MF_HD void tile_rank(const Shape &st, const TileMem &m, const u64 (&v)[kRegs], int32_t N, u32 (&fin)[kRegs],
                     const u32 (&ab)[kRegs])
{
    u32 x[kRegs], hi[kRegs];
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        x[j] = 0u;
        hi[j] = 0u;
        if (sv_valid(v[j])) {
            const u32 bk = ab[j] >> 8;
            x[j] = m.bk[bk];
            hi[j] = (bk + 1u < (u32)st.S) ? m.bk[bk + 1] : (u32)N;
        }
        fin[j] = x[j];
    }
    // Buckets hold consecutive key ranges, so the entries after an item's
    // bucket, up to the padding past the last one, all order above it: the
    // first kRankPad entries from the bucket's start are compared without
    // a bound, the rest of a longer bucket in a loop.  A bucket of one item
    // (the item itself) needs no comparison.
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        u32 f = 0u;
        if (hi[j] - x[j] > 1u) {
#pragma unroll
            for (int u = 0; u < kRankPad; u++) f += (m.mbuf[x[j] + (u32)u] < v[j]) ? 1u : 0u;
            for (u32 q = x[j] + (u32)kRankPad; q < hi[j]; q++) f += (m.mbuf[q] < v[j]) ? 1u : 0u;
        }
        fin[j] += f;
    }
}

// The pair orders read only the slots of the tile order, not the keys.
MF_HD void tile_place(const TileMem &m, const u64 (&v)[kRegs], const u32 (&fin)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if (sv_valid(v[j])) m.sslot[fin[j]] = (u16)tv_slot(v[j]);
}

// Per thread: the slots of its kRegs consecutive tile-order items (into w,
// 0xFFFF past the end) and their count per block, packed 16 bits per block.
MF_HD u64 tile_label_counts(const Shape &s, const TileMem &m, int32_t tid, int32_t N, u32 (&w)[kRegs])
{
    u64 c = 0ull;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const int32_t q = tid * kRegs + j;
        w[j] = q < N ? (u32)m.sslot[q] : 0xFFFFu;
        if (q < N) c += 1ull << (16 * (int32_t)(w[j] >> s.logS));
    }
    return c;
}

// Per thread: with excl = the packed counts of all earlier items, the
// merged positions of its items in both of their pairs (M and the position
// maps), each pair's first median (A's item of own rank h) and output 0
// (x, y: the elements output 0 is copied from and to, 32- or 64-bit).
template <typename V>
MF_HD void tile_positions(const Shape &s, const Tile &T, const TileMem &m, u64 excl, const u32 (&w)[kRegs],
                          const V *x, V *y, int32_t *argmed)
{
    // with more than one walk chunk, also the count histogram of phase 4
    // (table_hist_item for both merged positions of every item)
    const bool hist = s.C > 1;
    const u32 Lr = recip32(s.L);
    const u32 CW = (u32)(s.C * s.Wrow);   // cells of a pair's table
    u64 c = excl;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        if (w[j] == 0xFFFFu) continue;
        const u32 b = w[j] >> s.logS;
        const u32 t = w[j] & (u32)(s.S - 1);
        const u32 sh = 16u * b;
        // field q of R: earlier items of blocks q and q + 1 = rank in pair q
        const u64 R = c + (c >> 16);
        // the item's table row within its pairs (t/L; rows past the last
        // pair's chunks only feed the column sums)
        const u32 rowc = hist ? mul24(udiv16(t, Lr), (u32)s.Wrow) + mul24(b, CW) : 0u;
        const u32 cb = (u32)(c >> sh) & 0xFFFFu;
        // pair b's M row and position map; pair b - 1's are one row before
        u16 *MA = m.M + mul24(b, (u32)s.Mstride);
        u16 *QA = (u16 *)(m.pos + mul24(b, (u32)s.Pstride)) + 2u * t;
        if ((int32_t)b < T.P) {   // A of pair b
            const u32 r = (u32)(R >> sh) & 0xFFFFu;
            m_entry(MA, r) = (u16)t;
            QA[0] = (u16)r;
            if (cb == (u32)s.h) m.pos[mul24(b, (u32)s.Pstride) + (u32)s.k] = r;
            if (hist) cnt_add(m, (int32_t)(rowc + (r >> 6)), 1u);
        }
        if (b >= 1u) {    // B of pair b - 1
            const u32 r = (u32)(R >> (sh - 16u)) & 0xFFFFu;
            m_entry(MA - s.Mstride, r) = (u16)(0x8000u | t);
            QA[1 - 2 * s.Pstride] = (u16)r;
            if (hist) cnt_add(m, (int32_t)(rowc - CW + (r >> 6)), 0x100u);
        }
        if (b == 0u && cb == (u32)s.h && T.j0 == 1) {   // output 0: the median of block 0
            y[0] = x[t];
            if (argmed) argmed[0] = (int32_t)t;
        }
        c += 1ull << sh;
    }
}

// Thread tid's share of the merged-order padding (tile order).
MF_HD void tile_mpad(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    // positions [2k, Mstride) of every pair (2k is never a multiple of 64,
    // so there is at least one), and [k + len B, 2k) of a last pair whose B
    // is short
    const int32_t npad = s.Mstride - 2 * s.k;
    const u32 padr = recip32(npad);
    for (int32_t it = tid; it < T.P * npad; it += NT) {
        const u32 p = udiv16((u32)it, padr);
        m.M[mul24(p, (u32)s.Mstride) + mslot(2 * s.k + it - (int32_t)mul24(p, (u32)npad))] = (u16)kMPad;
    }
    if (T.P > 0)
        for (int32_t r = s.k + T.lenLast + tid; r < 2 * s.k; r += NT)
            m.M[(T.P - 1) * s.Mstride + mslot(r)] = (u16)kMPad;
}

// ---------------------------------------------------------------- 2+. presorted tiles
//
// A tile whose items already stand in sort order (the benign inputs of the
// paper's experiments, Section 7: ascending or nearly ascending data) needs
// no sort: the bucket sort is skipped and every item goes straight to its
// sorted position.  The check rides on the passes that find the key range:
// each thread notes its first value before their barrier (presort_note),
// then checks its own items and the step to the next item (presort_check),
// setting flag bit 2 on any descent.  In tile order the whole tile must be
// in (key, slot) order; in block order each block in (key, t) order.

MF_HD u64 first_value(const u64 (&v)[kRegs])
{
    u64 f = kPadAll;
#pragma unroll
    for (int j = kRegs - 1; j >= 0; j--)
        if (sv_valid(v[j])) f = v[j];
    return f;
}

// Before the barrier (the scratch is the merge-sort buffer, free here).
MF_HD void presort_note(const Shape &s, const TileMem &m, int32_t tid, const u64 (&v)[kRegs])
{
    // with S >= kRegs a thread's valid items are a prefix of its slots
    m.mbuf[tid] = s.S >= kRegs ? (sv_valid(v[0]) ? v[0] : kPadAll) : first_value(v);
}

// After the barrier; tile: tile-order values (else block order).
MF_HD void presort_check(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT,
                         const u64 (&v)[kRegs], bool tile)
{
    bool ok = true, any = false;
    u64 last = 0ull;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        if (sv_valid(v[j])) {
            ok = ok && (!any || last < v[j]);
            last = v[j];
            any = true;
        }
    }
    if (any) {
        // the item after the thread's last: the next thread's first, or, when
        // the last ends its block, the first of the next block (tile order)
        const u32 u = tile ? tv_slot(last) : (((u32)sv_block(last) << s.logS) | sv_t(last));
        const int32_t b = (int32_t)(u >> s.logS), t = (int32_t)(u & (u32)(s.S - 1));
        u64 next = kPadAll;
        if (t == block_len(s, T, b) - 1) {
            if (tile && b + 1 < T.NB) next = m.mbuf[((b + 1) << s.logS) / kRegs];
        } else if (tid + 1 < NT) {
            next = m.mbuf[tid + 1];
        }
        ok = ok && (next == kPadAll || last < next);
    }
    if (!ok) MF_OR32(m.flag, 4u);
}

// Sorted positions of a presorted tile: in tile order the rank of block b's
// item t is b*k + t (every block before the last is full); in block order
// an item stays at its slot.
MF_HD void presort_place(const Shape &s, const TileMem &m, const u64 (&v)[kRegs], bool tile)
{
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        if (!sv_valid(v[j])) continue;
        if (tile) {
            const u32 u = tv_slot(v[j]);
            const int32_t b = (int32_t)(u >> s.logS), t = (int32_t)(u & (u32)(s.S - 1));
            m.sslot[b * s.k + t] = (u16)u;
        } else {
            put_block_value(s, m, (sv_block(v[j]) << s.logS) + (int32_t)sv_t(v[j]), v[j]);
        }
    }
}

// ---------------------------------------------------------------- 3. pair merge


MF_HD int32_t merge_items_per_pair(const Shape &s) { return (2 * s.k + s.seg - 1) / s.seg; }

// 16-byte stores of merged-order padding per pair: every 32-position group
// from the one holding the pair's last position on (the merge then writes
// the group's real entries).
MF_HD int32_t pad_items_per_pair(const Shape &s) { return (s.Mstride - (((s.k + 1) >> 5) << 5)) / 8; }

// Item = (pair p, store q) of the padding.
MF_HD void pair_pad_item(const Shape &s, const Tile &T, const TileMem &m, int32_t p, int32_t q)
{
    const int32_t mlen = s.k + block_len(s, T, p + 1);
    const int32_t r0 = s.Mstride - 8 * (pad_items_per_pair(s) - q);
    if (r0 < ((mlen >> 5) << 5)) return;
    const uint4 pad = {0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu};
    *(uint4 *)(m.M + p * s.Mstride + r0) = pad;
}

// Item = (pair p, segment g): merged positions [g*seg, (g+1)*seg) of pair p, by
// merge path over the sorted blocks A = p and B = p + 1 (A first on equal
// keys), writing M and the position maps.
MF_HD void pair_merge_item(const Shape &s, const Tile &T, const TileMem &m,
                           int32_t p, int32_t g)
{
    const int32_t lenA = s.k;
    const int32_t lenB = block_len(s, T, p + 1);
    const int32_t mlen = lenA + lenB;
    const int32_t A = (int32_t)p << s.logS, B = (int32_t)(p + 1) << s.logS;   // first slots
    u16 *Mp = m.M + p * s.Mstride;
    u16 *pos = (u16 *)(m.pos + p * s.Pstride);
    const int32_t d = g * s.seg;
    if (d >= mlen) return;   // the padding is written by pair_pad_item
    int32_t lo = d > lenB ? d - lenB : 0;
    int32_t hi = d < lenA ? d : lenA;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        // A[mid] precedes B[d-1-mid] iff keyA <= keyB (A first on ties)
        if (m.skey[A + mid] <= m.skey[B + d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    int32_t a = lo, b = d - lo;
    u64 va = a < lenA ? sorted_kt(s, m, A + a) : 0ull, vb = b < lenB ? sorted_kt(s, m, B + b) : 0ull;
    for (int q = 0; q < s.seg; q++) {
        const int32_t r = d + q;
        if (r >= mlen) break;
        const bool takeA = a < lenA && (b >= lenB || sv_key(va) <= sv_key(vb));
        const u32 t = sv_t(takeA ? va : vb);
        Mp[mslot(r)] = (u16)(takeA ? t : (0x8000u | t));
        pos[2 * t + (takeA ? 0 : 1)] = (u16)r;   // posA low half, posB high half
        a += takeA ? 1 : 0;
        b += takeA ? 0 : 1;
        const int32_t ni = takeA ? a : b;
        const bool more = takeA ? (a < lenA) : (b < lenB);
        const u64 nv = more ? sorted_kt(s, m, (takeA ? A : B) + ni) : 0ull;
        va = takeA ? nv : va;
        vb = takeA ? vb : nv;
    }
}

// ---------------------------------------------------------------- 4. tables


// Count table of pair p: row c (chunk start c*L), column w (64-position
// word): after the passes below, entry (c, w) is the number of members of
// the window before step c*L among merged positions < 64w; column Wn holds
// the total (k).  A position holding A's item t is a member before step cL
// iff t >= cL, one holding B's item t iff t < cL.


// Item = 32-bit word e of the tables (two cells): zero it.
MF_HD void table_zero_item(const TileMem &m, int32_t e) { ((u32 *)m.cnt)[e] = 0u; }


// Item = merged position r of pair p (r < k + len B): count its item in
// bucket (t/L, r/64); A items in the low half, B items in the high.  Every
// pair has C rows: a last pair with a short B walks fewer chunks, and its
// later rows hold only A items, which reach the earlier rows through the
// column sums.  Lrcp = recip32(L) makes t/L a high multiply (exact for
// t, L < 2^16).
MF_HD void table_hist_item(const Shape &s, const TileMem &m, int32_t p, int32_t r, u32 Lrcp)
{
    const u32 e = m.M[p * s.Mstride + mslot(r)];
    const u32 t = e & 0x7FFFu;
    const int32_t b = (int32_t)udiv16(t, Lrcp);
    cnt_add(m, cnt_row_idx(s, p, b) + (r >> 6), (e & 0x8000u) ? 0x100u : 1u);
}


// Column pass: entry (c, w) becomes the members of word w at chunk start
// c, (A items with bucket >= c) + (B items with bucket < c).  A lane takes
// the two cells of one row dword (words 2d and 2d + 1) at once: their A
// bytes and B bytes are summed as two 16-bit fields each (a column holds
// at most 64 items, so the fields never carry).  Each column's rows are cut
// into kColGroups groups of R = ceil(C / 8) consecutive rows
// (tail_table_columns).

MF_HD int32_t col_rows(const Shape &s) { return (s.C + kColGroups - 1) / kColGroups; }

// Item = (pair p, chunk c): exclusive prefix over the words, sixteen cells
// (eight dwords, read before any is written) at a time.
MF_HD void table_row_item(const Shape &s, const TileMem &m, int32_t p, int32_t c)
{
    u32 *row = (u32 *)cnt_row(s, m, p, c);
    const int32_t nd = s.Wrow / 2;
    u32 acc = 0u;
    for (int32_t d0 = 0; d0 < nd; d0 += 8) {
        u32 in[8];
#pragma unroll
        for (int q = 0; q < 8; q++) in[q] = d0 + q < nd ? row[d0 + q] : 0u;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const u32 lo = acc, hi = acc + (in[q] & 0xFFFFu);
            acc = hi + (in[q] >> 16);
            if (d0 + q < nd) row[d0 + q] = (lo & 0xFFFFu) | (hi << 16);
        }
    }
}

// Item = pair p: the window before step 0 is all of A, whose median is A's
// item of sorted rank h; its merged position is stored in the spare entry
// pos[k] of the pair (k is odd, so the row has at least one spare entry).
MF_HD void pair_first_median(const Shape &s, const TileMem &m, int32_t p)
{
    const u32 t = m.sslot[(p << s.logS) + s.h] & (u32)(s.S - 1);
    const u32 *pos = m.pos + p * s.Pstride;
    m.pos[p * s.Pstride + s.k] = pos[t] & 0xFFFFu;
}

// ---------------------------------------------------------------- 5. walk

MF_HD int ctz32(u32 v) { return __builtin_ctz(v); }   // v != 0

// Lowest set bit and leading zeros of a 32-bit word, all ones for 0: one
// find-first-bit instruction each on the GPU (written out, so that the
// compiler does not rebuild the 64-bit forms below with extra selects).
MF_HD u32 ffbl32(u32 v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    u32 r;
    asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(v));
    return r;
#else
    return v == 0u ? 0xFFFFFFFFu : (u32)__builtin_ctz(v);
#endif
}
MF_HD u32 ffbh32(u32 v)
{
#if defined(__HIP_DEVICE_COMPILE__)
    u32 r;
    asm("v_ffbh_u32 %0, %1" : "=v"(r) : "v"(v));
    return r;
#else
    return v == 0u ? 0xFFFFFFFFu : (u32)__builtin_clz(v);
#endif
}

// Lowest set bit of v, or a value of 64 or more when v = 0.
MF_HD u32 low64_or_big(u64 v)
{
    const u32 a = ffbl32((u32)v), b = ffbl32((u32)(v >> 32)) | 32u;
    return a < b ? a : b;
}

// Highest set bit of v, or a value of 64 or more when v = 0.
MF_HD u32 high64_or_big(u64 v)
{
    const u32 a = ffbh32((u32)(v >> 32)), b = ffbh32((u32)v) | 32u;
    return 63u - (a < b ? a : b);
}

MF_HD int hibit32(u32 v)   // index of the highest set bit, v != 0
{
    return 31 - __builtin_clz(v);
}

// Membership dword of positions [32w, 32w+32) after step i, read from M with
// 16-byte loads (M rows are 64-byte aligned).  For an entry e = isB << 15 | t
// the 16-bit difference i - e has its sign bit set exactly when the item is a
// member after step i (A: t > i; B: t <= i; padding: never; i = -1 is the
// state before step 0), so one packed subtraction tests two positions.
MF_HD u32 member_dword(const Shape &s, const u16 *Mp, int32_t w, int32_t i)
{
    if (w < 0 || w >= m_dwords(s)) return 0u;
    const uint4 *src = (const uint4 *)(Mp + w * 32);
    const u32 ii = ((u32)i & 0xFFFFu) * 0x10001u;
    u32 word = 0u;
#pragma unroll
    for (int g = 0; g < 4; g++) {
        const uint4 v = src[g];
        word |= (psub16(ii, v.x) & 0x80008000u) >> (15 - 4 * g);
        word |= (psub16(ii, v.y) & 0x80008000u) >> (14 - 4 * g);
        word |= (psub16(ii, v.z) & 0x80008000u) >> (13 - 4 * g);
        word |= (psub16(ii, v.w) & 0x80008000u) >> (12 - 4 * g);
    }
    return word;
}

// The walk keeps the membership of 64 consecutive merged positions
// [base, base + 64) in one 64-bit register (base a multiple of 32, chosen so
// that the median starts at least 16 positions from either end).  Steps
// whose answer lies outside it take win_search_far, which reads membership
// from M, and then re-centre the window.

MF_HD u64 win_read(const Shape &s, const u16 *Mp, int32_t base, int32_t i)
{
    const int32_t d = base >> 5;
    return (u64)member_dword(s, Mp, d, i) | ((u64)member_dword(s, Mp, d + 1, i) << 32);
}

// Window base for median position r: r - base in [16, 48).
MF_HD int32_t win_base_for(int32_t r) { return ((r - 16) >> 5) << 5; }

// Next member strictly above r (dir > 0) or below r (dir < 0), searched
// dword by dword through M at step i (window bits are not needed: a dword
// of M read at step i already reflects every step).
MF_HD int32_t win_search_far(const Shape &s, const u16 *Mp, int32_t r, int32_t dir, int32_t i)
{
    int32_t q = r + dir;
    int32_t wq = q >> 5;
    u32 word = member_dword(s, Mp, wq, i);
    word &= (dir > 0) ? (0xFFFFFFFFu << (q & 31)) : (0xFFFFFFFFu >> (31 - (q & 31)));
#pragma unroll 1
    for (int32_t guard = 0; guard <= m_dwords(s) + 1; guard++) {
        if (word) return wq * 32 + (dir > 0 ? ctz32(word) : hibit32(word));
        wq += dir;
        if (wq < 0 || wq >= m_dwords(s)) return -1;
        word = member_dword(s, Mp, wq, i);
    }
    return -1;
}

// One step of a walk: A[i] leaves and B[i] joins the window (q = posA |
// posB << 16, their merged positions); the median's position base + rel
// and the membership window W of [base, base + 64) follow.  Sets bad (and
// leaves a placeholder) if a search runs off the merged order.
MF_HD void walk_step(const Shape &s, const u16 *Mp, u32 q, int32_t i, int32_t &base, int32_t &rel, u64 &W, int &bad)
{
    // A[i] leaves (its bit is set), B[i] joins (its bit is clear); bits
    // outside the window shift a zero
    const int32_t da = (int32_t)(q & 0xFFFFu) - base, db = (int32_t)(q >> 16) - base;
    W ^= (u64)((u32)da < 64u) << (da & 63);
    W ^= (u64)((u32)db < 64u) << (db & 63);
    // The median moves to the next member up when the window loses a
    // member at or below it (A[i] itself included) and gains one above
    // it, to the next member down when it gains one below and loses one
    // at or above it, and stays otherwise (B[i] was not a member, so it
    // is never at the median's position).
    const bool ltB = db < rel;
    const bool up = !ltB && da <= rel;
    const bool down = ltB && da >= rel;
    // the nearest member above and below (64 or more: none in the window)
    const u32 nup = low64_or_big(W & (~1ull << rel));
    const u32 ndn = high64_or_big(W & ((1ull << rel) - 1ull));
    u32 nrel = down ? ndn : (u32)rel;
    nrel = up ? nup : nrel;
    if (nrel >= 64u) {
        const int32_t dir = up ? 1 : -1;
        if (up ? rel >= 32 : rel < 32) {
            // the median drifts out of the window (sorted or slowly
            // varying input): slide the window half its width toward the
            // move, which keeps the half that holds it and reads one
            // membership dword
            if (up) {
                base += 32;
                rel -= 32;
                W = (W >> 32) | ((u64)member_dword(s, Mp, (base >> 5) + 1, i) << 32);
                nrel = low64_or_big(W & (~1ull << rel));
            } else {
                base -= 32;
                rel += 32;
                W = (W << 32) | (u64)member_dword(s, Mp, base >> 5, i);
                nrel = high64_or_big(W & ((1ull << rel) - 1ull));
            }
        }
        if (nrel >= 64u) {
            const int32_t nr = win_search_far(s, Mp, base + rel, dir, i);
            if (nr < 0) {
                bad = 1;
                base = 0;
                nrel = 0u;
            } else {
                base = win_base_for(nr);
                W = win_read(s, Mp, base, i);
                nrel = (u32)(nr - base);
            }
        }
    }
    rel = (int32_t)nrel;
}

// Walk of chunk c of pair p: steps [c*L, min((c+1)*L, len B)).  Returns 0,
// or -1 if a search ran off the merged order (cannot happen for a correct
// table; the bound keeps the loop finite).
MF_HD int walk_item(const Shape &s, const Tile &T, const TileMem &m, int32_t p, int32_t c)
{
    const int32_t lenB = block_len(s, T, p + 1);
    const int32_t i0 = c * s.L;
    const int32_t i1 = (i0 + s.L < lenB) ? i0 + s.L : lenB;
    const u16 *Mp = m.M + mul24((u32)p, (u32)s.Mstride);
    const u16 *pc = cnt_row(s, m, p, c);
    const u32 *pos = m.pos + mul24((u32)p, (u32)s.Pstride);
    u16 *stage = m.stage + mul24((u32)p, (u32)s.k);
    const int32_t h = s.h;

    // chunk 0 starts from A's median (pair_first_median); later chunks find
    // the rank-h member of the window before step i0 from the count table:
    // it lies in the largest word w with pc[w] <= h
    // (every lane runs the same membership reads, so that the lanes of a
    // wave, which start different chunks, do not diverge here)
    int32_t lo, r0 = 0;
    if (c == 0) {
        r0 = (int32_t)pos[s.k];
        lo = r0 >> 6;
    } else {
        lo = 0;
        int32_t hi = s.Wn;
        while (hi - lo > 1) {
            const int32_t mid = (lo + hi) >> 1;
            if ((int32_t)pc[mid] <= h) lo = mid;
            else hi = mid;
        }
    }
    const u32 dlo = member_dword(s, Mp, 2 * lo, i0 - 1);
    const u32 dhi = member_dword(s, Mp, 2 * lo + 1, i0 - 1);
    const u64 word = (u64)dlo | ((u64)dhi << 32);
    const int32_t below_lo = c == 0 ? 0 : (int32_t)pc[lo];   // members below word lo
    const int32_t r = c == 0 ? r0 : lo * 64 + select64(word, h - below_lo);

    // the window: word lo itself, or shifted half a word toward r when r
    // lies in its outer quarters (one more membership dword)
    int32_t base = win_base_for(r);
    const bool below = base < lo * 64;
    const u32 dx = member_dword(s, Mp, below ? 2 * lo - 1 : 2 * lo + 2, i0 - 1);
    u64 W = word;
    if (base != lo * 64) W = below ? (u64)dx | ((u64)dlo << 32) : (u64)dhi | ((u64)dx << 32);

    int bad = 0;
    int32_t rel = r - base;   // the median's bit in the window, in [0, 64)
    // the position words of the next four steps are in flight
    u32 q1 = pos[i0], q2 = i0 + 1 < i1 ? pos[i0 + 1] : 0u, q3 = i0 + 2 < i1 ? pos[i0 + 2] : 0u;
    u32 q4 = i0 + 3 < i1 ? pos[i0 + 3] : 0u;
#pragma unroll 1
    for (int32_t i = i0; i < i1; i++) {
        const u32 q = q1;
        q1 = q2;
        q2 = q3;
        q3 = q4;
        if (i + 4 < i1) q4 = pos[i + 4];
        walk_step(s, Mp, q, i, base, rel, W, bad);
        stage[i] = (u16)(base + rel);
    }
    if (bad)   // a failed search leaves a valid placeholder for the whole chunk
        for (int32_t q = i0; q < i1; q++) stage[q] = 0;
    return bad ? -1 : 0;
}

// ---------------------------------------------------------------- tail phases
//
// Thread tid's share (of NT threads) of each phase after the blocks are
// sorted; the kernel separates consecutive phases with barriers, the host
// check runs each phase for every tid in turn.


MF_HD void tail_first_medians(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    for (int32_t p = tid; p < T.P; p += NT) pair_first_median(s, m, p);
}

MF_HD void tail_table_zero(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    // 16-byte stores (the tables start 16-byte aligned), then the last words
    const int32_t nwords = T.P * s.C * s.Wrow / 2;
    const uint4 z = {0u, 0u, 0u, 0u};
    for (int32_t it = tid; it < (nwords >> 2); it += NT) ((uint4 *)m.cnt)[it] = z;
    for (int32_t it = (nwords & ~3) + tid; it < nwords; it += NT) table_zero_item(m, it);
}

MF_HD void tail_table_hist(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    const u32 Lr = recip32(s.L);
    const int32_t per = 2 * s.k;
    const u32 perr = recip32(per);
    for (int32_t it = tid; it < T.P * per; it += NT) {
        const int32_t p = (int32_t)udiv16((u32)it, perr), r = it - p * per;
        const int32_t lenB = block_len(s, T, p + 1);
        if (r < s.k + lenB) table_hist_item(s, m, p, r, Lr);
    }
}

// A barrier among the lanes of one wave: LDS written by any lane of the
// wave before it is visible to every lane after it.
MF_HD void wave_sync()
{
#if defined(__HIP_DEVICE_COMPILE__)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#endif
}

// The column pass as one phase: item = (pair p, row dword d, group g) with
// the kColGroups groups of a column on consecutive items, it = (p * Wd + d)
// * kColGroups + g, so that on the GPU they are neighbouring lanes of one
// wave.  Each lane sums its group's rows (A and B bytes of both cells), the
// lanes of a column exchange their totals (the A items of groups g.. and
// the B items of groups ..g-1) and each lane then writes its rows' member
// counts.  The host check, which runs one item at a time, handles a whole
// column at its group 0.
MF_HD void tail_table_columns(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    const int32_t stride = s.Wrow >> 1, R = col_rows(s), Wd = col_dwords(s);
    const u32 Wr = recip32(Wd);
    const int32_t total = T.P * Wd * kColGroups;
    for (int32_t it = tid; it < total; it += NT) {
        const int32_t g = it & (kColGroups - 1), pd = it / kColGroups;
        const int32_t p = (int32_t)udiv16((u32)pd, Wr), d = pd - p * Wd;
        u32 *col = (u32 *)cnt_row(s, m, p, 0) + d;
#if defined(__HIP_DEVICE_COMPILE__)
        const int32_t c0 = g * R, c1 = (c0 + R < s.C) ? c0 + R : s.C;
        u32 ta = 0u, tb = 0u;
        for (int32_t c = c0; c < c1; c++) {
            const u32 v = col[c * stride];
            ta += v & 0x00FF00FFu;
            tb += (v >> 8) & 0x00FF00FFu;
        }
        // inclusive prefix of the totals over the column's groups
        u32 ia = ta, ib = tb;
#pragma unroll
        for (int o = 1; o < kColGroups; o <<= 1) {
            const u32 ya = (u32)__shfl_up((int)ia, (unsigned)o, kColGroups);
            const u32 yb = (u32)__shfl_up((int)ib, (unsigned)o, kColGroups);
            if (g >= o) {
                ia += ya;
                ib += yb;
            }
        }
        const u32 all_a = (u32)__shfl((int)ia, kColGroups - 1, kColGroups);
        u32 sa = all_a - (ia - ta);   // A items of this and later groups
        u32 pb = ib - tb;             // B items of earlier groups
        for (int32_t c = c0; c < c1; c++) {
            const u32 v = col[c * stride];
            col[c * stride] = sa + pb;
            sa -= v & 0x00FF00FFu;
            pb += (v >> 8) & 0x00FF00FFu;
        }
#else
        if (g != 0) continue;
        u32 sa = 0u, pb = 0u;
        for (int32_t c = 0; c < s.C; c++) sa += col[c * stride] & 0x00FF00FFu;
        for (int32_t c = 0; c < s.C; c++) {
            const u32 v = col[c * stride];
            col[c * stride] = sa + pb;
            sa -= v & 0x00FF00FFu;
            pb += (v >> 8) & 0x00FF00FFu;
        }
#endif
    }
}

MF_HD void tail_table_rows(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    const u32 Cr = recip32(s.C);
    for (int32_t it = tid; it < T.P * s.C; it += NT) {
        const int32_t p = (int32_t)udiv16((u32)it, Cr), c = it - p * s.C;
        if (c < pair_chunks(s, T, p)) table_row_item(s, m, p, c);
    }
}

// Returns nonzero if a walk reported an inconsistency.
MF_HD int tail_walk(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    int bad = 0;
    const u32 Cr = recip32(s.C);
    for (int32_t it = tid; it < T.P * s.C; it += NT) {
        const int32_t p = (int32_t)udiv16((u32)it, Cr), c = it - p * s.C;
        if (c < pair_chunks(s, T, p)) bad |= walk_item(s, T, m, p, c) != 0;
    }
    return bad;
}

// ---------------------------------------------------------------- 4-5. one-pair tiles in global memory
//
// A tile of one pair with k > 4095 keeps its merged order and position maps
// in the workspace, and its count table counts members per column of
// kGcolWords words (1024 merged positions) instead of per word: C rows of
// gcols(s) cells.  The table is built in LDS (u32 cells: A items in the low
// half, B items in the high half; a column holds at most 1024 items, so the
// halves never carry), and its passes turn the cells into member
// counts.  A chunk's first median (chunk 0 included: the window before
// step 0 is all of A) is found in two steps: the column from the table row
// (the row pass), the word inside the column by counting membership words
// at the chunk start (the walk lane).  With the table this small, chunks
// can be short, which gives the walk a few hundred lanes per pair.

// Pointers into global memory in the global address space: reached through
// generic pointers, the workspace is accessed with flat instructions, which
// the compiler can only wait for together with the LDS operations around
// them (every load then costs a full round trip).
#if defined(__HIP_DEVICE_COMPILE__)
#define MF_GLOBAL __attribute__((address_space(1)))
#else
#define MF_GLOBAL
#endif
template <typename T>
MF_HD MF_GLOBAL T *gmem(T *p) { return (MF_GLOBAL T *)p; }

static const int32_t kGcolWords = 16;      // 64-position words per table column
static const int32_t kGcolShift = 10;      // log2 of the merged positions per column
static const int32_t kGcolGroups = 16;     // row groups per column in the column pass
static const int32_t kGchunkMax = 1024;    // walk chunks of a one-pair tile, at most

MF_HD int32_t gcols(const Shape &s) { return (s.Wn + kGcolWords - 1) / kGcolWords; }

// Walk chunks of a one-pair tile whose workgroup has lds bytes of dynamic
// LDS: at least 31 steps (a chunk's start costs a table search and a scan
// of up to kGcolWords membership words), and as many as the coarse table
// (C rows of gcols u32 cells, plus kGcolGroups rows of column-group totals)
// in that LDS allows, up to kGchunkMax.
MF_HD void global_chunks(Shape *s, int32_t lds)
{
    const int32_t G = gcols(*s);
    int32_t cmax = lds / (4 * G) - kGcolGroups;
    if (cmax > kGchunkMax) cmax = kGchunkMax;
    int32_t L = (s->k + cmax - 1) / cmax;
    if (L < 31) L = 31;
    s->L = L | 1;
    s->C = (s->k + s->L - 1) / s->L;
}

// Phase: zero the LDS table tb (C rows of gcols cells).
MF_HD void gtab_zero(const Shape &s, u32 *tb, int32_t tid, int32_t NT)
{
    const int32_t n = s.C * gcols(s);
    for (int32_t e = tid; e < n; e += NT) tb[e] = 0u;
}

// Phase: A's item t goes to cell (t / L, posA / 1024), B's item t (t < len
// B) to cell (t / L, posB / 1024) in the high half.
MF_HD void gtab_hist(const Shape &s, const Tile &T, const TileMem &m, u32 *tb, int32_t tid, int32_t NT)
{
    const int32_t G = gcols(s);
    const int32_t lenB = block_len(s, T, 1);
    const u32 Lr = recip32(s.L);
    const MF_GLOBAL u32 *pos = gmem(m.pos);
    for (int32_t t0 = tid; t0 < s.k; t0 += 4 * NT) {
        u32 q[4];
#pragma unroll
        for (int j = 0; j < 4; j++) q[j] = t0 + j * NT < s.k ? pos[t0 + j * NT] : 0u;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int32_t t = t0 + j * NT;
            if (t >= s.k) break;
            const u32 row = mul24(udiv16((u32)t, Lr), (u32)G);
            MF_ADD32(tb + row + ((q[j] & 0xFFFFu) >> kGcolShift), 1u);
            if (t < lenB) MF_ADD32(tb + row + (q[j] >> (16 + kGcolShift)), 0x10000u);
        }
    }
}

// Phase: item (column w, group g) sums its group's rows [g R, g R + R) of
// column w into gt[w * kGcolGroups + g] (R = ceil(C / kGcolGroups)).
MF_HD void gtab_col_sums(const Shape &s, const u32 *tb, u32 *gt, int32_t tid, int32_t NT)
{
    const int32_t G = gcols(s), R = (s.C + kGcolGroups - 1) / kGcolGroups;
    for (int32_t it = tid; it < G * kGcolGroups; it += NT) {
        const int32_t w = it / kGcolGroups, g = it - w * kGcolGroups;
        const int32_t c0 = g * R, c1 = c0 + R < s.C ? c0 + R : s.C;
        u32 acc = 0u;
        for (int32_t c = c0; c < c1; c++) acc += tb[c * G + w];
        gt[it] = acc;
    }
}

// Phase: cell (c, w) becomes the members of column w at chunk start c: A
// items with t >= cL (rows c..) plus B items with t < cL (rows ..c-1).
MF_HD void gtab_col_apply(const Shape &s, u32 *tb, const u32 *gt, int32_t tid, int32_t NT)
{
    const int32_t G = gcols(s), R = (s.C + kGcolGroups - 1) / kGcolGroups;
    for (int32_t it = tid; it < G * kGcolGroups; it += NT) {
        const int32_t w = it / kGcolGroups, g = it - w * kGcolGroups;
        const int32_t c0 = g * R, c1 = c0 + R < s.C ? c0 + R : s.C;
        u32 sa = 0u, pb = 0u;   // A items of groups g.., B items of groups ..g-1
        for (int32_t q = 0; q < kGcolGroups; q++) {
            const u32 v = gt[w * kGcolGroups + q];
            if (q >= g) sa += v & 0xFFFFu;
            else pb += v >> 16;
        }
        for (int32_t c = c0; c < c1; c++) {
            const u32 v = tb[c * G + w];
            tb[c * G + w] = sa + pb;
            sa -= v & 0xFFFFu;
            pb += v >> 16;
        }
    }
}

// Phase: for each row c, the column holding the rank-h member of the
// window before step cL: the largest w whose prefix over the columns
// (members among merged positions < 1024 w) is at most h, and that prefix,
// into info[c] = w | prefix << 16.
MF_HD void gtab_rows(const Shape &s, const u32 *tb, u32 *info, int32_t tid, int32_t NT)
{
    const int32_t G = gcols(s);
    const u32 h = (u32)s.h;
    for (int32_t c = tid; c < s.C; c += NT) {
        u32 acc = 0u, lo = 0u, below = 0u;
        for (int32_t w = 0; w < G; w++) {
            if (acc <= h) {
                lo = (u32)w;
                below = acc;
            }
            acc += tb[c * G + w];
        }
        info[c] = lo | (below << 16);
    }
}

// 64 membership bits of word w of the merged order at step i.
MF_HD u64 member_word(const Shape &s, const u16 *Mp, int32_t w, int32_t i)
{
    return (u64)member_dword(s, Mp, 2 * w, i) | ((u64)member_dword(s, Mp, 2 * w + 1, i) << 32);
}

// Walk of chunk c of a one-pair tile: steps [c*L, min((c+1)*L, len B)),
// with AHEAD position words in flight.  The rank-h member of the
// window before step cL (chunk 0 included: that window is all of A) lies
// in column info[c]: the words of that column are counted up to the one
// that holds it.  Chunk 0 of the first tile writes output 0 (the median of
// block 0).  Returns 0, or -1 as walk_item does.
template <int AHEAD, typename V>
MF_HD int gwalk_item(const Shape &s, const Tile &T, const TileMem &m, const u32 *info, int32_t c, const V *x,
                     V *y, int32_t *argmed)
{
    const int32_t lenB = block_len(s, T, 1);
    const int32_t i0 = c * s.L;
    const int32_t i1 = (i0 + s.L < lenB) ? i0 + s.L : lenB;
    const u16 *Mp = m.M;
    const MF_GLOBAL u32 *pos = gmem(m.pos);
    MF_GLOBAL u16 *stage = gmem(m.stage);
    const int32_t h = s.h;

    const u32 inf = info[c];
    int32_t lo = (int32_t)(inf & 0xFFFFu) * kGcolWords;
    int32_t below = (int32_t)(inf >> 16);
    const int32_t lend = ((lo + kGcolWords < s.Wn) ? lo + kGcolWords : s.Wn) - 1;
    u64 word = member_word(s, Mp, lo, i0 - 1);
#pragma unroll 1
    while (lo < lend) {
        const int32_t n = popc64(word);
        if (below + n > h) break;
        below += n;
        lo++;
        word = member_word(s, Mp, lo, i0 - 1);
    }
    const int32_t r = lo * 64 + select64(word, h - below);
    if (c == 0 && T.j0 == 1) {
        const u32 e = m_entry(Mp, (u32)r);
        y[0] = x[e];
        if (argmed) argmed[0] = (int32_t)e;
    }

    // the window, as in walk_item: word lo, or shifted half a word toward r
    int32_t base = win_base_for(r);
    const bool bel = base < lo * 64;
    const u32 dx = member_dword(s, Mp, bel ? 2 * lo - 1 : 2 * lo + 2, i0 - 1);
    u64 W = word;
    if (base != lo * 64) W = bel ? (u64)dx | (word << 32) : (word >> 32) | ((u64)dx << 32);

    int bad = 0;
    int32_t rel = r - base;
    // steps in groups of AHEAD, unrolled: slot j of the ring is read only
    // by its own step and then refilled for the step AHEAD on
    // (moving an in-flight register would wait for its load), and every
    // load is unconditional (an index past the chunk reads its last word),
    // so that the compiler waits for exactly the load a step needs
    const int32_t ilast = i1 - 1;
    u32 qr[AHEAD];
#pragma unroll
    for (int j = 0; j < AHEAD; j++) qr[j] = pos[i0 + j < ilast ? i0 + j : ilast];
#pragma unroll 1
    for (int32_t i = i0; i < i1; i += AHEAD) {
#pragma unroll
        for (int j = 0; j < AHEAD; j++) {
            const u32 q = qr[j];
            const int32_t nx = i + j + AHEAD;
            qr[j] = pos[nx < ilast ? nx : ilast];
            if (i + j < i1) {
                walk_step(s, Mp, q, i + j, base, rel, W, bad);
                stage[i + j] = (u16)(base + rel);
            }
        }
    }
    if (bad)
        for (int32_t q = i0; q < i1; q++) stage[q] = 0;
    return bad ? -1 : 0;
}

template <int AHEAD, typename V>
MF_HD int gtail_walk(const Shape &s, const Tile &T, const TileMem &m, const u32 *info, int32_t tid, int32_t NT,
                     const V *x, V *y, int32_t *argmed)
{
    int bad = 0;
    for (int32_t c = tid; c < T.Clast; c += NT) bad |= gwalk_item<AHEAD>(s, T, m, info, c, x, y, argmed) != 0;
    return bad;
}

// Output of a one-pair tile (tail_output with the staged medians in the
// workspace and M in LDS; x, y and argmed in global memory): output it of
// the tile is o0 + it, it < len B, with every gather issued before the
// first store.
template <typename V>
MF_HD void gtail_output(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT, const V *x,
                        V *y, int32_t *argmed)
{
    const MF_GLOBAL u16 *stage = gmem((const u16 *)m.stage);
    const MF_GLOBAL V *xt = gmem(x + T.e0);
    MF_GLOBAL V *yt = gmem(y + T.o0);
    MF_GLOBAL int32_t *at = argmed ? gmem(argmed + T.o0) : nullptr;
    const int32_t e0 = (int32_t)T.e0;
    const int32_t nout = T.lenLast;
    for (int32_t base = 0; base < nout; base += NT * kRegs) {
        V v[kRegs];
        u32 g[kRegs];
#pragma unroll
        for (int j = 0; j < kRegs; j++) {
            const int32_t it = base + j * NT + tid;
            g[j] = 0u;
            v[j] = 0;
            if (it < nout) {
                const u32 e = m_entry(m.M, (u32)stage[it]);
                g[j] = mul24(e >> 15, (u32)s.k) + (e & 0x7FFFu);
                v[j] = xt[g[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < kRegs; j++) {
            const int32_t it = base + j * NT + tid;
            if (it < nout) {
                yt[it] = v[j];
                if (at) at[it] = e0 + (int32_t)g[j];
            }
        }
    }
}

// ---------------------------------------------------------------- 6. output

// Number of outputs written by a tile: sum of len(B) over its pairs, plus
// output 0 (the median of block 0) for the first tile.
MF_HD int64_t tile_outputs(const Shape &s, const Tile &T)
{
    int64_t cnt = 0;
    if (T.P > 0) cnt = (int64_t)(T.P - 1) * s.k + block_len(s, T, T.P);
    return cnt;
}

template <typename V>
MF_HD void tail_output(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT,
                       const V *x, V *y, int32_t *argmed)
{
    // the tile's outputs are o0 + it for it = p*k + i, it < (P-1)k + len of
    // the last block; every gather is issued before the first store
    const V *xt = x + T.e0;
    V *yt = y + T.o0;
    int32_t *at = argmed ? argmed + T.o0 : nullptr;
    const int32_t e0 = (int32_t)T.e0;
    const int32_t nout = (T.P - 1) * s.k + T.lenLast;
    const u32 kr = recip32(s.k);
    // addresses are 32-bit byte offsets from the tile's bases (a tile spans
    // far less than 4 GB), so that the loads and stores take the
    // scalar-base form without 64-bit address arithmetic per lane
    const unsigned char *xb = (const unsigned char *)xt;
    unsigned char *yb = (unsigned char *)yt, *ab = (unsigned char *)at;
    for (int32_t base = 0; base < nout; base += NT * kRegs) {
        V v[kRegs];
        u32 g[kRegs];
#pragma unroll
        for (int j = 0; j < kRegs; j++) {
            const int32_t it = base + j * NT + tid;
            g[j] = 0u;
            v[j] = 0;
            if (it < nout) {
                const u32 p = udiv16((u32)it, kr);
                const int32_t r = m.stage[it];
                const u32 e = m_entry(m.M + mul24(p, (u32)s.Mstride), (u32)r);
                g[j] = mul24(p + (e >> 15), (u32)s.k) + (e & 0x7FFFu);
                v[j] = *(const V *)(xb + g[j] * (u32)sizeof(V));
            }
        }
#pragma unroll
        for (int j = 0; j < kRegs; j++) {
            const int32_t it = base + j * NT + tid;
            if (it < nout) {
                *(V *)(yb + (u32)it * (u32)sizeof(V)) = v[j];
                if (at) *(int32_t *)(ab + (u32)it * 4u) = e0 + (int32_t)g[j];
            }
        }
    }
}

// Output 0: the median of block 0 (Section 3: Y_0's only element).
template <typename V>
MF_HD void output_first(const Shape &s, const Tile &T, const TileMem &m, const V *x, V *y, int32_t *argmed)
{
    const int32_t t = (int32_t)(m.sslot[s.h] & (u32)(s.S - 1));
    y[0] = x[t];
    if (argmed) argmed[0] = t;
}

// Thread tid's share of the pair orders (phase 3) and output 0.
MF_HD void tail_pair_pad(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT)
{
    const int32_t ipp = pad_items_per_pair(s);
    const u32 ir = recip32(ipp);
    for (int32_t it = tid; it < T.P * ipp; it += NT) {
        const int32_t p = (int32_t)udiv16((u32)it, ir);
        pair_pad_item(s, T, m, p, it - p * ipp);
    }
}

template <typename V>
MF_HD void tail_pair_merge(const Shape &s, const Tile &T, const TileMem &m, int32_t tid, int32_t NT,
                           const V *x, V *y, int32_t *argmed)
{
    const int32_t ipp = merge_items_per_pair(s);
    const u32 ir = recip32(ipp);
    for (int32_t it = tid; it < T.P * ipp; it += NT) {
        const int32_t p = (int32_t)udiv16((u32)it, ir);
        pair_merge_item(s, T, m, p, it - p * ipp);
    }
    if (T.j0 == 1 && tid == 0) output_first(s, T, m, x, y, argmed);
}

// ---------------------------------------------------------------- 64-bit inputs
//
// The tile phases compare 32-bit keys.  A 64-bit signal (Section 7 measures
// 32- and 64-bit versions) first has each tile's items ranked by (64-bit
// key, index): a total order without ties.  The ranks (kept in the tile's
// LDS, or written tile by tile, (Pmax + 1) k entries per tile, so that a
// block shared by two tiles appears in both) are 32-bit keys that order
// every tile's items exactly as the 64-bit values with the index tie-break
// do; the 32-bit tile phases then run on them unchanged and produce the
// 64-bit signal's argmed.
//
// The ranking is one merge sort of (key, slot) pairs, slots being item
// offsets from the tile's first item (at most kRegs * threads).  A thread
// starts with kRegs consecutive slots, sorted in registers by (key, slot);
// the merges are stable (ties take the left run, whose slots are all
// smaller), so every run stays in (key, slot) order.

// Order-preserving unsigned key of a double: -0.0 as +0.0, every NaN above
// +inf (all NaNs equal).
MF_HD u64 key_of_f64(u64 u)
{
    if ((u & 0x7FFFFFFFFFFFFFFFull) > 0x7FF0000000000000ull) return ~0ull;
    if (u == 0x8000000000000000ull) u = 0ull;
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

MF_HD u64 key_of_i64(u64 u) { return u ^ 0x8000000000000000ull; }

// Keys and slots of thread tid over the span items at xt: slots
// tid*kRegs + j; slots past the span get the largest key (their slots order
// them after every item).
template <bool F64>
MF_HD void rank64_load(const u64 *xt, int32_t span, int32_t tid, u64 (&kv)[kRegs], u32 (&sv)[kRegs])
{
    const int32_t i0 = tid * kRegs;
    const u64 *src = xt + i0;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        sv[j] = (u32)(i0 + j);
        kv[j] = ~0ull;
        if (i0 + j < span) kv[j] = F64 ? key_of_f64(src[j]) : key_of_i64(src[j]);
    }
}

MF_HD void cswap_ks(u64 &ka, u32 &sa, u64 &kb, u32 &sb, bool up)
{
    const bool gt = ka > kb || (ka == kb && sa > sb);
    const bool sw = up ? gt : !gt;
    const u64 k0 = sw ? kb : ka, k1 = sw ? ka : kb;
    const u32 s0 = sw ? sb : sa, s1 = sw ? sa : sb;
    ka = k0; kb = k1; sa = s0; sb = s1;
}

// Bitonic sort of the thread's kRegs pairs by (key, slot), ascending.
MF_HD void sort_regs_ks(u64 (&kv)[kRegs], u32 (&sv)[kRegs])
{
#pragma unroll
    for (int size = 2; size <= kRegs; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
#pragma unroll
            for (int i = 0; i < kRegs; i++) {
                const int j = i ^ stride;
                if (j > i) cswap_ks(kv[i], sv[i], kv[j], sv[j], (i & size) == 0);
            }
        }
    }
}

// One stable merge-path level over keys K and slots S (runs of length w):
// thread tid produces sorted positions [tid*kRegs, tid*kRegs + kRegs).
MF_HD void merge_level_ks(const u64 *K, const u16 *S, int32_t w, int32_t tid, u64 (&ko)[kRegs],
                          u32 (&so)[kRegs])
{
    const int32_t first = tid * kRegs;
    const int32_t s0 = first & ~(2 * w - 1);
    const u64 *A = K + s0, *B = K + s0 + w;
    const u16 *SA = S + s0, *SB = S + s0 + w;
    const int32_t d = first - s0;
    int32_t lo = d > w ? d - w : 0;
    int32_t hi = d < w ? d : w;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[d - 1 - mid]) lo = mid + 1;
        else hi = mid;
    }
    int32_t a = lo, b = d - lo;
    u64 va = a < w ? A[a] : 0ull, vb = b < w ? B[b] : 0ull;
    u32 sa = a < w ? SA[a] : 0u, sb = b < w ? SB[b] : 0u;
#pragma unroll
    for (int q = 0; q < kRegs; q++) {
        const bool takeA = (b >= w) || (a < w && va <= vb);
        ko[q] = takeA ? va : vb;
        so[q] = takeA ? sa : sb;
        if (takeA) {
            a++;
            va = a < w ? A[a] : 0ull;
            sa = a < w ? SA[a] : 0u;
        } else {
            b++;
            vb = b < w ? B[b] : 0ull;
            sb = b < w ? SB[b] : 0u;
        }
    }
}

// Rank of each item: its position in the sorted order (the thread holds
// positions tid*kRegs + j).
MF_HD void rank64_ranks(int32_t span, int32_t tid, const u32 (&sv)[kRegs], u32 *rank)
{
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if ((int32_t)sv[j] < span) rank[sv[j]] = (u32)(tid * kRegs + j);
}

// Common path of the ranking: a bucket sort.  The tile's keys are spread
// over cap buckets by their top bits above the tile's minimum key, counted
// (16-bit counters, two to an LDS word), scanned, scattered in bucket order
// and ranked within their bucket by (key, slot).  A tile with a bucket of
// kRank64BucketMax or more items (heavy ties, clustered keys) takes the
// merge sort instead.
static const u32 kRank64BucketMax = 32;

// The thread's key range over its items (lo = ~0, hi = 0 if none).
MF_HD void rank64_range(int32_t span, const u64 (&kv)[kRegs], const u32 (&sv)[kRegs], u64 &lo, u64 &hi)
{
    lo = ~0ull;
    hi = 0ull;
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if ((int32_t)sv[j] < span) {
            lo = kv[j] < lo ? kv[j] : lo;
            hi = kv[j] > hi ? kv[j] : hi;
        }
}

// Shift mapping [lo, hi] onto 2^lognb buckets: (key - lo) >> sh.
MF_HD u32 rank64_shift(u64 lo, u64 hi, int32_t lognb)
{
    const u64 r = hi - lo;
    const int32_t bits = r ? hibit64(r) + 1 : 0;
    return bits > lognb ? (u32)(bits - lognb) : 0u;
}

MF_HD u32 rank64_bucket(u64 key, u64 lo, u32 sh) { return (u32)((key - lo) >> sh); }

// 16-bit counter b of the packed array C (two per word).
MF_HD u32 cnt16(const u32 *C, u32 b) { return (C[b >> 1] >> ((b & 1u) << 4)) & 0xFFFFu; }

// Arrival numbers of the thread's items in their buckets; true if one
// reaches kRank64BucketMax.
MF_HD bool rank64_count(int32_t span, const u64 (&kv)[kRegs], const u32 (&sv)[kRegs], u64 lo, u32 sh,
                        u32 *C, u32 (&arr)[kRegs])
{
    bool full = false;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        arr[j] = 0u;
        if ((int32_t)sv[j] < span) {
            const u32 b = rank64_bucket(kv[j], lo, sh);
            const u32 sft = (b & 1u) << 4;
            arr[j] = (MF_ADDRTN32(C + (b >> 1), 1u << sft) >> sft) & 0xFFFFu;
            full = full || arr[j] >= kRank64BucketMax;
        }
    }
    return full;
}

// Bucket counts of thread tid (buckets tid*kRegs .. +kRegs) into their
// exclusive prefix within the thread; returns the thread's total.
MF_HD u32 rank64_scan_local(const u32 *C, int32_t tid, u32 (&c)[kRegs])
{
    u32 run = 0u;
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const u32 v = cnt16(C, (u32)(tid * kRegs + j));
        c[j] = run;
        run += v;
    }
    return run;
}

// Bucket starts (16-bit, packed) from the thread's prefix and its offset.
MF_HD void rank64_scan_store(u32 *C, int32_t tid, u32 excl, const u32 (&c)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j += 2)
        C[(tid * kRegs + j) >> 1] = ((excl + c[j]) & 0xFFFFu) | ((excl + c[j + 1]) << 16);
}

// Items into bucket order: keys to K, slots to S.
MF_HD void rank64_scatter(int32_t span, const u64 (&kv)[kRegs], const u32 (&sv)[kRegs], u64 lo, u32 sh,
                          const u32 *C, const u32 (&arr)[kRegs], u64 *K, u16 *S)
{
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if ((int32_t)sv[j] < span) {
            const u32 pos = cnt16(C, rank64_bucket(kv[j], lo, sh)) + arr[j];
            K[pos] = kv[j];
            S[pos] = (u16)sv[j];
        }
}

// Sorted position of each item: its bucket's start plus the bucket's items
// below it by (key, slot); nb buckets, the last ending at span.
MF_HD void rank64_bucket_rank(int32_t span, const u64 (&kv)[kRegs], const u32 (&sv)[kRegs], u64 lo, u32 sh,
                              const u32 *C, u32 nb, const u64 *K, const u16 *S, u32 (&fin)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        fin[j] = 0u;
        if ((int32_t)sv[j] < span) {
            const u32 b = rank64_bucket(kv[j], lo, sh);
            const u32 st = cnt16(C, b);
            const u32 en = b + 1u < nb ? cnt16(C, b + 1u) : (u32)span;
            u32 below = 0u;
            for (u32 e = st; e < en; e++) {
                const u64 ke = K[e];
                below += (ke < kv[j] || (ke == kv[j] && (u32)S[e] < sv[j])) ? 1u : 0u;
            }
            fin[j] = st + below;
        }
    }
}

// rank[slot] = sorted position, for the thread's items.
MF_HD void rank64_place(int32_t span, const u32 (&sv)[kRegs], const u32 (&fin)[kRegs], u32 *rank)
{
#pragma unroll
    for (int j = 0; j < kRegs; j++)
        if ((int32_t)sv[j] < span) rank[sv[j]] = fin[j];
}

// The rank keys of thread tid's slots, as load_raw gives a tile's inputs,
// from the tile's ranks by item offset (rank64_place / rank64_ranks).
MF_HD void rank_raw(const Shape &s, const Tile &T, const u32 *rank, int32_t tid, u32 (&raw)[kRegs])
{
#pragma unroll
    for (int j = 0; j < kRegs; j++) {
        const int32_t u = tid * kRegs + j;
        const int32_t b = u >> s.logS, t = u & (s.S - 1);
        const int32_t len = b < T.NB ? block_len(s, T, b) : 0;
        raw[j] = t < len ? rank[b * s.k + t] : 0u;
    }
}

// Ranks of a pair of more than NT * kRegs items (windows above 4095): the
// pair is cut into chunks of that many items, each chunk is ranked in LDS
// and written in sorted order (key, offset), and merge levels combine the
// sorted runs in global memory, one output tile of NT * kRegs items at a
// time: merge path at the tile's first and last output gives the tile's
// input range of each run, both ranges are staged in LDS, and each thread
// merges kRegs outputs from there.
//
// The number of A items among the first d outputs of the merge of runs A
// and B ((key, offset) pairs, all distinct).
MF_HD int32_t merge_split_ko(const u64 *KA, const u32 *OA, int32_t lenA, const u64 *KB, const u32 *OB,
                             int32_t lenB, int32_t d)
{
    int32_t lo = d > lenB ? d - lenB : 0;
    int32_t hi = d < lenA ? d : lenA;
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        const int32_t bm = d - 1 - mid;
        const u64 ka = KA[mid], kb = KB[bm];
        if (ka < kb || (ka == kb && OA[mid] < OB[bm])) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Thread outputs [q0, q0 + kRegs) (fewer at the end) of the merge of the
// staged runs LK/LO[0, na) and LK/LO[na, na + nb); returns their number.
MF_HD int32_t merge_local_ko(const u64 *LK, const u32 *LO, int32_t na, int32_t nb, int32_t q0,
                             u64 (&kv)[kRegs], u32 (&ov)[kRegs])
{
    const int32_t tot = na + nb;
    if (q0 >= tot) return 0;
    int32_t a = merge_split_ko(LK, LO, na, LK + na, LO + na, nb, q0);
    int32_t b = q0 - a;
    const u64 *KB = LK + na;
    const u32 *OB = LO + na;
    const int32_t cnt = tot - q0 < kRegs ? tot - q0 : kRegs;
#pragma unroll
    for (int q = 0; q < kRegs; q++) {
        if (q >= cnt) break;
        const bool takeA = b >= nb || (a < na && (LK[a] < KB[b] || (LK[a] == KB[b] && LO[a] < OB[b])));
        kv[q] = takeA ? LK[a] : KB[b];
        ov[q] = takeA ? LO[a] : OB[b];
        if (takeA) a++;
        else b++;
    }
    return cnt;
}

// The runs of the merge that output position ob belongs to: start s0 and
// lengths of A = [s0, s0 + lenA) and B = [s0 + w, s0 + w + lenB).
MF_HD void merge_runs(int32_t span, int32_t w, int32_t ob, int32_t &s0, int32_t &lenA, int32_t &lenB)
{
    s0 = ob & ~(2 * w - 1);
    const int32_t rest = span - s0;
    lenA = rest < w ? rest : w;
    lenB = rest - lenA < w ? rest - lenA : w;
}

// Scratch bytes of one workgroup ranking a pair of window k: two copies of
// (key, offset) for 2k items.
MF_HD int64_t pair_rank_scratch(int32_t k) { return ((24ll * 2 * k) + 255) & ~255ll; }

// Entries per tile of the rank buffer.
MF_HD int64_t rank64_stride(const Shape &s) { return (int64_t)(s.Pmax + 1) * s.k; }

}  // namespace mf
