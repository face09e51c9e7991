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
//   1. load      x -> xv (raw 32-bit patterns), block b at slot b*S.
//   2. sort      each block sorted by (key, t): packed u64 values
//                (block << 48 | key << 16 | t), bitonic-16 in registers,
//                then merge-path levels of run length 16, 32, .., S/2.
//                Packing the local index t makes every value distinct, so
//                the sort is stable in the sense of Section 5.2.
//   3. pair merge  for each pair, the merged order of A and B by
//                (key, A-before-B, t) -> M[r] = isB << 15 | t, and the
//                merged positions posA[t], posB[t].
//   4. tables    membership words of the merged order at the start of each
//                walk chunk (steps c*L), by XOR of the flips of earlier
//                steps, plus prefix popcounts.
//   5. walk      one lane per chunk of L steps: the window of step i is
//                A[i+1..] u B[..i] (Section 3 "Postprocessing").  In merged
//                order, position r is a member after step i iff
//                (isA and t > i) or (isB and t <= i).  Step i removes
//                A[i] and adds B[i]; the rank-h member then moves to the
//                next or previous member, or stays: this is the block
//                structures' cursor update (Section 5.3) and rebalancing
//                (Section 6.2) with both cursors folded into one position
//                of the merged order.  A 128-bit register window of
//                membership bits around the median is kept up to date.
//   6. output    y[o] = x[argmed[o]] (bit copy), argmed[o] global index.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MF_HD __host__ __device__ __forceinline__
#else
#define MF_HD static inline
#endif

namespace mf {

typedef uint64_t u64;
typedef uint32_t u32;
typedef uint16_t u16;

static const u64 kPadAll = ~0ull;          // slot beyond the tile's blocks
static const u32 kMPad = 0xFFFFu;          // merged-order padding: never a member
static const int kRegs = 16;               // sort values per thread
static const int32_t kPairBudget = 48 * 1024; // bytes of M + pos per tile

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
    int32_t L;       // walk chunk length (multiple of 64)
    int32_t C;       // chunks of a full pair, ceil(k / L)
    int32_t Wn;      // 64-position words of a pair's merged order, ceil(2k/64)
    int32_t Mstride; // u16 entries per pair in M (= Wn * 64)
};

// LDS (or scratch) layout of a tile, in bytes from the base.
struct Layout {
    int32_t xv;      // u32[cap]
    int32_t srt;     // u64[cap]
    int32_t M;       // u16[Pmax * Mstride]
    int32_t pos;     // u32[Pmax * k]     posA | posB << 16
    int32_t words;   // u64[Pmax * C * Wn]         (aliases srt)
    int32_t pc;      // u16[Pmax * C * (Wn + 1)]   (aliases srt)
    int32_t stage;   // u16[Pmax * k]              (aliases srt)
    int32_t total;   // bytes
};

MF_HD int32_t ceil_div32(int64_t a, int64_t b) { return (int32_t)((a + b - 1) / b); }

// Fills s for window k over n items with `threads` threads per tile.
// Returns 0, or -1 when k does not fit this capacity (two blocks needed).
MF_HD int make_shape(int64_t n, int32_t k, int32_t threads, Shape *s)
{
    s->n = n;
    s->k = k;
    s->h = (k - 1) / 2;
    int32_t S = 1, logS = 0;
    while (S < k) { S <<= 1; logS++; }
    s->S = S;
    s->logS = logS;
    s->cap = threads * kRegs;
    if (2 * S > s->cap) return -1;
    // chunk length: a multiple of 64 keeping at most 16 chunks per pair
    int32_t L = 64;
    while ((k + L - 1) / L > 16) L += 64;
    s->L = L;
    s->C = ceil_div32(k, L);
    s->Wn = ceil_div32(2 * (int64_t)k, 64);
    s->Mstride = s->Wn * 64;
    // pairs per tile: as many blocks as the sort holds, but the merged
    // orders and position maps of all pairs stay within kPairBudget bytes
    int32_t P = s->cap / S - 1;
    const int32_t per_pair = 2 * s->Mstride + 4 * k + 16;
    if (P * per_pair > kPairBudget) P = kPairBudget / per_pair;
    if (P < 1) P = 1;
    s->Pmax = P;
    s->nblocks = (n + k - 1) / k;
    s->npairs = s->nblocks - 1;
    s->ntiles = s->npairs > 0 ? (s->npairs + s->Pmax - 1) / s->Pmax : 1;
    return 0;
}

MF_HD void make_layout(const Shape &s, Layout *l)
{
    int32_t off = 0;
    l->xv = off;     off += 4 * s.cap;
    l->srt = off;    off += 8 * s.cap;
    l->M = off;      off += 2 * s.Pmax * s.Mstride;
    off = (off + 15) & ~15;
    l->pos = off;    off += 4 * s.Pmax * s.k;
    off = (off + 15) & ~15;
    l->total = off;
    int32_t a = l->srt;
    l->words = a;    a += 8 * s.Pmax * s.C * s.Wn;
    l->pc = a;       a += 2 * s.Pmax * s.C * (s.Wn + 1);
    a = (a + 15) & ~15;
    l->stage = a;    a += 2 * s.Pmax * s.k;
    if (a > l->srt + 8 * s.cap) l->total = -1;   // aliased region overflows
}

// The tile of pairs [j0, j0 + P).
struct Tile {
    int64_t j0;      // first pair (>= 1)
    int32_t P;       // pairs (0 only for a single-block signal)
    int32_t NB;      // blocks = P + 1
    int64_t e0;      // global index of the first element of the tile
    int64_t o0;      // first output index written by the pairs: (j0-1)k + 1
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
    return T;
}

MF_HD int32_t block_len(const Shape &s, const Tile &T, int32_t b)
{
    int64_t start = T.e0 + (int64_t)b * s.k;
    int64_t rem = s.n - start;
    return (int32_t)(rem < s.k ? rem : s.k);
}

// ---------------------------------------------------------------- views

struct TileMem {
    u32 *xv;
    u64 *srt;
    u16 *M;
    u32 *pos;
    u64 *words;
    u16 *pc;
    u16 *stage;
};

MF_HD TileMem tile_mem(unsigned char *base, const Layout &l)
{
    TileMem m;
    m.xv = (u32 *)(base + l.xv);
    m.srt = (u64 *)(base + l.srt);
    m.M = (u16 *)(base + l.M);
    m.pos = (u32 *)(base + l.pos);
    m.words = (u64 *)(base + l.words);
    m.pc = (u16 *)(base + l.pc);
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

// ---------------------------------------------------------------- 3. pair merge

// Sort values carry the key in bits 16..47 and t in bits 0..15.
MF_HD u32 sv_key(u64 v) { return (u32)(v >> 16); }
MF_HD u32 sv_t(u64 v) { return (u32)(v & 0xFFFFu); }

static const int kMergeSeg = 32;   // merged outputs per pair-merge item

MF_HD int32_t merge_items_per_pair(const Shape &s) { return s.Mstride / kMergeSeg; }

// Item = (pair p, segment g): merged positions [g*32, g*32 + 32) of pair p.
MF_HD void pair_merge_item(const Shape &s, const Tile &T, const TileMem &m,
                           int32_t p, int32_t g)
{
    const int32_t lenA = s.k;
    const int32_t lenB = block_len(s, T, p + 1);
    const int32_t mlen = lenA + lenB;
    const u64 *A = m.srt + ((int32_t)p << s.logS);
    const u64 *B = m.srt + ((int32_t)(p + 1) << s.logS);
    u16 *Mp = m.M + p * s.Mstride;
    u32 *pos = m.pos + p * s.k;
    const int32_t d = g * kMergeSeg;
    int32_t lo = d > lenB ? d - lenB : 0;
    int32_t hi = d < lenA ? d : lenA;
    if (d >= mlen) {   // padding of the merged order
        for (int q = 0; q < kMergeSeg; q++) Mp[d + q] = (u16)kMPad;
        return;
    }
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        // A[mid] precedes B[d-1-mid] iff keyA <= keyB (A first on ties)
        if (sv_key(A[mid]) <= sv_key(B[d - 1 - mid])) lo = mid + 1;
        else hi = mid;
    }
    int32_t a = lo, b = d - lo;
    for (int q = 0; q < kMergeSeg; q++) {
        const int32_t r = d + q;
        if (r >= mlen) { Mp[r] = (u16)kMPad; continue; }
        bool takeA;
        if (a >= lenA) takeA = false;
        else if (b >= lenB) takeA = true;
        else takeA = sv_key(A[a]) <= sv_key(B[b]);
        if (takeA) {
            const u32 t = sv_t(A[a++]);
            Mp[r] = (u16)t;
            ((u16 *)(pos + t))[0] = (u16)r;          // posA (low half)
        } else {
            const u32 t = sv_t(B[b++]);
            Mp[r] = (u16)(0x8000u | t);
            ((u16 *)(pos + t))[1] = (u16)r;          // posB (high half)
        }
    }
}

// ---------------------------------------------------------------- 4. tables

MF_HD int32_t pair_chunks(const Shape &s, const Tile &T, int32_t p)
{
    return ceil_div32(block_len(s, T, p + 1), s.L);
}

// Membership word of positions [64w, 64w+64) of pair p after step i
// (i = -1: before the first step, when the window is all of A).
MF_HD u64 member_word(const Shape &s, const u16 *Mp, int32_t w, int32_t i)
{
    if (w < 0 || w >= s.Wn) return 0ull;
    u64 word = 0ull;
    const u16 *e = Mp + w * 64;
    for (int q = 0; q < 64; q++) {
        const int32_t v = e[q];
        const int32_t t = v & 0x7FFF;
        const bool mem = (v & 0x8000) ? (t <= i) : (t > i);
        word |= (u64)mem << q;
    }
    return word;
}

// Item = (pair p, word w): chunk 0 gets the word before step 0, later
// chunks start from zero (flips are XORed in, then prefix-XORed).
MF_HD void table_init_item(const Shape &s, const TileMem &m, int32_t p, int32_t w)
{
    u64 *W = m.words + (int64_t)p * s.C * s.Wn;
    W[w] = member_word(s, m.M + p * s.Mstride, w, -1);
    for (int c = 1; c < s.C; c++) W[c * s.Wn + w] = 0ull;
}

#if defined(__HIP_DEVICE_COMPILE__)
#define MF_XOR64(ptr, v) atomicXor((unsigned long long *)(ptr), (unsigned long long)(v))
#else
#define MF_XOR64(ptr, v) (*(ptr) ^= (v))
#endif

// Item = (pair p, step i): the flips of step i reach every chunk starting
// after it.  They are accumulated in chunk c = i/L + 1.
MF_HD void table_flip_item(const Shape &s, const Tile &T, const TileMem &m, int32_t p, int32_t i)
{
    const int32_t c = i / s.L + 1;
    if (c >= pair_chunks(s, T, p)) return;
    u64 *W = m.words + ((int64_t)p * s.C + c) * s.Wn;
    const u32 pab = m.pos[p * s.k + i];
    const u32 pa = pab & 0xFFFFu, pb = pab >> 16;
    MF_XOR64(W + (pa >> 6), 1ull << (pa & 63));
    MF_XOR64(W + (pb >> 6), 1ull << (pb & 63));
}

// Item = (pair p, word w): prefix XOR over the chunks.
MF_HD void table_prefix_item(const Shape &s, const Tile &T, const TileMem &m, int32_t p, int32_t w)
{
    u64 *W = m.words + (int64_t)p * s.C * s.Wn;
    const int32_t C = pair_chunks(s, T, p);
    u64 acc = W[w];
    for (int c = 1; c < C; c++) {
        acc ^= W[c * s.Wn + w];
        W[c * s.Wn + w] = acc;
    }
}

// Item = (pair p, chunk c): prefix popcounts over the words.
MF_HD void table_count_item(const Shape &s, const TileMem &m, int32_t p, int32_t c)
{
    const u64 *W = m.words + ((int64_t)p * s.C + c) * s.Wn;
    u16 *pc = m.pc + ((int64_t)p * s.C + c) * (s.Wn + 1);
    int32_t acc = 0;
    for (int w = 0; w < s.Wn; w++) {
        pc[w] = (u16)acc;
        acc += popc64(W[w]);
    }
    pc[s.Wn] = (u16)acc;
}

// ---------------------------------------------------------------- 5. walk

// Window of two membership words covering positions [64*wl, 64*wl + 128).
struct Win {
    int32_t wl;
    u64 lo, hi;
};

MF_HD u64 win_word(const Shape &s, const u16 *Mp, const Win &W, int32_t wq, int32_t i)
{
    if (wq == W.wl) return W.lo;
    if (wq == W.wl + 1) return W.hi;
    return member_word(s, Mp, wq, i);
}

// Keep r at least 16 positions inside the window; otherwise move the
// window so that r sits in its middle half.
MF_HD void win_center(const Shape &s, const u16 *Mp, Win &W, int32_t r, int32_t i)
{
    const int32_t d = r - W.wl * 64;
    if (d >= 16 && d < 112) return;
    const int32_t wr = r >> 6;
    const int32_t wl = ((r & 63) >= 32) ? wr : wr - 1;
    if (wl == W.wl) return;
    const u64 nlo = win_word(s, Mp, W, wl, i);
    const u64 nhi = win_word(s, Mp, W, wl + 1, i);
    W.wl = wl;
    W.lo = nlo;
    W.hi = nhi;
}

MF_HD void win_flip(Win &W, int32_t p, bool set)
{
    const int32_t d = p - W.wl * 64;
    if (d < 0 || d >= 128) return;
    const u64 bit = 1ull << (d & 63);
    if (d < 64) W.lo = set ? (W.lo | bit) : (W.lo & ~bit);
    else        W.hi = set ? (W.hi | bit) : (W.hi & ~bit);
}

// Walk of chunk c of pair p: steps [c*L, min((c+1)*L, len B)).
// Returns 0, or -1 if a search ran off the merged order (cannot happen
// for a correct table; the bound keeps the loop finite).
MF_HD int walk_item(const Shape &s, const Tile &T, const TileMem &m, int32_t p, int32_t c)
{
    const int32_t lenB = block_len(s, T, p + 1);
    const int32_t i0 = c * s.L;
    const int32_t i1 = (i0 + s.L < lenB) ? i0 + s.L : lenB;
    const u16 *Mp = m.M + p * s.Mstride;
    const u64 *Wc = m.words + ((int64_t)p * s.C + c) * s.Wn;
    const u16 *pc = m.pc + ((int64_t)p * s.C + c) * (s.Wn + 1);
    const u32 *pos = m.pos + p * s.k;
    u16 *stage = m.stage + p * s.k;
    const int32_t h = s.h;

    // rank-h member before step i0: largest w with pc[w] <= h
    int32_t lo = 0, hi = s.Wn;
    while (hi - lo > 1) {
        const int32_t mid = (lo + hi) >> 1;
        if ((int32_t)pc[mid] <= h) lo = mid;
        else hi = mid;
    }
    int32_t r = lo * 64 + select64(Wc[lo], h - (int32_t)pc[lo]);

    Win W;
    W.wl = ((r & 63) >= 32) ? (r >> 6) : (r >> 6) - 1;
    W.lo = (W.wl >= 0) ? Wc[W.wl] : 0ull;
    W.hi = (W.wl + 1 < s.Wn) ? Wc[W.wl + 1] : 0ull;

    const int32_t maxw = s.Wn + 2;
    int32_t i = i0;
    int bad = 0;
    for (; i < i1 && !bad; i++) {
        const u32 pab = pos[i];
        const int32_t pa = (int32_t)(pab & 0xFFFFu), pb = (int32_t)(pab >> 16);
        win_flip(W, pa, false);
        win_flip(W, pb, true);
        int32_t dir;
        if (pa == r) dir = (pb < r) ? -1 : 1;
        else dir = (int32_t)(pa < r) - (int32_t)(pb < r);
        if (dir > 0) {
            int32_t q = r + 1;
            for (int32_t guard = 0;; guard++) {
                const int32_t wq = q >> 6;
                if (guard > maxw || wq >= s.Wn) { bad = 1; break; }
                const u64 word = win_word(s, Mp, W, wq, i) & (~0ull << (q & 63));
                if (word) { r = wq * 64 + ctz64(word); break; }
                q = (wq + 1) * 64;
            }
            if (!bad) win_center(s, Mp, W, r, i);
        } else if (dir < 0) {
            int32_t q = r - 1;
            for (int32_t guard = 0;; guard++) {
                if (guard > maxw || q < 0) { bad = 1; break; }
                const int32_t wq = q >> 6;
                const u64 mask = ((q & 63) == 63) ? ~0ull : ((2ull << (q & 63)) - 1ull);
                const u64 word = win_word(s, Mp, W, wq, i) & mask;
                if (word) { r = wq * 64 + hibit64(word); break; }
                q = wq * 64 - 1;
            }
            if (!bad) win_center(s, Mp, W, r, i);
        }
        stage[i] = (u16)(bad ? 0 : r);
    }
    // after a failed search the rest of the chunk gets a valid placeholder
    for (; i < i1; i++) stage[i] = 0;
    return bad ? -1 : 0;
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

// Item = u-th output of the pairs (o = o0 + u).
MF_HD void output_item(const Shape &s, const Tile &T, const TileMem &m, int64_t u,
                       u32 *y, int32_t *argmed)
{
    const int32_t p = (int32_t)(u / s.k);
    const int32_t i = (int32_t)(u - (int64_t)p * s.k);
    const int32_t r = m.stage[p * s.k + i];
    const u32 e = m.M[p * s.Mstride + r];
    const int32_t b = p + (int32_t)(e >> 15);
    const int32_t t = (int32_t)(e & 0x7FFFu);
    const int64_t o = T.o0 + u;
    y[o] = m.xv[(b << s.logS) + t];
    if (argmed) argmed[o] = (int32_t)(T.e0 + (int64_t)b * s.k + t);
}

// Output 0: the median of block 0 (Section 3: Y_0's only element).
MF_HD void output_first(const Shape &s, const Tile &T, const TileMem &m, u32 *y, int32_t *argmed)
{
    const int32_t t = (int32_t)sv_t(m.srt[s.h]);
    y[0] = m.xv[t];
    if (argmed) argmed[0] = t;
}

}  // namespace mf
