/*
 * CPU oracle for the sorting-based median filter (Suomela, "Median Filtering
 * is Equivalent to Sorting", arXiv:1406.1717).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code, header, table or
 * helper with the HIP implementation.
 *
 * Two independent forward oracles live here:
 *
 *   oracle_window_median_*   The problem statement of Section 1 written out:
 *                            for one window, order its (value, index) pairs
 *                            and take the element of rank h = (k-1)/2.
 *
 *   oracle_sortmedian_*      The paper's method: piecewise stable sort
 *                            (Section 3 "Piecewise Sorting", Section 5.2),
 *                            block data structures (Section 5: the interface
 *                            of figure "Block data structure interface", the
 *                            invariants of Section 5.3) on dancing links
 *                            (Section 4, eqs. del / undo-del), and the
 *                            postprocessing of Section 6.2, with eq. (inv)
 *                            checked after every step.
 *
 * How the block structure is written here.  A block keeps its list L as
 * prev/next links with a tail index (the block length), a counter s of
 * small items, and a cursor m.  Section 5.3 fixes the invariant m = p_s:
 * the cursor stands on the list element with exactly s elements before it
 * (the tail when s = |L|).  Each interface operation below changes L and s
 * as the interface says (delete: s <- max(0, s-1); undelete: s unchanged;
 * advance: s <- s+1), keeps count of how many list elements precede the
 * cursor, and then moves the cursor along the links until that count is s
 * again.  The cursor moves this produces are the ones Section 5.3 states;
 * the run-time check of eq. (inv) and the pins in tests/ confirm it.
 *
 * Readings taken where the paper is silent:
 *   - Arbitrary n (Section 3 says the extension is straightforward): blocks
 *     of length k, the last one partial with r = n - (b-1)k items; the last
 *     pair walks r steps.  Output o (0-based) is the median of x[o..o+k-1].
 *   - Ties: all comparisons are on (value, global index) pairs (Sections 5.2
 *     and 6.3: equal elements keep input order; A's items count as smaller).
 *   - The +infinity of Section 5.3 (alpha[k]) is a pair strictly above every
 *     real pair, so real +inf data cannot collide with it.
 *   - Float order: -0.0 equals +0.0 (IEEE equality, tie broken by index);
 *     every NaN is above +inf and all NaNs are equal (tie broken by index).
 *   - 32-bit and 64-bit elements (Section 7 benchmarks both widths) follow
 *     the same rules; signed integers compare as signed.
 *   - k must be odd with 1 <= k <= n.
 *
 * Backward (not in the paper): grad_x[j] = sum of grad_y[o] over all o with
 * argmed[o] == j, accumulated in float64 in increasing o, rounded once
 * (float32 gradients) or not at all (float64 gradients).
 *
 * Every function is reentrant (no static state), so callers may run
 * several signals or output ranges in parallel threads.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

enum { OR_OK = 0, OR_EINVAL = -1, OR_ENOMEM = -2, OR_EINVARIANT = -3 };

/* ---------------------------------------------------------------------- */
/* Value order.  cmp returns <0, 0, >0.                                    */

/* Element types: the paper benchmarks 32-bit and 64-bit versions
 * (Section 7); the order rules are the same for both widths. */
enum { T_I32 = 0, T_F32 = 1, T_I64 = 2, T_F64 = 3 };

typedef struct {
    const void *x;       /* the whole signal */
    int type;            /* T_I32, T_F32, T_I64 or T_F64 */
} values_t;

static int cmp_value(const values_t *v, int64_t a, int64_t b)
{
    switch (v->type) {
    case T_F32: {
        const float fa = ((const float *)v->x)[a];
        const float fb = ((const float *)v->x)[b];
        const int na = isnan(fa) != 0, nb = isnan(fb) != 0;
        if (na || nb) return na - nb;            /* NaN above all; NaNs tie */
        return (fa > fb) - (fa < fb);            /* -0.0 == +0.0 */
    }
    case T_F64: {
        const double fa = ((const double *)v->x)[a];
        const double fb = ((const double *)v->x)[b];
        const int na = isnan(fa) != 0, nb = isnan(fb) != 0;
        if (na || nb) return na - nb;
        return (fa > fb) - (fa < fb);
    }
    case T_I64: {
        const int64_t ia = ((const int64_t *)v->x)[a];
        const int64_t ib = ((const int64_t *)v->x)[b];
        return (ia > ib) - (ia < ib);
    }
    default: {
        const int32_t ia = ((const int32_t *)v->x)[a];
        const int32_t ib = ((const int32_t *)v->x)[b];
        return (ia > ib) - (ia < ib);
    }
    }
}

/* Lexicographic (value, index) order on global indices. */
static int pair_less(const values_t *v, int64_t a, int64_t b)
{
    const int c = cmp_value(v, a, b);
    if (c != 0) return c < 0;
    return a < b;
}

/* Section 5.2: the sorting permutation of x[base .. base+len) taken from
 * the pairs (value, index) in lexicographic order.  A bottom-up merge sort
 * on the local indices (tmp: len entries of scratch). */
static void sort_pairs(const values_t *v, int64_t base, int32_t len, int32_t *pi, int32_t *tmp)
{
    for (int32_t i = 0; i < len; i++) pi[i] = i;
    int32_t *src = pi, *dst = tmp;
    for (int32_t w = 1; w < len; w *= 2) {
        for (int32_t lo = 0; lo < len; lo += 2 * w) {
            const int32_t mid = lo + w < len ? lo + w : len;
            const int32_t hi = lo + 2 * w < len ? lo + 2 * w : len;
            int32_t a = lo, b = mid, o = lo;
            while (a < mid && b < hi)
                dst[o++] = pair_less(v, base + src[b], base + src[a]) ? src[b++] : src[a++];
            while (a < mid) dst[o++] = src[a++];
            while (b < hi) dst[o++] = src[b++];
        }
        int32_t *t = src;
        src = dst;
        dst = t;
    }
    if (src != pi) memcpy(pi, src, sizeof(int32_t) * (size_t)len);
}

/* ---------------------------------------------------------------------- */
/* Definition oracle: one window at a time.                                */

static int window_oracle(const values_t *v, int64_t n, int32_t k,
                         const int64_t *outs, int64_t count, int32_t *argmed)
{
    if (k < 1 || (k & 1) == 0 || n < k) return OR_EINVAL;
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    if (!order || !tmp) {
        free(order);
        free(tmp);
        return OR_ENOMEM;
    }
    int rc = OR_OK;
    for (int64_t q = 0; q < count; q++) {
        const int64_t o = outs[q];
        if (o < 0 || o + k > n) {
            rc = OR_EINVAL;
            break;
        }
        /* the window's pairs in order; the median has h = (k-1)/2 below it */
        sort_pairs(v, o, k, order, tmp);
        argmed[q] = (int32_t)(o + order[(k - 1) / 2]);
    }
    free(order);
    free(tmp);
    return rc;
}

/* Median (as a global index) of each window listed in outs[0..count). */
int oracle_window_median_f32(const float *x, int64_t n, int32_t k,
                             const int64_t *outs, int64_t count, int32_t *argmed)
{
    values_t v = {x, T_F32};
    return window_oracle(&v, n, k, outs, count, argmed);
}

int oracle_window_median_i32(const int32_t *x, int64_t n, int32_t k,
                             const int64_t *outs, int64_t count, int32_t *argmed)
{
    values_t v = {x, T_I32};
    return window_oracle(&v, n, k, outs, count, argmed);
}

int oracle_window_median_f64(const double *x, int64_t n, int32_t k,
                             const int64_t *outs, int64_t count, int32_t *argmed)
{
    values_t v = {x, T_F64};
    return window_oracle(&v, n, k, outs, count, argmed);
}

int oracle_window_median_i64(const int64_t *x, int64_t n, int32_t k,
                             const int64_t *outs, int64_t count, int32_t *argmed)
{
    values_t v = {x, T_I64};
    return window_oracle(&v, n, k, outs, count, argmed);
}

/* ---------------------------------------------------------------------- */
/* Block data structure (Section 5).                                       */

typedef struct {
    const values_t *v;
    int64_t base;        /* global index of alpha[0] */
    int32_t len;         /* items of the block (k, or r for a partial last
                            block); index len is the tail of the list and
                            stands for alpha[len] = +infinity */
    int32_t *pi;         /* sorting permutation (Section 5.2) */
    int32_t *tmp;        /* sort scratch */
    int32_t *prev;       /* len + 1 links */
    int32_t *next;
    int32_t m;           /* cursor: the first large item, or the tail */
    int32_t s;           /* small items: the first s of L */
    int32_t ahead;       /* list elements before the cursor (= s when settled) */
} block_t;

/* Is item i ordered before the cursor?  The tail is +infinity, so with
 * the cursor on the tail every item is. */
static int before_cursor(const block_t *B, int32_t i)
{
    if (B->m == B->len) return 1;
    return pair_less(B->v, B->base + i, B->base + B->m);
}

/* Eq. (del): take item i out of the list. */
static void unlink_item(block_t *B, int32_t i)
{
    B->prev[B->next[i]] = B->prev[i];
    B->next[B->prev[i]] = B->next[i];
}

/* Eq. (undo-del): put item i back where it was. */
static void relink_item(block_t *B, int32_t i)
{
    B->prev[B->next[i]] = i;
    B->next[B->prev[i]] = i;
}

/* Section 5.3's invariant m = p_s: move the cursor along the list until
 * exactly s list elements stand before it. */
static void settle(block_t *B)
{
    while (B->ahead > B->s) {
        B->m = B->prev[B->m];
        B->ahead -= 1;
    }
    while (B->ahead < B->s) {
        B->m = B->next[B->m];
        B->ahead += 1;
    }
}

/* construct(alpha, pi): L holds the block in sorted order (the links follow
 * pi from the tail around to the tail), and the first h items are small. */
static void construct(block_t *B, int32_t h)
{
    int32_t last = B->len;
    for (int32_t r = 0; r < B->len; r++) {
        B->next[last] = B->pi[r];
        B->prev[B->pi[r]] = last;
        last = B->pi[r];
    }
    B->next[last] = B->len;
    B->prev[B->len] = last;
    B->m = B->next[B->len];      /* cursor on the first element, nothing ahead */
    B->ahead = 0;
    B->s = h < B->len ? h : B->len;
    settle(B);
}

/* delete(B, i): remove alpha[i] from L; s <- max(0, s-1). */
static void delete_item(block_t *B, int32_t i)
{
    if (i == B->m) B->m = B->next[i];            /* same number of elements ahead */
    else if (before_cursor(B, i)) B->ahead -= 1;
    unlink_item(B, i);
    if (B->s > 0) B->s -= 1;
    settle(B);
}

/* undelete(B, i): put alpha[i] back into L; s unchanged. */
static void undelete_item(block_t *B, int32_t i)
{
    relink_item(B, i);
    if (before_cursor(B, i)) B->ahead += 1;
    settle(B);
}

/* unwind(B): delete(B, len-1), ..., delete(B, 0); L ends empty. */
static void unwind(block_t *B)
{
    for (int32_t i = B->len - 1; i >= 0; i--) delete_item(B, i);
}

/* advance(B): s <- s + 1. */
static void advance(block_t *B)
{
    B->s += 1;
    settle(B);
}

/* peek(B): the first large element as a global index, or -1 for +infinity. */
static int64_t peek(const block_t *B)
{
    return B->m == B->len ? -1 : B->base + B->m;
}

/* Order of two peeks, +infinity (-1) above every real pair: is a <= b?
 * Two real peeks are never equal (distinct global indices); both infinite
 * cannot occur while eq. (inv) holds. */
static int peek_le(const values_t *v, int64_t a, int64_t b)
{
    if (a < 0) return b < 0;
    if (b < 0) return 1;
    return pair_less(v, a, b);
}

static int block_alloc(block_t *B, int32_t cap)
{
    B->pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    B->tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    B->prev = (int32_t *)malloc(sizeof(int32_t) * ((size_t)cap + 1));
    B->next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)cap + 1));
    return (B->pi && B->tmp && B->prev && B->next) ? OR_OK : OR_ENOMEM;
}

static void block_free(block_t *B)
{
    free(B->pi);
    free(B->tmp);
    free(B->prev);
    free(B->next);
}

/* Block X_j with its sorting permutation P_j (Section 6.1). */
static void load_block(block_t *B, const values_t *v, int64_t base, int32_t len)
{
    B->v = v;
    B->base = base;
    B->len = len;
    sort_pairs(v, base, len, B->pi, B->tmp);
}

/* ---------------------------------------------------------------------- */
/* Postprocessing (Section 6.2).                                           */

static int sortmedian(const values_t *v, int64_t n, int32_t k, int32_t *argmed)
{
    if (k < 1 || (k & 1) == 0 || n < k || n > INT32_MAX) return OR_EINVAL;
    const int32_t h = (k - 1) / 2;
    const int64_t b = (n + k - 1) / k;       /* blocks X_0 .. X_{b-1} */

    block_t blocks[2];
    memset(blocks, 0, sizeof(blocks));
    int rc = block_alloc(&blocks[0], k);
    if (rc == OR_OK) rc = block_alloc(&blocks[1], k);
    if (rc != OR_OK) {
        block_free(&blocks[0]);
        block_free(&blocks[1]);
        return rc;
    }

    /* Y_0: the median of X_0 is its first large item */
    block_t *B = &blocks[0];
    load_block(B, v, 0, k);
    construct(B, h);
    argmed[0] = (int32_t)peek(B);

    for (int64_t j = 1; j < b && rc == OR_OK; j++) {
        /* the pair (A, B) = (X_{j-1}, X_j); B starts empty (unwound) */
        block_t *A = B;
        B = (A == &blocks[0]) ? &blocks[1] : &blocks[0];
        const int64_t base = j * (int64_t)k;
        const int32_t len = (int32_t)((n - base) < k ? (n - base) : k);
        load_block(B, v, base, len);
        construct(B, h);
        unwind(B);
        for (int32_t i = 0; i < len; i++) {
            /* slide the window: alpha_A[i] leaves, alpha_B[i] enters */
            delete_item(A, i);
            undelete_item(B, i);
            /* restore h small items: the smaller peek becomes small (A wins
             * ties: its items precede B's in the input) */
            if (A->s + B->s < h) {
                if (peek_le(v, peek(A), peek(B))) advance(A);
                else advance(B);
            }
            /* eq. (inv): exactly h small items, counters in range, and a
             * large item left to report */
            if (A->s + B->s != h || A->s < 0 || B->s < 0 || (peek(A) < 0 && peek(B) < 0)) {
                rc = OR_EINVARIANT;
                break;
            }
            /* the window's median: the smaller of the two peeks */
            const int64_t pa = peek(A), pb = peek(B);
            const int64_t o = (j - 1) * (int64_t)k + i + 1;
            argmed[o] = (int32_t)(peek_le(v, pa, pb) ? pa : pb);
        }
    }
    block_free(&blocks[0]);
    block_free(&blocks[1]);
    return rc;
}

int oracle_sortmedian_f32(const float *x, int64_t n, int32_t k, float *y, int32_t *argmed)
{
    values_t v = {x, T_F32};
    const int rc = sortmedian(&v, n, k, argmed);
    if (rc != OR_OK) return rc;
    if (y)
        for (int64_t o = 0; o + k <= n; o++) memcpy(&y[o], &x[argmed[o]], sizeof(float));
    return OR_OK;
}

int oracle_sortmedian_i32(const int32_t *x, int64_t n, int32_t k, int32_t *y, int32_t *argmed)
{
    values_t v = {x, T_I32};
    const int rc = sortmedian(&v, n, k, argmed);
    if (rc != OR_OK) return rc;
    if (y)
        for (int64_t o = 0; o + k <= n; o++) y[o] = x[argmed[o]];
    return OR_OK;
}

int oracle_sortmedian_f64(const double *x, int64_t n, int32_t k, double *y, int32_t *argmed)
{
    values_t v = {x, T_F64};
    const int rc = sortmedian(&v, n, k, argmed);
    if (rc != OR_OK) return rc;
    if (y)
        for (int64_t o = 0; o + k <= n; o++) memcpy(&y[o], &x[argmed[o]], sizeof(double));
    return OR_OK;
}

int oracle_sortmedian_i64(const int64_t *x, int64_t n, int32_t k, int64_t *y, int32_t *argmed)
{
    values_t v = {x, T_I64};
    const int rc = sortmedian(&v, n, k, argmed);
    if (rc != OR_OK) return rc;
    if (y)
        for (int64_t o = 0; o + k <= n; o++) y[o] = x[argmed[o]];
    return OR_OK;
}

/* ---------------------------------------------------------------------- */
/* Backward: the scatter of the upstream gradient to the selected inputs.   */

int oracle_backward(const float *grad_y, const int32_t *argmed, int64_t n, int32_t k,
                    double *grad_x64, float *grad_x)
{
    if (k < 1 || (k & 1) == 0 || n < k) return OR_EINVAL;
    for (int64_t j = 0; j < n; j++) grad_x64[j] = 0.0;
    for (int64_t o = 0; o + k <= n; o++) {
        const int32_t j = argmed[o];
        if (j < o || j > o + k - 1) return OR_EINVAL;
        grad_x64[j] += (double)grad_y[o];
    }
    if (grad_x)
        for (int64_t j = 0; j < n; j++) grad_x[j] = (float)grad_x64[j];
    return OR_OK;
}

/* The same scatter for a float64 upstream gradient (float64 signals): the
 * float64 sums in increasing o are the result, with no final rounding. */
int oracle_backward_f64(const double *grad_y, const int32_t *argmed, int64_t n, int32_t k,
                        double *grad_x)
{
    if (k < 1 || (k & 1) == 0 || n < k) return OR_EINVAL;
    for (int64_t j = 0; j < n; j++) grad_x[j] = 0.0;
    for (int64_t o = 0; o + k <= n; o++) {
        const int32_t j = argmed[o];
        if (j < o || j > o + k - 1) return OR_EINVAL;
        grad_x[j] += grad_y[o];
    }
    return OR_OK;
}
