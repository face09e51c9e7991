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
 *                            for one window, sort its (value, index) pairs
 *                            and take the element of rank h = (k-1)/2.  A
 *                            library sort (qsort) is the only step used.
 *
 *   oracle_sortmedian_*      The paper's method: piecewise stable sort
 *                            (Section 3 "Piecewise Sorting", Section 5.2),
 *                            the block data structure (Section 5.3, figure
 *                            "Block data structure implementation") built on
 *                            dancing links (Section 4, eqs. del / undo-del),
 *                            and the postprocessing driver (Section 6.2,
 *                            figure "Algorithm for median filtering:
 *                            postprocessing phase"), with the invariant of
 *                            eq. (inv) checked at run time.
 *
 * Readings taken where the paper is silent:
 *   - Arbitrary n (Section 3 says the extension is straightforward): blocks
 *     of length k, the last one partial with r = n - (b-1)k items; the last
 *     pair walks r steps.  Output o (0-based) is the median of x[o..o+k-1].
 *   - Ties: all comparisons are on (value, global index) pairs (Sections 5.2
 *     and 6.3: equal elements keep input order; A's items count as smaller).
 *   - The +infinity sentinel of Section 5.3 is a pair strictly above every
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

/* qsort has no context argument; the comparator reads these statics.  The
 * oracle is single-threaded by design. */
static const values_t *g_sort_vals;
static int64_t g_sort_base;

static int qsort_pair_cmp(const void *pa, const void *pb)
{
    const int64_t a = g_sort_base + *(const int32_t *)pa;
    const int64_t b = g_sort_base + *(const int32_t *)pb;
    const int c = cmp_value(g_sort_vals, a, b);
    if (c != 0) return c;
    return (a > b) - (a < b);
}

/* Stable argsort of x[base .. base+len) by (value, index): Section 5.2 sorts
 * the pairs (alpha[i], i) with any sort and keeps the second components. */
static void sort_block(const values_t *v, int64_t base, int32_t len, int32_t *pi)
{
    for (int32_t i = 0; i < len; i++) pi[i] = i;
    g_sort_vals = v;
    g_sort_base = base;
    qsort(pi, (size_t)len, sizeof(int32_t), qsort_pair_cmp);
}

/* ---------------------------------------------------------------------- */
/* Definition oracle: one window at a time.                                */

static int window_median(const values_t *v, int64_t n, int32_t k, int64_t o,
                         int32_t *scratch, int64_t *out_index)
{
    if (o < 0 || o + k > n) return OR_EINVAL;
    sort_block(v, o, k, scratch);
    *out_index = o + scratch[(k - 1) / 2];
    return OR_OK;
}

static int window_oracle(const values_t *v, int64_t n, int32_t k,
                         const int64_t *outs, int64_t count, int32_t *argmed)
{
    if (k < 1 || (k & 1) == 0 || n < k) return OR_EINVAL;
    int32_t *scratch = (int32_t *)malloc(sizeof(int32_t) * (size_t)k);
    if (!scratch) return OR_ENOMEM;
    int rc = OR_OK;
    for (int64_t q = 0; q < count && rc == OR_OK; q++) {
        int64_t idx = 0;
        rc = window_median(v, n, k, outs[q], scratch, &idx);
        argmed[q] = (int32_t)idx;
    }
    free(scratch);
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
/* The paper's block data structure (Section 5).                           */

typedef struct {
    const values_t *v;
    int64_t base;        /* global index of alpha[0] */
    int32_t len;         /* number of items in the block (k, or r if last) */
    int32_t *pi;         /* stable sorting permutation */
    int32_t *prev;       /* len + 1 entries; slot len is the list head/tail */
    int32_t *next;
    int32_t m;           /* first large item, or len (= tail) */
    int32_t s;           /* number of small items */
} block_t;

static int32_t tail_of(const block_t *B) { return B->len; }
static int at_end(const block_t *B) { return B->m == tail_of(B); }

/* Is alpha[i] small?  True if every item is small (cursor at the end), or
 * (alpha[i], i) < (alpha[m], m). */
static int is_small(const block_t *B, int32_t i)
{
    if (at_end(B)) return 1;
    return pair_less(B->v, B->base + i, B->base + B->m);
}

/* construct(alpha, pi): link the items in sorted order, h of them small. */
static void block_construct(block_t *B, int32_t h)
{
    int32_t p = tail_of(B);
    for (int32_t r = 0; r < B->len; r++) {
        const int32_t q = B->pi[r];
        B->next[p] = q;
        B->prev[q] = p;
        p = q;
    }
    B->next[p] = tail_of(B);
    B->prev[tail_of(B)] = p;
    B->s = h;
    /* A partial block (len <= h) is only ever the right block of the last
     * pair, which is unwound at once; its cursor is set there. */
    B->m = (h < B->len) ? B->pi[h] : tail_of(B);
}

/* delete(B, i): unlink item i (eq. del) and keep (m, s) consistent. */
static void block_delete(block_t *B, int32_t i)
{
    const int small = is_small(B, i);
    B->next[B->prev[i]] = B->next[i];
    B->prev[B->next[i]] = B->prev[i];
    if (small) {
        B->s -= 1;
    } else {
        if (B->m == i) B->m = B->next[B->m];
        if (B->s > 0) {
            B->m = B->prev[B->m];
            B->s -= 1;
        }
    }
}

/* undelete(B, i): relink item i (eq. undo-del). */
static void block_undelete(block_t *B, int32_t i)
{
    B->next[B->prev[i]] = i;
    B->prev[B->next[i]] = i;
    if (is_small(B, i)) B->m = B->prev[B->m];
}

/* unwind(B): delete items len-1 .. 0; afterwards the list is empty. */
static void block_unwind(block_t *B)
{
    for (int32_t i = B->len - 1; i >= 0; i--) {
        B->next[B->prev[i]] = B->next[i];
        B->prev[B->next[i]] = B->prev[i];
    }
    B->m = tail_of(B);
    B->s = 0;
}

static void block_advance(block_t *B)
{
    B->m = B->next[B->m];
    B->s += 1;
}

/* Peek(A) <= Peek(B) on (value, global index) pairs, where a cursor at the
 * end stands for a pair above every real pair.  A's items precede B's in
 * the input, so on equal values A's item is the smaller one. */
static int peek_le(const block_t *A, const block_t *B)
{
    if (at_end(A)) return 0;            /* +inf <= real pair is false; both at
                                            the end cannot happen */
    if (at_end(B)) return 1;
    return pair_less(A->v, A->base + A->m, B->base + B->m);
}

static int64_t peek_index(const block_t *B) { return B->base + B->m; }

static int block_alloc(block_t *B, int32_t cap)
{
    B->pi = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
    B->prev = (int32_t *)malloc(sizeof(int32_t) * ((size_t)cap + 1));
    B->next = (int32_t *)malloc(sizeof(int32_t) * ((size_t)cap + 1));
    return (B->pi && B->prev && B->next) ? OR_OK : OR_ENOMEM;
}

static void block_free(block_t *B)
{
    free(B->pi);
    free(B->prev);
    free(B->next);
}

static void block_load(block_t *B, const values_t *v, int64_t base, int32_t len)
{
    B->v = v;
    B->base = base;
    B->len = len;
    sort_block(v, base, len, B->pi);
}

/* ---------------------------------------------------------------------- */
/* Postprocessing driver (Section 6.2).                                    */

static int sortmedian(const values_t *v, int64_t n, int32_t k, int32_t *argmed)
{
    if (k < 1 || (k & 1) == 0 || n < k || n > INT32_MAX) return OR_EINVAL;
    const int32_t h = (k - 1) / 2;
    const int64_t nb = (n + k - 1) / k;     /* number of blocks */

    block_t blk[2];
    memset(blk, 0, sizeof(blk));
    int rc = block_alloc(&blk[0], k);
    if (rc == OR_OK) rc = block_alloc(&blk[1], k);
    if (rc != OR_OK) {
        block_free(&blk[0]);
        block_free(&blk[1]);
        return rc;
    }

    block_t *B = &blk[0];
    block_load(B, v, 0, k);                  /* block 0 is always full */
    block_construct(B, h);
    argmed[0] = (int32_t)peek_index(B);      /* step (double dagger) */

    for (int64_t j = 1; j < nb && rc == OR_OK; j++) {
        block_t *A = B;
        B = (A == &blk[0]) ? &blk[1] : &blk[0];
        const int64_t base = j * (int64_t)k;
        const int32_t len = (int32_t)((n - base) < k ? (n - base) : k);
        block_load(B, v, base, len);
        block_construct(B, h);
        block_unwind(B);
        for (int32_t i = 0; i < len; i++) {
            block_delete(A, i);              /* step (dagger) */
            block_undelete(B, i);
            if (A->s + B->s < h) {
                if (peek_le(A, B)) block_advance(A);
                else block_advance(B);
            }
            /* eq. (inv): exactly h small items, counters in range, and at
             * least one block has a large item to report. */
            if (A->s + B->s != h || A->s < 0 || B->s < 0 ||
                (at_end(A) && at_end(B))) {
                rc = OR_EINVARIANT;
                break;
            }
            const int64_t o = (j - 1) * (int64_t)k + i + 1;
            argmed[o] = (int32_t)(peek_le(A, B) ? peek_index(A) : peek_index(B));
        }
    }
    block_free(&blk[0]);
    block_free(&blk[1]);
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
