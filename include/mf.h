/*
 * mf.h - sorting-based median filter on AMD MI355X (gfx950).
 *
 * The method is J. Suomela, "Median Filtering is Equivalent to Sorting"
 * (arXiv:1406.1717): sort the input in blocks of the window length k
 * (Section 3 "Piecewise Sorting"), then walk each pair of adjacent blocks,
 * removing items of the left block and adding items of the right block
 * while the window median is tracked (Sections 4-6, postprocessing).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Output o (0-based) is the median of x[o .. o+k-1], o = 0 .. n-k (the
 *   problem statement of Section 1).  k must be odd, 1 <= k <= n.
 * - Ties are broken by input index: the element of rank h = (k-1)/2 in
 *   lexicographic (value, index) order is the median (Sections 5.2, 6.3).
 *   For floats, -0.0 equals +0.0 and every NaN is above +inf.
 * - y[o] is a bit copy of x[argmed[o]]; argmed[o] is the 0-based index of
 *   the median within its signal (int32).
 * - Data pointers (x, y, argmed, grad_*) are DEVICE pointers owned by the
 *   caller.  Offset and window arrays of the batched calls are HOST arrays.
 * - `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Calls are asynchronous on that stream; arguments are validated before
 *   anything is enqueued, and nothing is written when a call fails.
 * - Limits: n <= 2^31 - 1 (argmed is int32), k <= 32767.
 * - Thread safety: entry points may be called from several host threads
 *   and on several streams.  The library's workspace (windows above 4096,
 *   64-bit signals on 1024-thread tiles) is leased to one call at a time,
 *   and each use waits on its stream for the one before it.  Executions of
 *   one plan (including the plans the one-call batched entry points keep)
 *   are serialized on the host and, across streams, on the device.
 * - Environment: MF_WS_LIMIT=<bytes> makes workspace requests above it fail
 *   with MF_ERR_NOMEM (a test switch); MF_LEASE_HOLD_US=<us> keeps each
 *   workspace lease that long before enqueueing (a test switch for
 *   concurrent callers); MF_LOG=1 prints plan and autotune decisions on
 *   stderr; MF_TUNE_CACHE=<path> is the tile-shape cache of
 *   mf_plan_autotune (read by new plans).
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum mf_status {
    MF_OK = 0,
    MF_ERR_INVALID_VALUE = 1, /* null pointer, n < 1, k < 1, k even, k > n   */
    MF_ERR_UNSUPPORTED = 2,   /* n > 2^31-1 or k > 32767                       */
    MF_ERR_NOMEM = 3,         /* the library's workspace could not be allocated */
    MF_ERR_HIP = 4,           /* a HIP runtime call failed (see mf_last_error)  */
    MF_ERR_INTERNAL = 5       /* a kernel reported an inconsistent walk         */
} mf_status;

/* Median filter of one float32 signal (Section 1; method of Sections 3-6).
 * x: n floats.  y: n-k+1 floats.  argmed: n-k+1 int32, or NULL to skip.
 * Work: one kernel launch (k <= 4096) or a workspace-backed launch for
 * larger k; the workspace is owned by the library. */
mf_status mf_median_filter(const float *x, int64_t n, int32_t k,
                           float *y, int32_t *argmed, void *stream);

/* mf_median_filter for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and checks as mf_median_filter (bit
 * for bit), but no call allocates or frees memory: windows above 4096 use a
 * fixed device array of the library (64 MiB per device, the first 256 bytes
 * a consistency flag read by mf_check_device_error, the rest per-workgroup
 * slots of 0.4-1.5 MB, as many workgroups as fit), which each device holds
 * from the first call until the process ends.  The first call on a device
 * looks the array up, clears the flag and waits on `stream` for that.
 * Every call on one device shares the array and nothing orders them: calls
 * that overlap on one device (two streams, two host threads) race and must
 * be serialized by the caller.  Errors: as mf_median_filter, plus
 * MF_ERR_UNSUPPORTED if one workgroup's slot would exceed the array (not
 * reached for k <= 32767). */
mf_status mf_median_filter_noalloc(const float *x, int64_t n, int32_t k,
                                   float *y, int32_t *argmed, void *stream);

/* The same for int32 signals (the paper benchmarks 32-bit integers,
 * Section 7).  y: n-k+1 int32. */
mf_status mf_median_filter_i32(const int32_t *x, int64_t n, int32_t k,
                               int32_t *y, int32_t *argmed, void *stream);

/* 64-bit signals (the paper measures 32- and 64-bit versions, Section 7):
 * float64 (same order rules as float32: -0.0 equals +0.0, NaNs above +inf)
 * and int64.  y: n-k+1 elements of the input type, bit copies of
 * x[argmed[o]].  The same windows as the 32-bit calls.  Each tile's items
 * are first ranked by (value, index) into 32-bit keys (in LDS for
 * k <= 2047; above, in the library's workspace: about 8 B per input item,
 * and for k > 4095 also 48k bytes per concurrent pair); the 32-bit tile
 * kernels then run on those keys and copy each median from x. */
mf_status mf_median_filter_f64(const double *x, int64_t n, int32_t k,
                               double *y, int32_t *argmed, void *stream);
mf_status mf_median_filter_i64(const int64_t *x, int64_t n, int32_t k,
                               int64_t *y, int32_t *argmed, void *stream);

/* Uniform batch: `rows` float32 signals of length n stored back to back
 * (row r at x + r*n), one window k.  Outputs row-major: y + r*(n-k+1). */
mf_status mf_median_filter_rows(const float *x, int64_t rows, int64_t n, int32_t k,
                                float *y, int32_t *argmed, void *stream);

/* The same for int32 rows. */
mf_status mf_median_filter_rows_i32(const int32_t *x, int64_t rows, int64_t n, int32_t k,
                                    int32_t *y, int32_t *argmed, void *stream);

/* 64-bit rows (float64, int64): the same layouts as mf_median_filter_rows. */
mf_status mf_median_filter_rows_f64(const double *x, int64_t rows, int64_t n, int32_t k,
                                    double *y, int32_t *argmed, void *stream);
mf_status mf_median_filter_rows_i64(const int64_t *x, int64_t rows, int64_t n, int32_t k,
                                    int64_t *y, int32_t *argmed, void *stream);

/* Ragged batch of float32 signals in one launch.  Signal s is
 * x[x_offsets[s] .. x_offsets[s+1]) with odd window ks[s] <= its length.
 * Outputs are packed in signal order: signal s writes
 * y[y_off(s) .. y_off(s) + len_s - ks[s] + 1) with
 * y_off(s) = x_offsets[s] - sum_{t<s} (ks[t] - 1); argmed is local to each
 * signal.  x_offsets (num_signals+1 entries, x_offsets[0] = 0, non-
 * decreasing) and ks are HOST arrays.  The library plans the launch (work
 * list, tile shapes) and caches the plan keyed by these arrays; see the
 * mf_plan_* calls for explicit control. */
mf_status mf_median_filter_batched(const float *x, const int64_t *x_offsets,
                                   const int32_t *ks, int32_t num_signals,
                                   float *y, int32_t *argmed, void *stream);
/* The same for int32 signals. */
mf_status mf_median_filter_batched_i32(const int32_t *x, const int64_t *x_offsets,
                                       const int32_t *ks, int32_t num_signals,
                                       int32_t *y, int32_t *argmed, void *stream);
/* Ragged batches of 64-bit signals (Section 7 measures 32- and 64-bit
 * versions): float64 and int64, same layout, offsets and windows as
 * mf_median_filter_batched, y of the input type (bit copies).  Signals with
 * windows up to 2047 run as one launch over the cached plan's work list
 * (each tile ranks its 64-bit items in LDS); larger windows run signal by
 * signal through the single-signal path, using the library's workspace. */
mf_status mf_median_filter_batched_f64(const double *x, const int64_t *x_offsets,
                                       const int32_t *ks, int32_t num_signals,
                                       double *y, int32_t *argmed, void *stream);
mf_status mf_median_filter_batched_i64(const int64_t *x, const int64_t *x_offsets,
                                       const int32_t *ks, int32_t num_signals,
                                       int64_t *y, int32_t *argmed, void *stream);

/* Backward of y = x[argmed]: grad_x[j] = sum of grad_y[o] over the outputs
 * o with argmed[o] == j, accumulated in float64 in increasing o and rounded
 * once to float32; 0 where no output selects j.  Deterministic (no
 * order-dependent atomics).  grad_y, argmed: n-k+1 entries; grad_x: n
 * entries, fully overwritten. */
mf_status mf_median_filter_backward(const float *grad_y, const int32_t *argmed,
                                    int64_t n, int32_t k, float *grad_x, void *stream);

/* Backward of mf_median_filter_f64 (and of the int64 forward's argmed):
 * float64 gradients, grad_x[j] = sum of grad_y[o] over the outputs o with
 * argmed[o] == j, accumulated in float64 in increasing o (no rounding);
 * 0 where no output selects j.  Deterministic; grad_x fully overwritten. */
mf_status mf_median_filter_backward_f64(const double *grad_y, const int32_t *argmed,
                                        int64_t n, int32_t k, double *grad_x, void *stream);

/* Backward of the 64-bit rows (float64 gradients, same layouts). */
mf_status mf_median_filter_backward_rows_f64(const double *grad_y, const int32_t *argmed,
                                             int64_t rows, int64_t n, int32_t k,
                                             double *grad_x, void *stream);

/* Backward of mf_median_filter_rows (same layouts). */
mf_status mf_median_filter_backward_rows(const float *grad_y, const int32_t *argmed,
                                         int64_t rows, int64_t n, int32_t k,
                                         float *grad_x, void *stream);

/* Backward of mf_median_filter_batched (same packed layouts). */
mf_status mf_median_filter_backward_batched(const float *grad_y, const int32_t *argmed,
                                            const int64_t *x_offsets, const int32_t *ks,
                                            int32_t num_signals, float *grad_x, void *stream);

/* Explicit plans for the ragged batch (x_offsets, ks: host arrays as for
 * mf_median_filter_batched, read only during the call).
 *
 * mf_plan_create_batched validates every signal (any invalid signal
 * rejects the whole batch with its status), assigns each signal a tile
 * family by its window, and uploads device work lists of (signal, tile)
 * units ordered by window, largest first.  mf_plan_execute enqueues the
 * whole forward batch on `stream` as one graph launch; the graph is
 * captured on first use and again whenever x, y, argmed or the launch
 * configuration change.  Executions of one plan are serialized: a call
 * holds the plan's lock while it captures and enqueues, and waits on its
 * stream for the plan's previous execution (its persistent launches share
 * one work counter per launch).  The plan owns its device memory until
 * mf_plan_destroy, which waits for the plan's last execution; destroying a
 * plan while another thread still calls it is not allowed. */
typedef struct mf_plan mf_plan;
mf_status mf_plan_create_batched(const int64_t *x_offsets, const int32_t *ks,
                                 int32_t num_signals, mf_plan **out);
mf_status mf_plan_execute(mf_plan *plan, const float *x, float *y, int32_t *argmed,
                          void *stream);
/* mf_plan_execute for int32 signals (the plan does not depend on the type). */
mf_status mf_plan_execute_i32(mf_plan *plan, const int32_t *x, int32_t *y, int32_t *argmed,
                              void *stream);
/* mf_plan_execute for float64 and int64 signals (as
 * mf_median_filter_batched_f64/_i64; not graph-captured, and the launch
 * configuration does not apply). */
mf_status mf_plan_execute_f64(mf_plan *plan, const double *x, double *y, int32_t *argmed,
                              void *stream);
mf_status mf_plan_execute_i64(mf_plan *plan, const int64_t *x, int64_t *y, int32_t *argmed,
                              void *stream);
mf_status mf_plan_execute_backward(mf_plan *plan, const float *grad_y, const int32_t *argmed,
                                   float *grad_x, void *stream);
int64_t   mf_plan_output_length(const mf_plan *plan);
void      mf_plan_destroy(mf_plan *plan);

/* Launch configurations of a plan's forward.  Windows above 4096 (global
 * workspace tiles) and k = 1 always have launches of their own. */
typedef enum {
    MF_LAUNCH_PER_FAMILY = 0,     /* one launch per tile family, one workgroup per tile */
    MF_LAUNCH_PERSISTENT = 1,     /* one persistent launch per tile family (default) */
    MF_LAUNCH_PERSISTENT_ONE = 2  /* one persistent launch for every LDS tile (k <= 4096),
                                     all as 1024-thread tiles */
} mf_launch_config;

/* Tunes the plan on these buffers, with the float kernels (the choices hold
 * for int32 executes too), in two steps:
 * 1. Tile shapes: the windows of each slot-stride bucket (2^b >= k, up to
 *    2048) that fit 512-thread tiles are timed as 512- and as 1024-thread
 *    tiles (`reps` launches each, 1..100, after a warm-up) and run with the
 *    faster from then on.  With MF_TUNE_CACHE=<path> set, the choices are
 *    merged into that JSON file, {"tile_threads": {"f32": {"<stride>":
 *    512 or 1024, ...}}}, which later plans read when they are created.
 * 2. Launch configurations: every configuration is timed (`reps` executes
 *    after one warm-up) and the fastest kept for later executes.
 * Writes y and argmed (the batch's outputs, as mf_plan_execute) and
 * synchronizes `stream`; MF_ERR_UNSUPPORTED while `stream` is being
 * captured.  On failure the configuration is left as it was. */
mf_status mf_plan_autotune(mf_plan *plan, const float *x, float *y, int32_t *argmed,
                           int32_t reps, void *stream);
/* Forces a configuration (an mf_launch_config value). */
mf_status mf_plan_set_config(mf_plan *plan, int32_t config);
/* The configuration in use, and (if tuned_ms is not null) the mean time
 * per execute of each configuration from the last mf_plan_autotune, in
 * milliseconds, -1 where not timed: tuned_ms has 3 entries. */
mf_status mf_plan_get_config(const mf_plan *plan, int32_t *config, float *tuned_ms);
/* Threads per tile (512 or 1024) that the plan's per-family and persistent
 * configurations use for window k; 0 for windows above 4096 and k = 1 (not
 * LDS tiles).  MF_ERR_INVALID_VALUE for an even or unsupported k. */
mf_status mf_plan_get_tile_threads(const mf_plan *plan, int32_t k, int32_t *threads);

/* n-k+1 for a valid (n, k), else -1.  Host only. */
int64_t mf_output_length(int64_t n, int32_t k);

/* Static description of a status code. */
const char *mf_status_string(mf_status s);

/* Detail of the last failure on the calling host thread ("" if none). */
const char *mf_last_error(void);

/* Kernel-side consistency flag: returns MF_ERR_INTERNAL if any kernel since
 * the last call reported an inconsistent walk, MF_OK otherwise, and clears
 * the flag.  Synchronizes `stream`. */
mf_status mf_check_device_error(void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MF_H */
