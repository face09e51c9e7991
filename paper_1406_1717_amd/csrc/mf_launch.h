// Launch interface between the host runtime (mf_api.cpp) and the kernels
// (mf_kernels.hip).  Internal to the library.
#pragma once
#include <stdint.h>
#include <hip/hip_runtime.h>

namespace mf {

// One signal of a launch, as offsets into the launch's base pointers:
// x + x_off (n items), y / argmed + y_off (n-k+1 outputs).
struct SigDesc {
    int64_t x_off;
    int64_t y_off;
    int64_t n;
    int32_t k;
    int32_t pad;
};

// One work unit of a multi-signal launch: tile `tile` of signal `sig`.
struct Unit {
    int32_t sig;
    int32_t pad;
    int64_t tile;
};

// Base pointers and the signal set of a launch.  Units come from `units`
// (a device table), or, when units is null, from `one`: tiles
// 0 .. tpr-1 of `rows` signals of equal shape laid out back to back.
struct Launch {
    const void *x;       // 32-bit patterns (float or int32)
    void *y;
    int32_t *argmed;     // may be null in the forward
    SigDesc one;
    int64_t rows;
    int64_t tpr;         // tiles per row
    const SigDesc *sigs;
    const Unit *units;
    int64_t nunits;
    // 64-bit signals (int32 LDS kernels only): rank_mode 1, x holds the rank
    // keys of the 64-bit signal x64, tile t's at x + t * xshift; 2 (int64)
    // and 3 (float64), each tile ranks x64 itself.  y holds 64-bit medians.
    int32_t rank_mode;
    int64_t xshift;      // items added to x per tile of `one`
    int64_t xrow;        // items of x per row of `one` (0: n)
    const void *x64;
};

// Backward launch: grad_y / argmed + y_off (n-k+1), grad_x + x_off (n);
// gradients are float32, or float64 with the 64-bit entry points.
struct BwdLaunch {
    const void *grad_y;
    const int32_t *argmed;
    void *grad_x;
    SigDesc one;
    int64_t rows;
    int64_t tpr;
    const SigDesc *sigs;
    const Unit *units;
    int64_t nunits;
    int32_t seg;         // 1: exact accumulation (float32, every window <= kBwdSegMaxK)
};

// Kernel families: k = 1; LDS tiles of kLdsSmall threads (blocks of up to
// kLdsSmall*kRegs/2 slots) or kLdsLarge threads; the global-memory path.
enum Path { PATH_IDENTITY = 0, PATH_LDS_SMALL = 1, PATH_LDS_LARGE = 2, PATH_GLOBAL = 3, PATH_NONE = -1 };

static const int kLdsSmall = 512;
static const int kLdsLarge = 1024;

static const int kGlobalThreads = 1024;
// Dynamic LDS of a global-memory tile: the sort buffer, then the bucket
// counters (2S 16-bit cells), the histogram row buffers and the copy of the
// merged order (2 Mstride bytes): 64 KB up to k = 16383 (two workgroups per
// CU), 128 KB above.
static const int kGlobalLdsSmall = 64 * 1024;
static const int kGlobalLdsLarge = 128 * 1024;
static const int kBwdThreads = 256;
static const int kBwdTargetsPerWave = 1024;
static const int kBwdTargetsPerBlock = kBwdTargetsPerWave * (kBwdThreads / 64);
static const int kBwdGroup = 4;   // candidate batches whose loads are issued together
// Exact-accumulation backward (float32 gradients): targets per wave and per
// workgroup, and the largest window it serves (larger ones, and float64
// gradients, take the grouping backward).
static const int kBwdSegTargetsPerWave = 512;
static const int kBwdSegTargetsPerBlock = kBwdSegTargetsPerWave * (kBwdThreads / 64);
static const int32_t kBwdSegMaxK = 1025;
static const int kBwdInflight = 4;   // candidate batches of 64 in flight per wave

// Which kernel family serves window k.
Path path_for(int32_t k);
// Tiles of a signal on a path, and the dynamic LDS bytes of one tile.
int64_t tiles_for(Path p, int64_t n, int32_t k);
int64_t lds_bytes_for(Path p, int32_t k);
// Global workspace bytes of one workgroup on the global path.
int64_t global_ws_stride(int32_t k);
// Workspace slots (concurrent tiles) of a global-path launch with this much
// dynamic LDS: two tiles per CU with 64 KB, one with 128 KB.
int64_t global_ws_slots(size_t lds_bytes);

hipError_t launch_forward(Path p, bool f32, const Launch &L, size_t lds_bytes,
                          unsigned char *ws, int64_t ws_stride, int64_t ws_slots,
                          int *d_err, hipStream_t st);

// LDS tiles of a work list as one persistent launch: a resident grid takes
// units from the counter *next, which is cleared on `st` first.
hipError_t launch_forward_persistent(Path p, bool f32, const Launch &L, size_t lds_bytes, uint32_t *next,
                                    int *d_err, hipStream_t st);

hipError_t launch_backward(const BwdLaunch &L, bool f64, hipStream_t st);

// Whether window k takes the exact-accumulation backward, and the backward
// tiles of a signal of length n with window k.
bool bwd_seg_for(int32_t k, bool f64);
int64_t bwd_tiles_for(int64_t n, int32_t k, bool f64);

// 64-bit signals on an LDS path: entries per tile of the rank buffer and
// the rank pre-pass (one workgroup per 1024-thread tile of each row); k = 1
// copies x (`total` items, rows of n) and writes each row's argmed[o] = o.
int64_t rank64_stride_for(Path p, int32_t k);
// Dynamic LDS of a tile that ranks its 64-bit items itself.
int64_t rank64_lds_bytes_for(Path p, int32_t k);
hipError_t launch_rank64(Path p, bool f64, const void *x, int64_t n, int32_t k, uint32_t *keys, int64_t stride,
                         int64_t ntiles, int64_t nunits, hipStream_t st);
// 64-bit signals on the global path: scratch bytes of one workgroup of the
// pair pre-pass, and the pre-pass itself (a grid of `slots` workgroups
// looping over the tiles).
int64_t rank64_pair_scratch(int32_t k);
hipError_t launch_rank64_pair(bool f64, const void *x, int64_t n, int32_t k, uint32_t *keys, int64_t stride,
                              unsigned char *ws, int64_t ws_stride, int64_t slots, int64_t ntiles, int64_t nunits,
                              hipStream_t st);
hipError_t launch_identity64(const void *x, void *y, int32_t *argmed, int64_t total, int64_t n, hipStream_t st);

hipError_t prepare_kernels();

// Fixed device scratch of the entry point that allocates nothing: the first
// kFixedFlagBytes hold its kernels' consistency flag, the rest serves as
// the global path's per-workgroup slots.  fixed_scratch returns this
// device's copy; the first call on a device (create = true) looks its
// address up and clears the flag, waiting for that on `st`.  With create =
// false, *out is null until a call has set the device up.
static const int64_t kFixedScratchBytes = 64ll << 20;
static const int64_t kFixedFlagBytes = 256;
hipError_t fixed_scratch(hipStream_t st, bool create, unsigned char **out);

}  // namespace mf
