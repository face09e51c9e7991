// C ABI of the median filter library (include/mf.h): argument checks,
// kernel-family dispatch, the library-owned workspace, and plans for the
// ragged batch (device work list + captured graph).
#include <hip/hip_runtime.h>

#include <stdarg.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <initializer_list>
#include <utility>
#include <chrono>
#include <thread>
#include <memory>
#include <mutex>
#include <string>
#include <unistd.h>
#include <vector>

#include "../../include/mf.h"
#include "mf_launch.h"

using namespace mf;

// ------------------------------------------------------------------ errors

static thread_local std::string t_last_error;

static mf_status fail(mf_status s, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
static mf_status fail(mf_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    t_last_error = buf;
    return s;
}

static mf_status hip_fail(hipError_t e, const char *what)
{
    return fail(MF_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

#define MF_HIP(call, what)                          \
    do {                                            \
        hipError_t e_ = (call);                     \
        if (e_ != hipSuccess) return hip_fail(e_, what); \
    } while (0)

// ------------------------------------------------------------------ environment

namespace {

// Diagnostics and test switches, read from the environment at each use:
//   MF_WS_LIMIT=<bytes>  workspace requests above it fail with
//                        MF_ERR_NOMEM, as a failed allocation would;
//   MF_LOG=1             plan and autotune decisions on stderr;
//   MF_LEASE_HOLD_US=<us> each workspace lease waits this long before the
//                        caller enqueues (test switch for concurrent use).
int64_t env_ws_limit()
{
    const char *e = getenv("MF_WS_LIMIT");
    return e ? atoll(e) : 0;
}

bool env_log()
{
    const char *e = getenv("MF_LOG");
    return e && e[0] == '1';
}

// MF_LEASE_HOLD_US=<microseconds>: a test switch that keeps each
// workspace lease for this long before its launches are enqueued, so that
// calls from other threads reach acquire_ws while the lease is held.
int64_t env_lease_hold_us()
{
    const char *e = getenv("MF_LEASE_HOLD_US");
    return e ? atoll(e) : 0;
}

}  // namespace

// ------------------------------------------------------------------ device state

namespace {

struct Device {
    bool ready = false;
    int *d_err = nullptr;               // kernel consistency flag
    unsigned char *ws = nullptr;        // global-path workspace
    int64_t ws_bytes = 0;
    hipEvent_t ws_done = nullptr;       // completion of the last use of ws
    std::mutex mu;                      // set-up
    std::mutex ws_mu;                   // held by the one workspace lease
};

const int kMaxDevices = 64;
Device g_dev[kMaxDevices];

mf_status device_state(Device **out)
{
    int dev = 0;
    MF_HIP(hipGetDevice(&dev), "hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(MF_ERR_UNSUPPORTED, "device index %d", dev);
    Device &D = g_dev[dev];
    std::lock_guard<std::mutex> lk(D.mu);
    if (!D.ready) {
        MF_HIP(prepare_kernels(), "hipFuncSetAttribute");
        MF_HIP(hipMalloc(&D.d_err, sizeof(int)), "hipMalloc(error flag)");
        MF_HIP(hipMemset(D.d_err, 0, sizeof(int)), "hipMemset(error flag)");
        MF_HIP(hipEventCreateWithFlags(&D.ws_done, hipEventDisableTiming), "hipEventCreate");
        D.ready = true;
    }
    *out = &D;
    return MF_OK;
}

// The workspace, leased to one caller at a time: the lease holds ws_mu from
// acquire_ws until the caller has enqueued its launches and release_ws has
// recorded ws_done after them (or until the lease is destroyed on an error
// path, which records ws_done as well).  Every use therefore waits on the
// stream for the use leased before it, so ws_done, recorded by the last
// lease, completes only after every earlier use: a buffer that must grow is
// freed after waiting for that one event.
struct WsLease {
    Device *D = nullptr;
    hipStream_t st = nullptr;
    std::unique_lock<std::mutex> lk;
    unsigned char *ws = nullptr;
    ~WsLease()
    {
        if (D && lk.owns_lock()) (void)hipEventRecord(D->ws_done, st);
    }
};

mf_status acquire_ws(Device &D, int64_t bytes, hipStream_t st, WsLease &L)
{
    const int64_t limit = env_ws_limit();
    if (limit > 0 && bytes > limit)
        return fail(MF_ERR_NOMEM, "workspace of %lld bytes (over MF_WS_LIMIT = %lld)", (long long)bytes,
                    (long long)limit);
    L.lk = std::unique_lock<std::mutex>(D.ws_mu);
    if (D.ws_bytes < bytes) {
        if (D.ws) {
            MF_HIP(hipEventSynchronize(D.ws_done), "hipEventSynchronize");
            MF_HIP(hipFree(D.ws), "hipFree(workspace)");
            D.ws = nullptr;
            D.ws_bytes = 0;
        }
        if (hipMalloc(&D.ws, (size_t)bytes) != hipSuccess) {
            D.ws = nullptr;
            return fail(MF_ERR_NOMEM, "workspace of %lld bytes", (long long)bytes);
        }
        D.ws_bytes = bytes;
    }
    MF_HIP(hipStreamWaitEvent(st, D.ws_done, 0), "hipStreamWaitEvent");
    L.D = &D;
    L.st = st;
    L.ws = D.ws;
    const int64_t hold = env_lease_hold_us();
    if (hold > 0) std::this_thread::sleep_for(std::chrono::microseconds(hold));
    return MF_OK;
}

mf_status release_ws(WsLease &L)
{
    const hipError_t e = hipEventRecord(L.D->ws_done, L.st);
    L.lk.unlock();
    if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    return MF_OK;
}

// ------------------------------------------------------------------ checks

mf_status check_signal(int64_t n, int32_t k)
{
    if (n < 1) return fail(MF_ERR_INVALID_VALUE, "n = %lld must be >= 1", (long long)n);
    if (k < 1 || (k & 1) == 0) return fail(MF_ERR_INVALID_VALUE, "k = %d must be odd and >= 1", k);
    if (k > n) return fail(MF_ERR_INVALID_VALUE, "k = %d exceeds n = %lld", k, (long long)n);
    if (n > INT32_MAX) return fail(MF_ERR_UNSUPPORTED, "n = %lld exceeds 2^31-1", (long long)n);
    if (path_for(k) == PATH_NONE) return fail(MF_ERR_UNSUPPORTED, "k = %d exceeds 32767", k);
    return MF_OK;
}

// Forward over `rows` equal signals (rows = 1: one signal).
mf_status forward_rows(const void *x, int64_t rows, int64_t n, int32_t k, void *y,
                       int32_t *argmed, bool f32, hipStream_t st)
{
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    if (rows < 1) return fail(MF_ERR_INVALID_VALUE, "rows = %lld must be >= 1", (long long)rows);
    mf_status s = check_signal(n, k);
    if (s != MF_OK) return s;
    Device *D = nullptr;
    if ((s = device_state(&D)) != MF_OK) return s;

    const Path p = path_for(k);
    const int64_t tpr = tiles_for(p, n, k);
    Launch L;
    memset(&L, 0, sizeof L);
    L.x = x;
    L.y = y;
    L.argmed = argmed;
    L.one.n = n;
    L.one.k = k;
    L.rows = rows;
    L.tpr = tpr;
    L.nunits = rows * tpr;
    if (p != PATH_IDENTITY && p != PATH_GLOBAL && L.nunits > 0x7FFFFFFFll)
        return fail(MF_ERR_UNSUPPORTED, "too many tiles (%lld)", (long long)L.nunits);
    const size_t lds = (size_t)lds_bytes_for(p, k);
    if (p == PATH_GLOBAL) {
        const int64_t stride = global_ws_stride(k);
        const int64_t slots = std::min<int64_t>(global_ws_slots(lds), L.nunits);
        WsLease lease;
        if ((s = acquire_ws(*D, stride * slots, st, lease)) != MF_OK) return s;
        MF_HIP(launch_forward(p, f32, L, lds, lease.ws, stride, slots, D->d_err, st), "forward launch");
        return release_ws(lease);
    }
    MF_HIP(launch_forward(p, f32, L, lds, nullptr, 0, 0, D->d_err, st), "forward launch");
    return MF_OK;
}

// Forward of `rows` 64-bit signals of length n (back to back) through the
// int32 tile kernels on 32-bit rank keys, which copy each median from the
// 64-bit x to y.  512-thread tiles rank their items in LDS; for 1024-thread
// tiles and one-pair tiles a pre-pass writes the keys unit by unit
// (unit = row * tiles + tile, (P+1)k entries each) into the workspace and
// each tile reads its span.
mf_status forward64(const void *x, int64_t rows, int64_t n, int32_t k, void *y, int32_t *argmed, bool f64,
                    hipStream_t st)
{
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    if (rows < 1) return fail(MF_ERR_INVALID_VALUE, "rows = %lld must be >= 1", (long long)rows);
    mf_status s = check_signal(n, k);
    if (s != MF_OK) return s;
    const Path p = path_for(k);
    const int64_t tiles = tiles_for(p, n, k);
    if (p != PATH_IDENTITY && p != PATH_GLOBAL && rows * tiles > 0x7FFFFFFFll)
        return fail(MF_ERR_UNSUPPORTED, "too many tiles (%lld)", (long long)(rows * tiles));
    Device *D = nullptr;
    if ((s = device_state(&D)) != MF_OK) return s;
    if (p == PATH_IDENTITY) {
        MF_HIP(launch_identity64(x, y, argmed, rows * n, n, st), "64-bit identity launch");
        return MF_OK;
    }
    const int64_t units = rows * tiles;
    Launch L;
    memset(&L, 0, sizeof L);
    L.y = y;
    L.argmed = argmed;
    L.one.n = n;
    L.one.k = k;
    L.rows = rows;
    L.tpr = tiles;
    L.nunits = units;
    L.x64 = x;
    if (p == PATH_LDS_SMALL) {   // 512-thread tiles rank their items in LDS
        L.x = x;
        L.rank_mode = f64 ? 3 : 2;
        MF_HIP(launch_forward(p, false, L, (size_t)rank64_lds_bytes_for(p, k), nullptr, 0, 0, D->d_err, st),
               "64-bit forward launch");
        return MF_OK;
    }
    const int64_t stride = rank64_stride_for(p, k);
    const int64_t key_bytes = (units * stride * 4 + 255) & ~255ll;
    L.rank_mode = 1;
    L.xshift = k;
    L.xrow = tiles * stride;
    WsLease lease;
    if (p == PATH_GLOBAL) {
        // one pair per tile: a pre-pass ranks each pair through its
        // workgroup's scratch, then the global-path tiles run on the ranks;
        // the scratch of the pre-pass and the tiles' workspace share memory
        const size_t lds = (size_t)lds_bytes_for(p, k);
        const int64_t gstride = global_ws_stride(k);
        const int64_t gslots = std::min<int64_t>(global_ws_slots(lds), units);
        const int64_t pstride = rank64_pair_scratch(k);
        const int64_t pslots = std::min<int64_t>(256, units);
        const int64_t scratch = std::max<int64_t>(gstride * gslots, pstride * pslots);
        if ((s = acquire_ws(*D, key_bytes + scratch, st, lease)) != MF_OK) return s;
        unsigned char *ws = lease.ws;
        uint32_t *keys = (uint32_t *)ws;
        MF_HIP(launch_rank64_pair(f64, x, n, k, keys, stride, ws + key_bytes, pstride, pslots, tiles, units, st),
               "64-bit pair rank launch");
        L.x = keys;
        MF_HIP(launch_forward(p, false, L, lds, ws + key_bytes, gstride, gslots, D->d_err, st),
               "64-bit forward launch");
        return release_ws(lease);
    }
    if ((s = acquire_ws(*D, key_bytes, st, lease)) != MF_OK) return s;
    uint32_t *keys = (uint32_t *)lease.ws;
    MF_HIP(launch_rank64(p, f64, x, n, k, keys, stride, tiles, units, st), "64-bit rank launch");
    L.x = keys;
    MF_HIP(launch_forward(p, false, L, (size_t)lds_bytes_for(p, k), nullptr, 0, 0, D->d_err, st),
           "64-bit forward launch");
    return release_ws(lease);
}

// Backward over `rows` equal signals; f64: float64 gradients.
mf_status backward_rows(const void *gy, const int32_t *argmed, int64_t rows, int64_t n,
                        int32_t k, void *gx, bool f64, hipStream_t st)
{
    if (!gy || !argmed || !gx) return fail(MF_ERR_INVALID_VALUE, "grad_y, argmed and grad_x must not be null");
    if (rows < 1) return fail(MF_ERR_INVALID_VALUE, "rows = %lld must be >= 1", (long long)rows);
    mf_status s = check_signal(n, k);
    if (s != MF_OK) return s;
    Device *D = nullptr;
    if ((s = device_state(&D)) != MF_OK) return s;
    BwdLaunch L;
    memset(&L, 0, sizeof L);
    L.grad_y = gy;
    L.argmed = argmed;
    L.grad_x = gx;
    L.one.n = n;
    L.one.k = k;
    L.rows = rows;
    L.tpr = bwd_tiles_for(n, k, f64);
    L.nunits = rows * L.tpr;
    L.seg = bwd_seg_for(k, f64) ? 1 : 0;
    MF_HIP(launch_backward(L, f64, st), "backward launch");
    return MF_OK;
}

}  // namespace

// ------------------------------------------------------------------ plans

struct PathGroup {
    Path path;
    bool persistent = false;     // resident grid over a work counter
    bool owns = true;            // d_units belongs to this group
    int64_t nunits = 0;
    SigDesc *d_sigs = nullptr;   // all signals of the plan
    Unit *d_units = nullptr;
    size_t lds = 0;
    int64_t ws_stride = 0;
};

const int kConfigs = 3;              // mf_launch_config values
const int kDefaultConfig = MF_LAUNCH_PERSISTENT;

// Tile shape buckets: windows whose slot stride is 2^b (b < kShapeBuckets)
// may run as 512- or 1024-thread tiles.
const int kShapeBuckets = 12;   // slot strides 1 .. 2048

struct mf_plan {
    int32_t num_signals = 0;
    int64_t total_in = 0, total_out = 0;
    std::vector<int64_t> offsets;
    std::vector<int32_t> ks;
    std::vector<SigDesc> sigs;                 // host copy of d_sigs
    int32_t bucket_threads[kShapeBuckets];     // 512 or 1024 per bucket
    SigDesc *d_sigs = nullptr;
    std::vector<PathGroup> groups[kConfigs];   // forward launches per configuration
    int32_t config = kDefaultConfig;
    float tuned_ms[kConfigs] = {-1.f, -1.f, -1.f};
    uint32_t *d_next = nullptr;                // work counters, one per group
    // backward work list
    // backward work lists (float32 gradients): [0] signals of the
    // exact-accumulation backward, [1] the others
    Unit *d_bunits[2] = {nullptr, nullptr};
    int64_t nbunits[2] = {0, 0};
    // captured forward graph and what it was captured with
    hipGraphExec_t gexec = nullptr;
    const void *gx = nullptr;
    void *gy = nullptr;
    int32_t *gam = nullptr;
    unsigned char *gws = nullptr;
    int32_t gconfig = -1;
    bool gf32 = true;
    int64_t ws_need = 0;
    // executions of one plan are serialized: on the host by mu (capture and
    // launch), on the device by done (the work counters and the captured
    // graph belong to one execution at a time)
    std::mutex mu;
    hipEvent_t done = nullptr;     // completion of the last execution
};

static void plan_free_groups(mf_plan *p)
{
    for (auto &gs : p->groups) {
        for (auto &g : gs)
            if (g.owns && g.d_units) (void)hipFree(g.d_units);
        gs.clear();
    }
    p->ws_need = 0;
}

static void plan_free(mf_plan *p)
{
    if (!p) return;
    if (p->done) {
        (void)hipEventSynchronize(p->done);
        (void)hipEventDestroy(p->done);
    }
    if (p->gexec) (void)hipGraphExecDestroy(p->gexec);
    plan_free_groups(p);
    if (p->d_sigs) (void)hipFree(p->d_sigs);
    if (p->d_next) (void)hipFree(p->d_next);
    for (int i = 0; i < 2; i++)
        if (p->d_bunits[i]) (void)hipFree(p->d_bunits[i]);
    delete p;
}

static int shape_bucket(int32_t k)
{
    int b = 0;
    while ((1 << b) < k) b++;
    return b;
}

// The LDS family a window runs in under the plan's tile shapes.
static Path plan_family(const mf_plan *p, int32_t k)
{
    const Path f = path_for(k);
    if (f == PATH_LDS_SMALL && p->bucket_threads[shape_bucket(k)] == kLdsLarge) return PATH_LDS_LARGE;
    return f;
}

// Uploads a work list as a new group of configuration `cfg`.
static mf_status plan_add_group(mf_plan *p, int cfg, Path f, bool persistent, const std::vector<Unit> &units,
                                size_t lds, int64_t ws_stride)
{
    if (f != PATH_IDENTITY && f != PATH_GLOBAL && units.size() > 0x7FFFFFFFull)
        return fail(MF_ERR_UNSUPPORTED, "too many tiles in one batch");
    PathGroup g;
    g.path = f;
    g.persistent = persistent;
    g.nunits = (int64_t)units.size();
    g.lds = lds;
    g.ws_stride = ws_stride;
    g.d_sigs = p->d_sigs;
    hipError_t e = hipMalloc(&g.d_units, sizeof(Unit) * units.size());
    if (e == hipSuccess) e = hipMemcpy(g.d_units, units.data(), sizeof(Unit) * units.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        if (g.d_units) (void)hipFree(g.d_units);
        return hip_fail(e, "plan work list");
    }
    if (f == PATH_GLOBAL) p->ws_need = std::max(p->ws_need, ws_stride * std::min<int64_t>(global_ws_slots(lds), g.nunits));
    p->groups[cfg].push_back(g);
    return MF_OK;
}

// ------------------------------------------------------------------ tile shape cache
//
// MF_TUNE_CACHE=<path>: a JSON file of tuned tile shapes, read when a plan
// is created and updated by mf_plan_autotune:
//   {"tile_threads": {"f32": {"<slot stride>": 512 or 1024, ...}}}
// (tuned on float32 signals; plans use it for every element type).

static const char *env_tune_cache()
{
    const char *e = getenv("MF_TUNE_CACHE");
    return (e && e[0]) ? e : nullptr;
}

// Entries "<stride>": <threads> of the "f32" object in the cache file.
static std::vector<std::pair<int64_t, int64_t>> tune_cache_read(const char *path)
{
    std::vector<std::pair<int64_t, int64_t>> out;
    FILE *f = fopen(path, "rb");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, got);
    fclose(f);
    const size_t at = text.find("\"f32\"");
    if (at == std::string::npos) return out;
    const size_t open = text.find('{', at), close = text.find('}', at);
    if (open == std::string::npos || close == std::string::npos || close < open) return out;
    size_t i = open + 1;
    while (i < close) {
        const size_t q1 = text.find('"', i);
        if (q1 == std::string::npos || q1 >= close) break;
        const size_t q2 = text.find('"', q1 + 1);
        const size_t colon = text.find(':', q2);
        if (q2 == std::string::npos || colon == std::string::npos || colon >= close) break;
        const int64_t key = atoll(text.c_str() + q1 + 1);
        const int64_t val = atoll(text.c_str() + colon + 1);
        out.emplace_back(key, val);
        i = colon + 1;
    }
    return out;
}

static void tune_cache_apply(mf_plan *p)
{
    const char *path = env_tune_cache();
    if (!path) return;
    for (const auto &kv : tune_cache_read(path)) {
        int b = 0;
        while (b < kShapeBuckets && (1ll << b) != kv.first) b++;
        if (b < kShapeBuckets && (kv.second == kLdsSmall || kv.second == kLdsLarge))
            p->bucket_threads[b] = (int32_t)kv.second;
    }
}

// Merges the plan's tuned buckets into the cache file (written whole to a
// temporary file of this process, then renamed over the old one; writers
// of one process take turns).
static void tune_cache_write(const mf_plan *p, const bool (&tuned)[kShapeBuckets])
{
    const char *path = env_tune_cache();
    if (!path) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lk(mu);
    int64_t threads[kShapeBuckets] = {0};
    for (const auto &kv : tune_cache_read(path))
        for (int b = 0; b < kShapeBuckets; b++)
            if ((1ll << b) == kv.first) threads[b] = kv.second;
    for (int b = 0; b < kShapeBuckets; b++)
        if (tuned[b]) threads[b] = p->bucket_threads[b];
    std::string text = "{\"tile_threads\": {\"f32\": {";
    bool first = true;
    for (int b = 0; b < kShapeBuckets; b++) {
        if (threads[b] != kLdsSmall && threads[b] != kLdsLarge) continue;
        char item[64];
        snprintf(item, sizeof item, "%s\"%lld\": %lld", first ? "" : ", ", 1ll << b, (long long)threads[b]);
        text += item;
        first = false;
    }
    text += "}}}\n";
    const std::string tmp = std::string(path) + ".tmp." + std::to_string((long long)getpid());
    FILE *f = fopen(tmp.c_str(), "wb");
    if (!f) return;
    const bool ok = fwrite(text.data(), 1, text.size(), f) == text.size();
    if (fclose(f) == 0 && ok) (void)rename(tmp.c_str(), path);
}

// Forward work lists of every launch configuration, from the plan's
// signals and tile shapes.  One list per kernel family; within a family the
// longest windows go first so that the heaviest tiles start early.
// MF_LAUNCH_PER_FAMILY and MF_LAUNCH_PERSISTENT share these lists (windows
// of a shape bucket tuned to 1024 threads join the 1024-thread family);
// MF_LAUNCH_PERSISTENT_ONE puts every LDS tile into one list of 1024-thread
// tiles, launched first.
static mf_status plan_build_groups(mf_plan *p)
{
    plan_free_groups(p);
    const int32_t num_signals = p->num_signals;
    const int32_t *ks = p->ks.data();
    const std::vector<SigDesc> &sigs = p->sigs;
    const Path fams[4] = {PATH_LDS_LARGE, PATH_LDS_SMALL, PATH_GLOBAL, PATH_IDENTITY};
    std::vector<int32_t> order((size_t)num_signals);
    for (int32_t s = 0; s < num_signals; s++) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return ks[a] > ks[b]; });
    mf_status st = MF_OK;
    {
        std::vector<Unit> units;
        size_t lds = 0;
        for (int32_t s : order) {
            const Path f = path_for(ks[s]);
            if (f != PATH_LDS_SMALL && f != PATH_LDS_LARGE) continue;
            const int64_t nt = tiles_for(PATH_LDS_LARGE, sigs[s].n, ks[s]);
            for (int64_t t = 0; t < nt; t++) units.push_back(Unit{s, 0, t});
            lds = std::max(lds, (size_t)lds_bytes_for(PATH_LDS_LARGE, ks[s]));
        }
        if (!units.empty() && (st = plan_add_group(p, MF_LAUNCH_PERSISTENT_ONE, PATH_LDS_LARGE, true, units, lds, 0)) != MF_OK)
            return st;
    }
    for (Path f : fams) {
        std::vector<Unit> units;
        size_t lds = 0;
        int64_t ws_stride = 0;
        for (int32_t s : order) {
            if (plan_family(p, ks[s]) != f) continue;
            const int64_t nt = tiles_for(f, sigs[s].n, ks[s]);
            for (int64_t t = 0; t < nt; t++) units.push_back(Unit{s, 0, t});
            lds = std::max(lds, (size_t)lds_bytes_for(f, ks[s]));
            if (f == PATH_GLOBAL) ws_stride = std::max(ws_stride, global_ws_stride(ks[s]));
        }
        if (units.empty()) continue;
        if ((st = plan_add_group(p, MF_LAUNCH_PER_FAMILY, f, false, units, lds, ws_stride)) != MF_OK) return st;
        PathGroup shared = p->groups[MF_LAUNCH_PER_FAMILY].back();
        shared.owns = false;
        shared.persistent = (f == PATH_LDS_SMALL || f == PATH_LDS_LARGE);
        p->groups[MF_LAUNCH_PERSISTENT].push_back(shared);
        if (f == PATH_GLOBAL || f == PATH_IDENTITY) {
            shared.persistent = false;
            p->groups[MF_LAUNCH_PERSISTENT_ONE].push_back(shared);
        }
    }
    return MF_OK;
}

extern "C" mf_status mf_plan_create_batched(const int64_t *x_offsets, const int32_t *ks,
                                            int32_t num_signals, mf_plan **out)
{
    if (!out) return fail(MF_ERR_INVALID_VALUE, "out must not be null");
    *out = nullptr;
    if (!x_offsets || !ks) return fail(MF_ERR_INVALID_VALUE, "x_offsets and ks must not be null");
    if (num_signals < 1) return fail(MF_ERR_INVALID_VALUE, "num_signals = %d must be >= 1", num_signals);
    if (x_offsets[0] != 0) return fail(MF_ERR_INVALID_VALUE, "x_offsets[0] must be 0");
    std::vector<SigDesc> sigs((size_t)num_signals);
    int64_t yoff = 0;
    for (int32_t s = 0; s < num_signals; s++) {
        const int64_t n = x_offsets[s + 1] - x_offsets[s];
        mf_status st = check_signal(n, ks[s]);
        if (st != MF_OK) return fail(st, "signal %d: %s", s, t_last_error.c_str());
        sigs[s].x_off = x_offsets[s];
        sigs[s].y_off = yoff;
        sigs[s].n = n;
        sigs[s].k = ks[s];
        sigs[s].pad = 0;
        yoff += n - ks[s] + 1;
    }
    Device *D = nullptr;
    mf_status st = device_state(&D);
    if (st != MF_OK) return st;

    mf_plan *p = new mf_plan();
    p->num_signals = num_signals;
    p->total_in = x_offsets[num_signals];
    p->total_out = yoff;
    p->offsets.assign(x_offsets, x_offsets + num_signals + 1);
    p->ks.assign(ks, ks + num_signals);

    hipError_t e = hipMalloc(&p->d_sigs, sizeof(SigDesc) * sigs.size());
    if (e == hipSuccess) e = hipMemcpy(p->d_sigs, sigs.data(), sizeof(SigDesc) * sigs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMalloc(&p->d_next, sizeof(uint32_t) * 8);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&p->done, hipEventDisableTiming);
    if (e != hipSuccess) { plan_free(p); return hip_fail(e, "plan signal table"); }

    for (int b = 0; b < kShapeBuckets; b++) p->bucket_threads[b] = kLdsSmall;
    tune_cache_apply(p);
    p->sigs = sigs;
    if ((st = plan_build_groups(p)) != MF_OK) { plan_free(p); return st; }
    // backward work list
    {
        std::vector<Unit> bunits[2];
        for (int32_t s = 0; s < num_signals; s++) {
            const int32_t k = sigs[s].k;
            const int list = bwd_seg_for(k, false) ? 0 : 1;
            const int64_t nt = bwd_tiles_for(sigs[s].n, k, false);
            for (int64_t t = 0; t < nt; t++) bunits[list].push_back(Unit{s, 0, t});
        }
        for (int i = 0; i < 2 && e == hipSuccess; i++) {
            p->nbunits[i] = (int64_t)bunits[i].size();
            if (bunits[i].empty()) continue;
            e = hipMalloc(&p->d_bunits[i], sizeof(Unit) * bunits[i].size());
            if (e == hipSuccess)
                e = hipMemcpy(p->d_bunits[i], bunits[i].data(), sizeof(Unit) * bunits[i].size(), hipMemcpyHostToDevice);
        }
        if (e != hipSuccess) { plan_free(p); return hip_fail(e, "plan backward work list"); }
    }
    if (env_log()) {
        static const char *names[] = {"k=1", "lds512", "lds1024", "global"};
        fprintf(stderr, "mf: plan of %d signals, %lld outputs\n", num_signals, (long long)p->total_out);
        for (int c = 0; c < kConfigs; c++)
            for (const PathGroup &g : p->groups[c])
                fprintf(stderr, "mf:   config %d: %s, %lld units, %zu B LDS%s\n", c, names[g.path],
                        (long long)g.nunits, g.lds, g.persistent ? ", persistent" : "");
    }
    *out = p;
    return MF_OK;
}

static mf_status plan_enqueue(mf_plan *p, Device &D, const void *x, void *y, int32_t *argmed,
                              unsigned char *ws, bool f32, hipStream_t st)
{
    const std::vector<PathGroup> &gs = p->groups[p->config];
    for (size_t gi = 0; gi < gs.size(); gi++) {
        const PathGroup &g = gs[gi];
        Launch L;
        memset(&L, 0, sizeof L);
        L.x = x;
        L.y = y;
        L.argmed = argmed;
        L.sigs = g.d_sigs;
        L.units = g.d_units;
        L.nunits = g.nunits;
        if (g.persistent) {
            MF_HIP(launch_forward_persistent(g.path, f32, L, g.lds, p->d_next + gi, D.d_err, st),
                   "batched persistent launch");
            continue;
        }
        const int64_t slots = std::min<int64_t>(global_ws_slots(g.lds), g.nunits);
        MF_HIP(launch_forward(g.path, f32, L, g.lds, ws, g.ws_stride, slots, D.d_err, st), "batched launch");
    }
    return MF_OK;
}

// One execution of plan p; the caller holds p->mu.
static mf_status plan_execute_locked(mf_plan *p, const void *x, void *y, int32_t *argmed, bool f32, void *stream)
{
    hipStream_t st = (hipStream_t)stream;
    Device *D = nullptr;
    mf_status s = device_state(&D);
    if (s != MF_OK) return s;
    WsLease lease;
    if (p->ws_need > 0 && (s = acquire_ws(*D, p->ws_need, st, lease)) != MF_OK) return s;
    unsigned char *ws = lease.ws;
    // the previous execution (maybe on another stream) has finished with the
    // work counters before this one clears them
    MF_HIP(hipStreamWaitEvent(st, p->done, 0), "hipStreamWaitEvent(plan)");
    // the graph bakes in the data and workspace pointers; capture again
    // when any of them changed (after the last launch of the old graph)
    if (!p->gexec || p->gx != x || p->gy != y || p->gam != argmed || p->gws != ws || p->gconfig != p->config ||
        p->gf32 != f32) {
        if (p->gexec) {
            MF_HIP(hipEventSynchronize(p->done), "hipEventSynchronize(plan)");
            (void)hipGraphExecDestroy(p->gexec);
            p->gexec = nullptr;
        }
        hipStream_t cs;
        MF_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking), "hipStreamCreate(capture)");
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        mf_status es = MF_OK;
        if (e == hipSuccess) es = plan_enqueue(p, *D, x, y, argmed, ws, f32, cs);
        hipError_t e2 = (e == hipSuccess) ? hipStreamEndCapture(cs, &graph) : e;
        if (e2 == hipSuccess && es == MF_OK) e2 = hipGraphInstantiate(&p->gexec, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (es != MF_OK) return es;
        if (e2 != hipSuccess) { p->gexec = nullptr; return hip_fail(e2, "graph capture"); }
        p->gx = x;
        p->gy = y;
        p->gam = argmed;
        p->gws = ws;
        p->gconfig = p->config;
        p->gf32 = f32;
    }
    MF_HIP(hipGraphLaunch(p->gexec, st), "hipGraphLaunch");
    MF_HIP(hipEventRecord(p->done, st), "hipEventRecord(plan)");
    if (p->ws_need > 0) return release_ws(lease);
    return MF_OK;
}

static mf_status plan_execute(mf_plan *p, const void *x, void *y, int32_t *argmed, bool f32, void *stream)
{
    if (!p) return fail(MF_ERR_INVALID_VALUE, "plan must not be null");
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    std::lock_guard<std::mutex> plk(p->mu);
    return plan_execute_locked(p, x, y, argmed, f32, stream);
}

extern "C" mf_status mf_plan_execute(mf_plan *p, const float *x, float *y, int32_t *argmed, void *stream)
{
    return plan_execute(p, x, y, argmed, true, stream);
}

extern "C" mf_status mf_plan_execute_i32(mf_plan *p, const int32_t *x, int32_t *y, int32_t *argmed, void *stream)
{
    return plan_execute(p, x, y, argmed, false, stream);
}

// One execution of plan p on 64-bit signals (f64: float64, else int64).
// The 512-thread tile family (windows up to 2047) runs as one launch over
// the plan's work list, each tile ranking its 64-bit items in LDS; signals
// of the other families run one after another through the single-signal
// path (rank pre-pass in the workspace, then their tiles).
static mf_status plan_execute64(mf_plan *p, const void *x, void *y, int32_t *argmed, bool f64, void *stream)
{
    if (!p) return fail(MF_ERR_INVALID_VALUE, "plan must not be null");
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    hipStream_t st = (hipStream_t)stream;
    Device *D = nullptr;
    mf_status s = device_state(&D);
    if (s != MF_OK) return s;
    std::lock_guard<std::mutex> plk(p->mu);
    MF_HIP(hipStreamWaitEvent(st, p->done, 0), "hipStreamWaitEvent(plan)");
    for (const PathGroup &g : p->groups[MF_LAUNCH_PER_FAMILY]) {
        if (g.path != PATH_LDS_SMALL) continue;
        size_t lds = 0;
        for (int32_t q = 0; q < p->num_signals; q++)
            if (path_for(p->ks[q]) == PATH_LDS_SMALL)
                lds = std::max(lds, (size_t)rank64_lds_bytes_for(PATH_LDS_SMALL, p->ks[q]));
        Launch L;
        memset(&L, 0, sizeof L);
        L.x = x;
        L.x64 = x;
        L.y = y;
        L.argmed = argmed;
        L.sigs = g.d_sigs;
        L.units = g.d_units;
        L.nunits = g.nunits;
        L.rank_mode = f64 ? 3 : 2;
        MF_HIP(launch_forward(PATH_LDS_SMALL, false, L, lds, nullptr, 0, 0, D->d_err, st), "64-bit batched launch");
    }
    const unsigned char *xb = (const unsigned char *)x;
    unsigned char *yb = (unsigned char *)y;
    int64_t yoff = 0;
    for (int32_t q = 0; q < p->num_signals; q++) {
        const int64_t n = p->offsets[q + 1] - p->offsets[q];
        const int32_t k = p->ks[q];
        if (path_for(k) != PATH_LDS_SMALL &&
            (s = forward64(xb + 8 * p->offsets[q], 1, n, k, yb + 8 * yoff, argmed ? argmed + yoff : nullptr, f64,
                           st)) != MF_OK)
            return s;
        yoff += n - k + 1;
    }
    MF_HIP(hipEventRecord(p->done, st), "hipEventRecord(plan)");
    return MF_OK;
}

extern "C" mf_status mf_plan_execute_f64(mf_plan *p, const double *x, double *y, int32_t *argmed, void *stream)
{
    return plan_execute64(p, x, y, argmed, true, stream);
}

extern "C" mf_status mf_plan_execute_i64(mf_plan *p, const int64_t *x, int64_t *y, int32_t *argmed, void *stream)
{
    return plan_execute64(p, x, y, argmed, false, stream);
}

extern "C" mf_status mf_plan_execute_backward(mf_plan *p, const float *grad_y, const int32_t *argmed,
                                              float *grad_x, void *stream)
{
    if (!p) return fail(MF_ERR_INVALID_VALUE, "plan must not be null");
    if (!grad_y || !argmed || !grad_x) return fail(MF_ERR_INVALID_VALUE, "grad_y, argmed and grad_x must not be null");
    BwdLaunch L;
    memset(&L, 0, sizeof L);
    L.grad_y = grad_y;
    L.argmed = argmed;
    L.grad_x = grad_x;
    L.sigs = p->d_sigs;
    std::lock_guard<std::mutex> plk(p->mu);
    for (int i = 0; i < 2; i++) {
        if (p->nbunits[i] == 0) continue;
        L.units = p->d_bunits[i];
        L.nunits = p->nbunits[i];
        L.seg = i == 0 ? 1 : 0;
        MF_HIP(launch_backward(L, false, (hipStream_t)stream), "batched backward launch");
    }
    MF_HIP(hipEventRecord(p->done, (hipStream_t)stream), "hipEventRecord(plan)");
    return MF_OK;
}

extern "C" int64_t mf_plan_output_length(const mf_plan *p) { return p ? p->total_out : -1; }

extern "C" mf_status mf_plan_set_config(mf_plan *p, int32_t config)
{
    if (!p) return fail(MF_ERR_INVALID_VALUE, "plan must not be null");
    if (config < 0 || config >= kConfigs)
        return fail(MF_ERR_INVALID_VALUE, "config = %d is not a launch configuration", config);
    std::lock_guard<std::mutex> plk(p->mu);
    p->config = config;
    return MF_OK;
}

extern "C" mf_status mf_plan_get_tile_threads(const mf_plan *p, int32_t k, int32_t *threads)
{
    if (!p || !threads) return fail(MF_ERR_INVALID_VALUE, "plan and threads must not be null");
    if (k < 1 || (k & 1) == 0 || path_for(k) == PATH_NONE)
        return fail(MF_ERR_INVALID_VALUE, "k = %d is not a supported window", k);
    const Path f = plan_family(p, k);
    *threads = f == PATH_LDS_SMALL ? kLdsSmall : f == PATH_LDS_LARGE ? kLdsLarge : 0;
    return MF_OK;
}

extern "C" mf_status mf_plan_get_config(const mf_plan *p, int32_t *config, float *tuned_ms)
{
    if (!p || !config) return fail(MF_ERR_INVALID_VALUE, "plan and config must not be null");
    *config = p->config;
    if (tuned_ms)
        for (int c = 0; c < kConfigs; c++) tuned_ms[c] = p->tuned_ms[c];
    return MF_OK;
}

// Tile shapes: for every shape bucket of windows that fit 512-thread
// tiles, the bucket's signals are timed as 512- and as 1024-thread tiles on
// the caller's buffers (one launch each, after a warm-up), and the faster
// shape is kept; the plan's work lists are then rebuilt and the cache file
// (MF_TUNE_CACHE) updated.  The caller holds p->mu.
static mf_status tune_shapes(mf_plan *p, const float *x, float *y, int32_t *argmed, int32_t reps, hipStream_t st,
                             hipEvent_t a, hipEvent_t b)
{
    Device *D = nullptr;
    mf_status s = device_state(&D);
    if (s != MF_OK) return s;
    // the captured graph and the work lists of an earlier execution go
    MF_HIP(hipEventSynchronize(p->done), "hipEventSynchronize(plan)");
    if (p->gexec) {
        (void)hipGraphExecDestroy(p->gexec);
        p->gexec = nullptr;
    }
    bool tuned[kShapeBuckets] = {false};
    for (int bk = 0; bk < kShapeBuckets; bk++) {
        float best_ms = -1.f;
        int32_t best_nt = p->bucket_threads[bk];
        for (int32_t nt : {kLdsSmall, kLdsLarge}) {
            const Path f = nt == kLdsSmall ? PATH_LDS_SMALL : PATH_LDS_LARGE;
            std::vector<Unit> units;
            size_t lds = 0;
            for (int32_t q = 0; q < p->num_signals; q++) {
                const int32_t k = p->ks[q];
                if (path_for(k) != PATH_LDS_SMALL || shape_bucket(k) != bk) continue;
                const int64_t tiles = tiles_for(f, p->sigs[q].n, k);
                for (int64_t t = 0; t < tiles; t++) units.push_back(Unit{q, 0, t});
                lds = std::max(lds, (size_t)lds_bytes_for(f, k));
            }
            if (units.empty()) break;
            Unit *du = nullptr;
            MF_HIP(hipMalloc(&du, sizeof(Unit) * units.size()), "hipMalloc(tuning work list)");
            hipError_t e = hipMemcpy(du, units.data(), sizeof(Unit) * units.size(), hipMemcpyHostToDevice);
            Launch L;
            memset(&L, 0, sizeof L);
            L.x = x;
            L.y = y;
            L.argmed = argmed;
            L.sigs = p->d_sigs;
            L.units = du;
            L.nunits = (int64_t)units.size();
            if (e == hipSuccess) e = launch_forward(f, true, L, lds, nullptr, 0, 0, D->d_err, st);
            if (e == hipSuccess) e = hipEventRecord(a, st);
            for (int r = 0; r < reps && e == hipSuccess; r++) e = launch_forward(f, true, L, lds, nullptr, 0, 0, D->d_err, st);
            if (e == hipSuccess) e = hipEventRecord(b, st);
            if (e == hipSuccess) e = hipEventSynchronize(b);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
            const hipError_t ef = hipFree(du);
            if (e != hipSuccess) return hip_fail(e, "tile shape tuning");
            if (ef != hipSuccess) return hip_fail(ef, "hipFree(tuning work list)");
            if (best_ms < 0.f || ms < best_ms) {
                best_ms = ms;
                best_nt = nt;
            }
            tuned[bk] = true;
        }
        if (tuned[bk]) {
            p->bucket_threads[bk] = best_nt;
            if (env_log()) fprintf(stderr, "mf: autotune slot stride %d: %d-thread tiles\n", 1 << bk, best_nt);
        }
    }
    if ((s = plan_build_groups(p)) != MF_OK) return s;
    tune_cache_write(p, tuned);
    return MF_OK;
}

extern "C" mf_status mf_plan_autotune(mf_plan *p, const float *x, float *y, int32_t *argmed, int32_t reps,
                                      void *stream)
{
    if (!p) return fail(MF_ERR_INVALID_VALUE, "plan must not be null");
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    if (reps < 1 || reps > 100) return fail(MF_ERR_INVALID_VALUE, "reps = %d must be in 1..100", reps);
    hipStream_t st = (hipStream_t)stream;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    MF_HIP(hipStreamIsCapturing(st, &cs), "hipStreamIsCapturing");
    if (cs != hipStreamCaptureStatusNone) return fail(MF_ERR_UNSUPPORTED, "cannot tune on a capturing stream");
    hipEvent_t a = nullptr, b = nullptr;
    MF_HIP(hipEventCreate(&a), "hipEventCreate");
    hipError_t e = hipEventCreate(&b);
    if (e != hipSuccess) {
        (void)hipEventDestroy(a);
        return hip_fail(e, "hipEventCreate");
    }
    std::lock_guard<std::mutex> plk(p->mu);
    mf_status s = tune_shapes(p, x, y, argmed, reps, st, a, b);
    if (s != MF_OK) {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        return s;
    }
    const int32_t before = p->config;
    int best = -1;
    for (int c = 0; c < kConfigs && s == MF_OK; c++) {
        p->config = c;
        s = plan_execute_locked(p, x, y, argmed, true, stream);   // warm-up (and capture)
        if (s != MF_OK) break;
        e = hipEventRecord(a, st);
        for (int r = 0; r < reps && s == MF_OK && e == hipSuccess; r++)
            s = plan_execute_locked(p, x, y, argmed, true, stream);
        if (s != MF_OK) break;
        if (e == hipSuccess) e = hipEventRecord(b, st);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
        if (e != hipSuccess) {
            s = hip_fail(e, "autotune timing");
            break;
        }
        p->tuned_ms[c] = ms / (float)reps;
        if (best < 0 || p->tuned_ms[c] < p->tuned_ms[best]) best = c;
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    p->config = (s == MF_OK && best >= 0) ? best : before;
    if (env_log() && s == MF_OK)
        fprintf(stderr, "mf: autotune %.3f / %.3f / %.3f ms per execute, config %d\n", p->tuned_ms[0],
                p->tuned_ms[1], p->tuned_ms[2], p->config);
    return s;
}


extern "C" void mf_plan_destroy(mf_plan *p)
{
    plan_free(p);   // waits for the plan's last execution
}

// ------------------------------------------------------------------ plan cache

namespace {
// Plans of the one-call batched entry points, keyed by the offsets and
// windows.  Each caller holds a reference while it uses a plan, so evicting
// an entry never destroys a plan that another call is executing; the last
// reference destroys it (after its last execution has finished).
struct CacheEntry {
    std::vector<int64_t> offsets;
    std::vector<int32_t> ks;
    std::shared_ptr<mf_plan> plan;
};
std::mutex g_cache_mu;
std::vector<CacheEntry> g_cache;   // most recent last
const size_t kCacheMax = 8;

mf_status cached_plan(const int64_t *off, const int32_t *ks, int32_t ns, std::shared_ptr<mf_plan> &out)
{
    if (!off || !ks) return fail(MF_ERR_INVALID_VALUE, "x_offsets and ks must not be null");
    if (ns < 1) return fail(MF_ERR_INVALID_VALUE, "num_signals = %d must be >= 1", ns);
    std::shared_ptr<mf_plan> evicted;   // destroyed after the lock is released
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (size_t i = 0; i < g_cache.size(); i++) {
        CacheEntry &c = g_cache[i];
        if ((int32_t)c.ks.size() == ns && memcmp(c.ks.data(), ks, sizeof(int32_t) * ns) == 0 &&
            memcmp(c.offsets.data(), off, sizeof(int64_t) * (ns + 1)) == 0) {
            out = c.plan;
            return MF_OK;
        }
    }
    mf_plan *p = nullptr;
    mf_status s = mf_plan_create_batched(off, ks, ns, &p);
    if (s != MF_OK) return s;
    std::shared_ptr<mf_plan> sp(p, [](mf_plan *q) { plan_free(q); });
    if (g_cache.size() >= kCacheMax) {
        evicted = std::move(g_cache.front().plan);
        g_cache.erase(g_cache.begin());
    }
    g_cache.push_back(CacheEntry{std::vector<int64_t>(off, off + ns + 1), std::vector<int32_t>(ks, ks + ns), sp});
    out = sp;
    return MF_OK;
}
}  // namespace

// ------------------------------------------------------------------ entry points

extern "C" mf_status mf_median_filter(const float *x, int64_t n, int32_t k, float *y, int32_t *argmed,
                                      void *stream)
{
    return forward_rows(x, 1, n, k, y, argmed, true, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_noalloc(const float *x, int64_t n, int32_t k, float *y, int32_t *argmed,
                                              void *stream)
{
    const hipStream_t st = (hipStream_t)stream;
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    mf_status s = check_signal(n, k);
    if (s != MF_OK) return s;
    const Path p = path_for(k);
    Launch L;
    memset(&L, 0, sizeof L);
    L.x = x;
    L.y = y;
    L.argmed = argmed;
    L.one.n = n;
    L.one.k = k;
    L.rows = 1;
    L.tpr = tiles_for(p, n, k);
    L.nunits = L.tpr;
    const size_t lds = (size_t)lds_bytes_for(p, k);
    int64_t stride = 0, slots = 0;
    if (p == PATH_GLOBAL) {
        // as many workgroup slots as the fixed scratch holds (the launch's
        // workgroups loop over the tiles)
        stride = global_ws_stride(k);
        const int64_t room = (kFixedScratchBytes - kFixedFlagBytes) / stride;
        if (room < 1)
            return fail(MF_ERR_UNSUPPORTED, "k = %d needs %lld bytes of scratch per workgroup, above the fixed %lld",
                        k, (long long)stride, (long long)(kFixedScratchBytes - kFixedFlagBytes));
        slots = std::min<int64_t>(std::min<int64_t>(global_ws_slots(lds), L.nunits), room);
    }
    unsigned char *sc = nullptr;
    MF_HIP(fixed_scratch(st, true, &sc), "fixed scratch set-up");
    MF_HIP(launch_forward(p, true, L, lds, sc + kFixedFlagBytes, stride, slots, (int *)sc, st), "forward launch");
    return MF_OK;
}

extern "C" mf_status mf_median_filter_i32(const int32_t *x, int64_t n, int32_t k, int32_t *y,
                                          int32_t *argmed, void *stream)
{
    return forward_rows(x, 1, n, k, y, argmed, false, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_f64(const double *x, int64_t n, int32_t k, double *y, int32_t *argmed,
                                          void *stream)
{
    return forward64(x, 1, n, k, y, argmed, true, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_i64(const int64_t *x, int64_t n, int32_t k, int64_t *y,
                                          int32_t *argmed, void *stream)
{
    return forward64(x, 1, n, k, y, argmed, false, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_rows(const float *x, int64_t rows, int64_t n, int32_t k, float *y,
                                           int32_t *argmed, void *stream)
{
    return forward_rows(x, rows, n, k, y, argmed, true, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_rows_i32(const int32_t *x, int64_t rows, int64_t n, int32_t k, int32_t *y,
                                               int32_t *argmed, void *stream)
{
    return forward_rows(x, rows, n, k, y, argmed, false, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_rows_f64(const double *x, int64_t rows, int64_t n, int32_t k, double *y,
                                               int32_t *argmed, void *stream)
{
    return forward64(x, rows, n, k, y, argmed, true, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_rows_i64(const int64_t *x, int64_t rows, int64_t n, int32_t k, int64_t *y,
                                               int32_t *argmed, void *stream)
{
    return forward64(x, rows, n, k, y, argmed, false, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_batched(const float *x, const int64_t *x_offsets, const int32_t *ks,
                                              int32_t num_signals, float *y, int32_t *argmed, void *stream)
{
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    std::shared_ptr<mf_plan> p;
    mf_status s = cached_plan(x_offsets, ks, num_signals, p);
    if (s != MF_OK) return s;
    return plan_execute(p.get(), x, y, argmed, true, stream);
}

extern "C" mf_status mf_median_filter_batched_i32(const int32_t *x, const int64_t *x_offsets, const int32_t *ks,
                                                  int32_t num_signals, int32_t *y, int32_t *argmed, void *stream)
{
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    std::shared_ptr<mf_plan> p;
    mf_status s = cached_plan(x_offsets, ks, num_signals, p);
    if (s != MF_OK) return s;
    return plan_execute(p.get(), x, y, argmed, false, stream);
}

extern "C" mf_status mf_median_filter_batched_f64(const double *x, const int64_t *x_offsets, const int32_t *ks,
                                                  int32_t num_signals, double *y, int32_t *argmed, void *stream)
{
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    std::shared_ptr<mf_plan> p;
    mf_status s = cached_plan(x_offsets, ks, num_signals, p);
    if (s != MF_OK) return s;
    return plan_execute64(p.get(), x, y, argmed, true, stream);
}

extern "C" mf_status mf_median_filter_batched_i64(const int64_t *x, const int64_t *x_offsets, const int32_t *ks,
                                                  int32_t num_signals, int64_t *y, int32_t *argmed, void *stream)
{
    if (!x || !y) return fail(MF_ERR_INVALID_VALUE, "x and y must not be null");
    std::shared_ptr<mf_plan> p;
    mf_status s = cached_plan(x_offsets, ks, num_signals, p);
    if (s != MF_OK) return s;
    return plan_execute64(p.get(), x, y, argmed, false, stream);
}

extern "C" mf_status mf_median_filter_backward(const float *grad_y, const int32_t *argmed, int64_t n,
                                               int32_t k, float *grad_x, void *stream)
{
    return backward_rows(grad_y, argmed, 1, n, k, grad_x, false, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_backward_f64(const double *grad_y, const int32_t *argmed, int64_t n,
                                                   int32_t k, double *grad_x, void *stream)
{
    return backward_rows(grad_y, argmed, 1, n, k, grad_x, true, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_backward_rows_f64(const double *grad_y, const int32_t *argmed, int64_t rows,
                                                        int64_t n, int32_t k, double *grad_x, void *stream)
{
    return backward_rows(grad_y, argmed, rows, n, k, grad_x, true, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_backward_rows(const float *grad_y, const int32_t *argmed, int64_t rows,
                                                    int64_t n, int32_t k, float *grad_x, void *stream)
{
    return backward_rows(grad_y, argmed, rows, n, k, grad_x, false, (hipStream_t)stream);
}

extern "C" mf_status mf_median_filter_backward_batched(const float *grad_y, const int32_t *argmed,
                                                       const int64_t *x_offsets, const int32_t *ks,
                                                       int32_t num_signals, float *grad_x, void *stream)
{
    std::shared_ptr<mf_plan> p;
    mf_status s = cached_plan(x_offsets, ks, num_signals, p);
    if (s != MF_OK) return s;
    return mf_plan_execute_backward(p.get(), grad_y, argmed, grad_x, stream);
}

extern "C" int64_t mf_output_length(int64_t n, int32_t k)
{
    if (n < 1 || k < 1 || (k & 1) == 0 || k > n) return -1;
    return n - k + 1;
}

extern "C" const char *mf_status_string(mf_status s)
{
    switch (s) {
    case MF_OK: return "success";
    case MF_ERR_INVALID_VALUE: return "invalid argument";
    case MF_ERR_UNSUPPORTED: return "unsupported size";
    case MF_ERR_NOMEM: return "out of device memory";
    case MF_ERR_HIP: return "HIP runtime error";
    case MF_ERR_INTERNAL: return "inconsistent walk reported by a kernel";
    }
    return "unknown status";
}

extern "C" const char *mf_last_error(void) { return t_last_error.c_str(); }

extern "C" mf_status mf_check_device_error(void *stream)
{
    Device *D = nullptr;
    mf_status s = device_state(&D);
    if (s != MF_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    int h = 0;
    MF_HIP(hipMemcpyAsync(&h, D->d_err, sizeof(int), hipMemcpyDeviceToHost, st), "hipMemcpyAsync(error flag)");
    MF_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
    if (h != 0) {
        MF_HIP(hipMemsetAsync(D->d_err, 0, sizeof(int), st), "hipMemsetAsync(error flag)");
        MF_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        return fail(MF_ERR_INTERNAL, "a kernel reported an inconsistent walk (flag %d)", h);
    }
    // the flag of the entry point without allocation, once it is set up here
    unsigned char *sc = nullptr;
    MF_HIP(fixed_scratch(st, false, &sc), "fixed scratch");
    if (sc) {
        MF_HIP(hipMemcpyAsync(&h, sc, sizeof(int), hipMemcpyDeviceToHost, st), "hipMemcpyAsync(error flag)");
        MF_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
        if (h != 0) {
            MF_HIP(hipMemsetAsync(sc, 0, sizeof(int), st), "hipMemsetAsync(error flag)");
            MF_HIP(hipStreamSynchronize(st), "hipStreamSynchronize");
            return fail(MF_ERR_INTERNAL, "a kernel reported an inconsistent walk (flag %d)", h);
        }
    }
    return MF_OK;
}
