"""Throughput of the sorting-based median filter on one MI355X.

One step = one full median filter pass (piecewise sort + pair walks, every
output and argmedian written) over the int32 workload of 2**26 items drawn
uniformly over the full int32 range, window k = 1001, inputs resident in HBM
before the timed region.  Prints one JSON line:

  value         whole-job medians per second over the K timed steps
  roofline      algorithmic bytes of the forward kernel (4 B read per input,
                4 B median + 4 B argmedian written per output) divided by
                its average duration measured with HIP events on the stream
                it runs on, against the 8 TB/s HBM3E peak; `traffic` is the
                HBM bytes per launch from the FETCH_SIZE / WRITE_SIZE
                counters recorded in profiles/ (null when not recorded for
                the current kernel)
  cpu_baseline  the CPU oracle (the paper's method in plain C, one thread) on
                a bounded prefix of the same signal, in medians per second

Flags: --gpus N (only 1 is supported: the method shards trivially, but this
build runs on one GPU), --steps K, --warmup W, --extras (also time the
duplicates-heavy input, the random-walk window sweep, the row batch with
backward, the ragged batch, and the paper's generator families over h;
minutes of host-side data generation).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "int32_full_64m"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_int32_full_64m_k1001.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=30)
    ap.add_argument("--extras", action="store_true")
    ap.add_argument("--only", metavar="WORKLOAD:K", default=None,
                    help="time only the forward of one float32 or int32 workload of workloads.py at window K "
                         "(for profiling a kernel other than the headline one), e.g. random_walk_f32_16m:30001")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first run a plain 256 MiB device copy (known bytes) for counter calibration")
    ap.add_argument("--phase-probe", action="store_true",
                    help="time the headline kernel stopped after each tile phase (needs the phase-probe "
                         "library: python -m paper_1406_1717_amd.build --phase-probe)")
    ap.add_argument("--phase-probe-global", metavar="K", type=int, default=None,
                    help="the same for the workspace path (4095 < K <= 32767) on the float32 random walk "
                         "random_walk_f32_16m")
    return ap.parse_args()


def timed_steps(fn, steps, warmup, torch):
    """Run fn warmup times, then time exactly `steps` calls.  Returns
    (total seconds from synchronize to synchronize, per-step event times)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for a, b in evs:
        a.record(st)
        fn()
        b.record(st)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [a.elapsed_time(b) * 1e-3 for a, b in evs]
    return t1 - t0, per


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x, k, budget_s=8.0):
    """The oracle (the paper's method in plain C) on the host: first on one
    thread over growing prefixes of x until about budget_s of work, then on
    every core (one thread per output range, each range sorting its own
    blocks with a k-1 halo) over the largest prefix that fits the same
    budget scaled by the core count."""
    import oracle
    chunk = 1 << 22
    m1, out1, t1 = 0, 0, 0.0
    while m1 < len(x) and t1 < budget_s:
        m1 = min(len(x), m1 + chunk)
        t = time.perf_counter()
        _, am = oracle.sortmedian(x[:m1], k)
        t1 = time.perf_counter() - t
        out1 = len(am)
    single = out1 / t1
    cores = os.cpu_count() or 1
    m = min(len(x), int(single * budget_s * cores) + k - 1)
    t = time.perf_counter()
    _, am = oracle.sortmedian_parallel(x[:m], k, threads=cores)
    tp = time.perf_counter() - t
    return {"value": len(am) / tp, "unit": "medians/s", "cores": cores, "kind": "oracle",
            "sample": "first %d items of the same signal (%d medians, %.1f s on %d threads, one output "
                      "range each); single thread: %.3g medians/s on the first %d items"
                      % (m, len(am), tp, cores, single, m1),
            "single_thread": single, "cpu_model": cpu_model()}


def copy_ceiling(torch, nbytes=1 << 30, reps=10):
    """GB/s of a plain device-to-device copy (read + write bytes over the
    kernel time): the practical HBM ceiling beside the 8 TB/s peak."""
    src = torch.empty(nbytes // 4, dtype=torch.int32, device="cuda:0")
    dst = torch.empty_like(src)
    src.fill_(1)
    dst.copy_(src)
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(st)
        dst.copy_(src)
        b.record(st)
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) * 1e-3)
    del src, dst
    return 2.0 * nbytes / float(np.median(times)) / 1e9


def flushed_ms(fn, torch, reps=5, flush_bytes=1 << 30):
    """Median HIP-event time of fn with the 256 MB Infinity Cache flushed
    before each call (a 1 GiB device write outside the timed events)."""
    scratch = torch.empty(flush_bytes // 4, dtype=torch.int32, device="cuda:0")
    st = torch.cuda.current_stream()
    fn()
    times = []
    for _ in range(reps):
        scratch.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        fn()
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    del scratch
    return float(np.median(times))


def sampled_windows_ok(x, k, y, am, samples=2000, seed=0):
    h = (k - 1) // 2
    outs = np.random.default_rng(seed).integers(0, len(am), samples)
    for o in outs:
        a = int(am[o])
        if not (o <= a <= o + k - 1) or y[o] != x[a]:
            return False
        w = x[o:o + k]
        idx = np.arange(o, o + k)
        below = np.count_nonzero((w < x[a]) | ((w == x[a]) & (idx < a)))
        if below != h:
            return False
    return True


def load_traffic():
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        return t
    except (OSError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported "
              "(the median filter would shard by output range, each GPU reading a k-1 halo)" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_1406_1717_amd as mf
    from paper_1406_1717_amd import lib, workloads

    if args.only:
        print(json.dumps(only(torch, lib, workloads, args)), flush=True)
        return
    if args.phase_probe_global is not None:
        print(json.dumps(phase_probe_global(torch, workloads, args)), flush=True)
        return
    dev = torch.device("cuda:0")
    w = workloads.workload(WORKLOAD)
    x_host, k = w["x"], w["k"]
    n = len(x_host)
    nout = n - k + 1
    x = torch.from_numpy(x_host).to(dev)
    y = torch.empty(nout, dtype=torch.int32, device=dev)
    am = torch.empty(nout, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    if args.phase_probe:
        print(json.dumps(phase_probe(torch, x, n, k, y, am, args)), flush=True)
        return

    if args.copy_probe:
        src = torch.empty(64 << 20, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        lib.mf_median_filter_i32(x, n, k, y, am)

    total, per = timed_steps(step, args.steps, args.warmup, torch)
    lib.mf_check_device_error()
    ms_per_step = total / args.steps * 1e3
    value = nout * args.steps / total
    kern_s = float(np.mean(per))
    alg_bytes = 4.0 * n + 8.0 * nout
    achieved = alg_bytes / kern_s / 1e9

    # spot check of the timed output: on sampled windows the argmedian lies
    # in the window, y is its value, and exactly h window items order below
    # it by (value, index)
    if not sampled_windows_ok(x_host, k, y.cpu().numpy(), am.cpu().numpy()):
        print("bench.py: sampled windows fail the median property", file=sys.stderr)
        sys.exit(3)

    traffic = None
    t = load_traffic()
    if t and t.get("kernel_source_sha") == kernel_source_sha():
        traffic = t.get("hbm_bytes_per_launch")

    line = {
        "metric": "median outputs/s",
        "value": value,
        "unit": "outputs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": n, "k": k, "values": "int32 uniform over the full range",
                   "seed": workloads.SEEDS[WORKLOAD], "outputs_per_step": nout},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_tile_lds<512,int32>", "kernel_ms": kern_s * 1e3,
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "copy_ceiling_gbs": copy_ceiling(torch)},
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(x_host, k)
    if args.extras:
        line["extras"] = extras(torch, mf, lib, workloads, args)
    print(json.dumps(line), flush=True)


# (stopping point, phase ending there): stop 6 (after the in-bucket rank)
# is not timed, since a kernel that stops there has no use for the ranks
# and loses them, and stop 11 follows stop 10 with nothing between (the
# column pass is one phase); 0 runs whole tiles
PHASES = [(1, "load, zero counters"), (2, "key range + presorted check"), (3, "count"), (4, "scan"),
          (5, "scatter"), (7, "rank + place"), (8, "per-block counts + scan + table zero"),
          (9, "pair positions + histogram"), (10, "column pass"), (12, "row prefix"), (13, "walk"),
          (0, "output")]


def phase_probe(torch, x, n, k, y, am, args):
    """The headline kernel built with a stop after each tile phase: the
    median launch time of every stopping point (HIP events), and each
    phase's share as the difference of consecutive points."""
    import ctypes
    path = os.path.join(ROOT, "paper_1406_1717_amd", "libmf_phase_probe.so")
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.mf_phase_probe_i32.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_int, P]
    L.mf_phase_probe_i32.restype = ctypes.c_int
    st = torch.cuda.current_stream()
    stops = [st_ for st_, _ in PHASES]
    ms = {}
    for stop in stops:
        def run():
            rc = L.mf_phase_probe_i32(P(x.data_ptr()), n, k, P(y.data_ptr()), P(am.data_ptr()), stop,
                                      P(st.cuda_stream))
            if rc != 0:
                raise RuntimeError("phase probe launch failed (%d)" % rc)
        _, per = timed_steps(run, max(args.steps, 10), args.warmup, torch)
        ms[stop] = float(np.median(per)) * 1e3
    cum = [ms[s] for s in stops]
    phases = []
    prev = 0.0
    for (stop, name), c in zip(PHASES, cum):
        phases.append({"stop": stop, "phase": name, "cumulative_ms": c, "ms": c - prev})
        prev = c
    return {"phase_probe": WORKLOAD, "n": n, "k": k, "phases": phases}


PHASES_GLOBAL = [(21, "key range"), (22, "arrival numbers (bucket counts)"), (23, "bucket starts"),
                 (24, "scatter"), (25, "rank in bucket, merged order, position maps"),
                 (26, "table zero + histogram"), (27, "column pass"),
                 (28, "row pass + chunk starting columns"), (29, "copy of M into LDS"), (30, "walk"),
                 (0, "output")]


def phase_probe_global(torch, workloads, args):
    """The workspace-path kernel (one pair per tile, k > 4095) built with a
    stop after each phase, on the float32 random walk of 2^24 items at
    window args.phase_probe_global: median launch time per stopping point
    and each phase's share."""
    import ctypes
    k = args.phase_probe_global
    w = workloads.workload("random_walk_f32_16m")
    xh = w["x"]
    n = len(xh)
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xh).to(dev)
    y = torch.empty(n - k + 1, dtype=x.dtype, device=dev)
    am = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    path = os.path.join(ROOT, "paper_1406_1717_amd", "libmf_phase_probe.so")
    L = ctypes.CDLL(path)
    P = ctypes.c_void_p
    L.mf_phase_probe_global_f32.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P, ctypes.c_int, P]
    L.mf_phase_probe_global_f32.restype = ctypes.c_int
    st = torch.cuda.current_stream()
    ms = {}
    for stop, _ in PHASES_GLOBAL:
        def run():
            rc = L.mf_phase_probe_global_f32(P(x.data_ptr()), n, k, P(y.data_ptr()), P(am.data_ptr()), stop,
                                             P(st.cuda_stream))
            if rc != 0:
                raise RuntimeError("phase probe launch failed (%d)" % rc)
        _, per = timed_steps(run, max(args.steps, 10), min(args.warmup, 5), torch)
        ms[stop] = float(np.median(per)) * 1e3
    phases = []
    prev = 0.0
    for stop, name in PHASES_GLOBAL:
        phases.append({"stop": stop, "phase": name, "cumulative_ms": ms[stop], "ms": ms[stop] - prev})
        prev = ms[stop]
    return {"phase_probe": "random_walk_f32_16m", "n": n, "k": k, "phases": phases}


def kernel_source_sha():
    """Hash of the forward kernels' device code (the tile header, and the
    kernel file up to its backward section) with comments and blank space
    removed: the HBM counters stay valid across comment edits and changes
    to the backward or the host side."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ("mf_tile.h", "mf_kernels.hip"):
        with open(os.path.join(ROOT, "paper_1406_1717_amd", "csrc", f)) as fh:
            text = fh.read()
        a = text.find("// " + "-" * 66 + " backward\n")
        if a >= 0:
            text = text[:a]
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        text = re.sub(r"//[^\n]*", "", text)
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def only(torch, lib, workloads, args):
    """The forward of one named workload at one window: HIP-event time per
    launch over args.steps launches after args.warmup."""
    name, kk = args.only.split(":")
    k = int(kk)
    w = workloads.workload(name)
    xh = w["x"]
    if xh.ndim != 1 or xh.dtype not in (np.float32, np.int32):
        raise SystemExit("bench.py --only: %s is not a one-dimensional float32 or int32 workload" % name)
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(xh).to(dev)
    n = len(xh)
    y = torch.empty(n - k + 1, dtype=xt.dtype, device=dev)
    a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    f = lib.mf_median_filter if xh.dtype == np.float32 else lib.mf_median_filter_i32
    total, per = timed_steps(lambda: f(xt, n, k, y, a), args.steps, args.warmup, torch)
    ms = float(np.median(per)) * 1e3
    return {"only": name, "n": n, "k": k, "steps": args.steps, "ms_median": ms,
            "outputs_per_s": (n - k + 1) / (ms * 1e-3),
            "hbm_frac": (4.0 * n + 8.0 * (n - k + 1)) / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def extras(torch, mf, lib, workloads, args):
    """Secondary measurements (not part of the headline value)."""
    dev = torch.device("cuda:0")
    out = {}
    # duplicates-heavy int32 (values 0..255)
    w = workloads.workload("int32_bytes_64m")
    xb = torch.from_numpy(w["x"]).to(dev)
    n, k = len(w["x"]), w["k"]
    y = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    total, per = timed_steps(lambda: lib.mf_median_filter_i32(xb, n, k, y, a), args.steps, args.warmup, torch)
    out["int32_bytes_64m"] = {"outputs_per_s": (n - k + 1) * args.steps / total,
                              "hbm_frac": (4.0 * n + 8.0 * (n - k + 1)) / np.mean(per) / 1e9 / HBM_PEAK_GBS}
    del xb, y, a
    # the headline kernel with the 256 MB Infinity Cache flushed before each
    # launch (a 1 GiB write outside the timed events): median of 10
    w = workloads.workload("int32_full_64m")
    xf = torch.from_numpy(w["x"]).to(dev)
    n, k = len(w["x"]), w["k"]
    y = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    scratch = torch.empty(1 << 28, dtype=torch.int32, device=dev)
    st = torch.cuda.current_stream()
    lib.mf_median_filter_i32(xf, n, k, y, a)
    times = []
    for _ in range(10):
        scratch.fill_(1)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(st)
        lib.mf_median_filter_i32(xf, n, k, y, a)
        e1.record(st)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) * 1e-3)
    med = float(np.median(times))
    out["int32_full_64m_flushed"] = {"kernel_ms_median": med * 1e3, "outputs_per_s": (n - k + 1) / med,
                                     "hbm_frac": (4.0 * n + 8.0 * (n - k + 1)) / med / 1e9 / HBM_PEAK_GBS}
    del xf, y, a, scratch
    # random walk, k sweep
    for name in ("random_walk_f32_16m", "sorted_walk_f32_16m"):
        w = workloads.workload(name)
        xr = torch.from_numpy(w["x"]).to(dev)
        n = len(w["x"])
        res = {}
        for k in w["ks"]:
            y = torch.empty(n - k + 1, dtype=torch.float32, device=dev)
            a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
            total, per = timed_steps(lambda: lib.mf_median_filter(xr, n, k, y, a), 5, 1, torch)
            # the whole working set (about 201 MB) fits the 256 MB Infinity
            # Cache: also timed with the cache flushed before each launch
            fl = flushed_ms(lambda: lib.mf_median_filter(xr, n, k, y, a), torch)
            res[str(k)] = {"outputs_per_s": (n - k + 1) * 5 / total,
                           "hbm_frac": (4.0 * n + 8.0 * (n - k + 1)) / np.mean(per) / 1e9 / HBM_PEAK_GBS,
                           "flushed_ms": fl, "flushed_outputs_per_s": (n - k + 1) / (fl * 1e-3),
                           "flushed_hbm_frac": (4.0 * n + 8.0 * (n - k + 1)) / (fl * 1e-3) / 1e9 / HBM_PEAK_GBS}
        out[name] = res
        del xr
    # 64-bit signals (rank pre-pass, int32 tiles on the ranks, gather)
    w = workloads.workload("int64_full_64m")
    x64 = torch.from_numpy(w["x"]).to(dev)
    n, k = len(w["x"]), w["k"]
    y = torch.empty(n - k + 1, dtype=torch.int64, device=dev)
    a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
    total, per = timed_steps(lambda: lib.mf_median_filter_i64(x64, n, k, y, a), args.steps, args.warmup, torch)
    out["int64_full_64m"] = {"k": k, "outputs_per_s": (n - k + 1) * args.steps / total,
                             "hbm_frac": (8.0 * n + 12.0 * (n - k + 1)) / np.mean(per) / 1e9 / HBM_PEAK_GBS,
                             "checked": sampled_windows_ok(w["x"], k, y.cpu().numpy(), a.cpu().numpy(),
                                                           samples=300)}
    del x64, y, a
    w = workloads.workload("random_walk_f64_16m")
    xr = torch.from_numpy(w["x"]).to(dev)
    n = len(w["x"])
    res = {}
    for k in w["ks"]:
        y = torch.empty(n - k + 1, dtype=torch.float64, device=dev)
        a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
        total, per = timed_steps(lambda: lib.mf_median_filter_f64(xr, n, k, y, a), 5, 1, torch)
        res[str(k)] = {"outputs_per_s": (n - k + 1) * 5 / total,
                       "hbm_frac": (8.0 * n + 12.0 * (n - k + 1)) / np.mean(per) / 1e9 / HBM_PEAK_GBS}
    out["random_walk_f64_16m"] = res
    del xr
    # differentiable rows (the seeded distinct-valued rows and upstream
    # gradient): forward vs forward + backward, at the C-ABI level and
    # through the autograd Function
    w = workloads.workload("distinct_normal_256")
    rows, n, k = w["x"].shape[0], w["x"].shape[1], w["k"]
    xs = torch.from_numpy(w["x"]).to(dev)
    g = torch.from_numpy(w["grad"]).to(dev)
    ys = torch.empty(rows, n - k + 1, device=dev)
    ams = torch.empty(rows, n - k + 1, dtype=torch.int32, device=dev)
    gx = torch.empty(rows, n, device=dev)
    tf, _ = timed_steps(lambda: lib.mf_median_filter_rows(xs, rows, n, k, ys, ams), 10, 2, torch)

    def fb():
        lib.mf_median_filter_rows(xs, rows, n, k, ys, ams)
        lib.mf_median_filter_backward_rows(g, ams, rows, n, k, gx)
    tfb, _ = timed_steps(fb, 10, 2, torch)
    tb, _ = timed_steps(lambda: lib.mf_median_filter_backward_rows(g, ams, rows, n, k, gx), 10, 2, torch)
    xa = xs.clone().requires_grad_(True)

    def af():
        with torch.no_grad():
            mf.MedianFilterFn.apply(xa, k)

    def afb():
        xa.grad = None
        yy, _ = mf.MedianFilterFn.apply(xa, k)
        yy.backward(g)
    taf, _ = timed_steps(af, 10, 2, torch)
    tafb, _ = timed_steps(afb, 10, 2, torch)
    out["distinct_normal_256"] = {"fwd_ms": tf / 10 * 1e3, "fwd_bwd_ms": tfb / 10 * 1e3,
                                  "bwd_ms": tb / 10 * 1e3, "ratio": tfb / tf,
                                  "autograd_fwd_ms": taf / 10 * 1e3, "autograd_fwd_bwd_ms": tafb / 10 * 1e3,
                                  "autograd_ratio": tafb / taf}
    del xs, g, ys, ams, gx, xa
    # ragged batch: one plan (graph) launch vs one plain launch per signal
    x, off, ks = workloads.ragged_impulse(10_000, workloads.SEEDS["ragged_impulse_10k"])
    xt = torch.from_numpy(x).to(dev)
    yo = mf.output_offsets(off, ks)
    y = torch.empty(int(yo[-1]), device=dev)
    am = torch.empty(int(yo[-1]), dtype=torch.int32, device=dev)
    plan = mf.Plan(off, ks)
    t0 = time.perf_counter()
    tune = plan.autotune(xt, y, am, reps=2)
    tune_s = time.perf_counter() - t0
    tb, _ = timed_steps(lambda: plan.execute(xt, y, am), 3, 1, torch)
    n_sig = len(ks)
    xs_v = [xt[off[s]:off[s + 1]] for s in range(n_sig)]
    ys_v = [y[yo[s]:yo[s + 1]] for s in range(n_sig)]
    as_v = [am[yo[s]:yo[s + 1]] for s in range(n_sig)]

    def per_signal():
        for s in range(n_sig):
            lib.mf_median_filter(xs_v[s], off[s + 1] - off[s], ks[s], ys_v[s], as_v[s])
    tp, _ = timed_steps(per_signal, 2, 1, torch)
    out["ragged_impulse_10k"] = {"items": int(off[-1]), "outputs": int(yo[-1]),
                                 "batched_ms": tb / 3 * 1e3, "per_signal_ms": tp / 2 * 1e3,
                                 "speedup": (tp / 2) / (tb / 3),
                                 "batched_outputs_per_s": int(yo[-1]) / (tb / 3),
                                 "launch_config": tune["config"], "tuned_ms_per_config": tune["tuned_ms"],
                                 "autotune_s": tune_s}
    plan.close()
    out["paper_generators"] = paper_sweep(torch, lib, workloads)
    out["paper_generators_64"] = paper_sweep(torch, lib, workloads, bits=64)
    out["paper_generators_bh1e6"] = paper_sweep(torch, lib, workloads, bh=10**6)
    out["paper_generators_64_bh1e6"] = paper_sweep(torch, lib, workloads, bh=10**6, bits=64)
    return out


def paper_sweep(torch, lib, workloads, bh=10**7, hs=(1, 10, 100, 1000, 10000), bits=32):
    """The paper's generator families (Section 7.3) with b*h fixed and the
    half-window h varied (n = (2h+1) b, k = 2h+1), int32 or int64: median
    outputs/s of the forward, each output spot-checked by the median
    property."""
    dev = torch.device("cuda:0")
    dt = torch.int32 if bits == 32 else torch.int64
    fn = lib.mf_median_filter_i32 if bits == 32 else lib.mf_median_filter_i64
    res = {}
    for fam in ("asc", "desc", "r-asc", "r-desc", "r-large", "r-small", "r-block"):
        row = {}
        for h in hs:
            b = bh // h
            k = 2 * h + 1
            n = b * k
            x_host = workloads.paper_family(fam, n, 700 + h, bits=bits)
            x = torch.from_numpy(x_host).to(dev)
            y = torch.empty(n - k + 1, dtype=dt, device=dev)
            a = torch.empty(n - k + 1, dtype=torch.int32, device=dev)
            total, _ = timed_steps(lambda: fn(x, n, k, y, a), 3, 1, torch)
            ok = sampled_windows_ok(x_host, k, y.cpu().numpy(), a.cpu().numpy(), samples=200)
            row[str(h)] = {"n": n, "k": k, "outputs_per_s": (n - k + 1) * 3 / total, "checked": ok}
            del x, y, a
        res[fam] = row
    return res


if __name__ == "__main__":
    main()
