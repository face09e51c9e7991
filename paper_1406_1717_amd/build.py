"""Build libmf.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree."""
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libmf.so")
BUILD_DIR = os.path.join(ROOT, "_build")

SOURCES = ["mf_kernels.hip", "mf_api.cpp"]
HEADERS = ["mf_tile.h", "mf_launch.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Packed fp32 instructions stay off: they are not needed here and some of
# their forms are not trusted on this hardware.
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-function", "-I" + os.path.join(ROOT, "include")]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src in SOURCES:
        obj = os.path.join(BUILD_DIR, src + ".o")
        cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            sys.stderr.write(r.stdout + r.stderr)
            raise RuntimeError("hipcc failed on " + src)
        objs.append(obj)
    tmp = OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


PROBE_OUT = os.path.join(PKG, "libmf_phase_probe.so")


def build_phase_probe(verbose: bool = False) -> str:
    """A measurement-only library: the int32 512-thread tile kernel
    instantiated with a stop after each tile phase (mf_phase_probe_i32), for
    timing and counting the phases one by one.  The product never loads it."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    obj = os.path.join(BUILD_DIR, "mf_kernels_probe.o")
    cmd = [HIPCC] + FLAGS + ["-DMF_PHASE_PROBE", "-c", os.path.join(CSRC, "mf_kernels.hip"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp = PROBE_OUT + ".tmp%d" % os.getpid()
    subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp, obj], check=True)
    os.replace(tmp, PROBE_OUT)
    return PROBE_OUT


if __name__ == "__main__":
    if len(sys.argv) > 1 and sys.argv[1] == "--phase-probe":
        build_phase_probe(verbose=True)
    else:
        build(verbose=True)
