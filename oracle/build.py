"""Compile the CPU oracle (plain C, gcc) into a shared library.

Test infrastructure only: the library built here is loaded by the test
suite, the smoke check and the CPU-baseline leg of the benchmark, never by
the product path.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "median_oracle.c")
LIB = os.path.join(HERE, "libmedian_oracle.so")


def build(verbose: bool = False) -> str:
    """Compile median_oracle.c with gcc -O2; returns the library path."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
