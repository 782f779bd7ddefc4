"""Compile the FP64 CPU oracle (oracle.c) into oracle/liboracle.so.

Test infrastructure: the oracle is the checker for the GPU library and is
loaded only by the tests, the smoke check and the CPU-baseline leg of the
benchmark.  Plain gcc with OpenMP; no architecture-specific flags so the
shared object runs on any x86-64 host.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fcx-limited-range", "-fPIC", "-shared",
           "-Wall", "-Wextra", SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
