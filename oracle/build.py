"""Compile the FP64 oracle (plain C, gcc, OpenMP) into oracle/liboracle.so.

Test infrastructure: the library it builds is loaded only by the tests, the
smoke check and the benchmark's CPU-baseline leg.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "stencil_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, native: bool = False, out: str | None = None) -> str:
    """Compile the oracle.  The in-tree library (the tests' reference) is
    built for any x86-64 host; native=True builds -O3 -march=native for the
    host that runs it (the CPU-baseline timing), into `out`.  ISO C mode
    keeps floating-point contraction off, so both give the same FP64 bits."""
    dest = out or LIB
    tmp = dest + f".tmp{os.getpid()}"
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", "-std=c11", *opt, "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, dest)
    return dest


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
