"""Build libstencil.so in-tree with hipcc for gfx950.

Both translation units go through hipcc.  Packed-FP32 instructions are
disabled for device code (-packed-fp32-ops): hipcc would otherwise emit
v_pk_fma_f32 and friends from ordinary float code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libstencil.so")
OBJDIR = os.path.join(HERE, "_build")

ARCH = os.environ.get("STENCIL_OFFLOAD_ARCH", "gfx950")
COMMON = ["-std=c++17", "-O3", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]
# Per-source flags.  The depth-2 wave kernel waits mostly on memory; the
# machine scheduler's strategy that keeps memory instructions together in
# clauses issues its loads earlier (2% per launch at 512^3, the same bits).
SOURCE_FLAGS = {"zmarch_tb.hip": ["-mllvm", "-amdgpu-sched-strategy=max-memory-clause"]}
SOURCES = ["zmarch_tb.hip", "zmarch_tb_heat.hip", "zmarch_tb_damp.hip", "heat2d_tb.hip", "program.hip", "zmarch_f32.hip", "zmarch_adj.hip", "zmarch_bf16.hip", "zmarch_f16.hip",
           "kernels.hip", "checks.hip", "runtime.cpp", "program_rtc.cpp"]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.splitext(src)[0] + ".o")
    cmd = ["hipcc", *COMMON, *SOURCE_FLAGS.get(src, []), "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    jobs = max(1, min(len(SOURCES), int(os.environ.get("MAX_JOBS", os.cpu_count() or 4))))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + f".tmp{os.getpid()}"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs, "-lhiprtc"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
