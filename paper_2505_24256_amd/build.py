"""Build the gfx950 shared library ``libzippel_hip.so`` in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libzippel_hip.so")
SOURCES = ["kernels.hip", "kernels_ilp.hip", "balanced.hip", "batch.hip", "microbench.hip", "zippel.cpp", "balanced.cpp", "batch.cpp", "serve.cpp", "noalloc.cpp", "multiprime.hip", "multiprime.cpp", "multi.cpp", "adaptive.cpp"]
ARCH = os.environ.get("ZR_OFFLOAD_ARCH", "gfx950")
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         # keep hipcc from forming packed fp32 instructions
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-Wno-unused-value", "-Wno-unused-command-line-argument"]


# Sources whose kernels are latency-bound chains at one wave per SIMD (the
# matrix-core solve, the product-tree convolution): LLVM's latency-aware
# scheduling strategy measured faster there.  Elsewhere it raised register use
# (the integer-VALU solve lost occupancy) or measured slower (batch.hip), and it
# crashes the compiler on balanced.hip, so every other source keeps the default.
ILP_SCHED_SOURCES = ("kernels_ilp.hip",)


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        extra = ["-mllvm", "-amdgpu-sched-strategy=iterative-ilp"] if src in ILP_SCHED_SOURCES else []
        cmd = ["hipcc", *FLAGS, *extra, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
