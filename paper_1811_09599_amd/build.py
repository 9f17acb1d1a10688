"""Build libqflex.so in-tree with hipcc for gfx950.

    python -m paper_1811_09599_amd.build            # or __graft_entry__.build()
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqflex.so")

HIP_SOURCES = ["grid_kernels.hip", "permute.hip", "gemm.hip", "gemm_split.hip", "reduce.hip",
               "fused.hip",
               "sample.hip", "noalloc.hip"]
HOST_SOURCES = ["model.cpp", "plan.cpp", "fused_plan.cpp", "exec.cpp", "exec_grad.cpp", "api.cpp", "tune_cache.cpp"]
ARCH = "gfx950"

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          "-I" + os.path.join(ROOT, "include")]
# Packed FP32 instructions are kept out of device code: some of their forms have given
# wrong results on this hardware without any error.
DEVICE = ["-x", "hip", "--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("command failed (%d): %s\n%s" % (r.returncode, " ".join(cmd), r.stdout))
    return r.stdout


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    cc = hipcc()
    jobs = []
    for s in HIP_SOURCES:
        jobs.append([cc] + COMMON + DEVICE + ["-c", os.path.join(CSRC, s), "-o",
                                              os.path.join(OUT_DIR, s + ".o")])
    for s in HOST_SOURCES:  # host code only; the target keeps hipcc off its default arch
        jobs.append([cc] + COMMON + ["--offload-arch=" + ARCH, "-c", os.path.join(CSRC, s),
                                     "-o", os.path.join(OUT_DIR, s + ".o")])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(OUT_DIR, s + ".o") for s in HIP_SOURCES + HOST_SOURCES]
    tmp = LIB + ".tmp"
    _run([cc, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
