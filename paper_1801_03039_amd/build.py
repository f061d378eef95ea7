"""Build libebic.so (HIP, gfx950) in-tree.

    python -m paper_1801_03039_amd.build

Compiles every source under ``csrc/`` with hipcc for gfx950 and links them
into ``paper_1801_03039_amd/libebic.so``.  Packed FP32 instructions are
disabled (``-packed-fp32-ops``) and floating-point contraction is off; no
fast-math, since NaN ordering is part of the evaluator's definition.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libebic.so")
BUILD_DIR = os.path.join(HERE, "_build")

ARCH = "gfx950"
SOURCES = ["ebic_kernels.hip", "ebic_index.hip", "ebic_batch_kernels.hip", "ebic_runtime.cpp", "ebic_evolve.cpp", "ebic_batch.cpp",
           "ebic_mlp_kernels.hip", "ebic_mlp.cpp", "ebic_surrogate.cpp", "ebic_scores.hip",
           "ebic_checkpoint.cpp", "ebic_noalloc.hip", "ebic_steps.hip",
           "ebic_mlp_fused.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-fast-math", "-Wall",
          "-I", INCLUDE, "-I", CSRC]
HIP_ONLY = ["-x", "hip", f"--offload-arch={ARCH}",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compile every source and link the library.  With ``incremental``, an
    object newer than its source and every header is reused."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    cc = hipcc()
    headers = [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".h")]
    headers += [os.path.join(INCLUDE, f) for f in os.listdir(INCLUDE) if f.endswith(".h")]
    newest_header = max(os.path.getmtime(h) for h in headers)
    cmds, objs = [], []
    for src in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD_DIR, src + ".o")
        objs.append(obj)
        if (incremental and os.path.exists(obj) and
                os.path.getmtime(obj) > max(os.path.getmtime(path), newest_header)):
            continue
        cmds.append([cc, "-c"] + (HIP_ONLY if src.endswith(".hip") else []) + [path, "-o", obj] +
                    COMMON)
    # sources compile in parallel (a few hipcc processes; the kernel files
    # dominate the build time)
    jobs = max(1, min(len(cmds) or 1, int(os.environ.get("MAX_JOBS", "4")), os.cpu_count() or 1))
    with concurrent.futures.ThreadPoolExecutor(jobs) as pool:
        procs = []
        for cmd in cmds:
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append(pool.submit(subprocess.run, cmd, check=True))
        for f in procs:
            f.result()
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
