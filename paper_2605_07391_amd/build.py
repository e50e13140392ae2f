"""Build libmerbit.so in-tree with hipcc for gfx950.

Run as ``python -m paper_2605_07391_amd.build`` or call ``build()``.  The
library lands next to this file; the Python binding loads it from there.
"""
from __future__ import annotations

import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmerbit.so")
SOURCES = ["merbit_api.hip", "merbit_api_iter.hip", "merbit_api_batched.hip",
           "merbit_api_adjoint.hip", "merbit_api_tune.hip", "merbit_plan.hip", "merbit_spmv.hip",
           "merbit_pagerank.hip", "merbit_hot.hip", "merbit_spmv_wave.hip", "merbit_batched.hip",
           "merbit_adjoint.hip", "merbit_bicgstab.hip", "merbit_stripes.hip",
           "merbit_api_stripes.hip", "merbit_api_noalloc.hip", "merbit_sort.hip"]
ARCH = os.environ.get("MERBIT_OFFLOAD_ARCH", "gfx950")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-Wno-unused-result",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    f"-I{os.path.join(ROOT, 'include')}",
]

# Per-file flags.  The wave kernel reads a tile-queue atomic's result one tile
# after issuing it; the atomic optimizer would turn the single-lane atomic into
# a wave reduction that reads the result (and waits for it) at once.
FILE_FLAGS = {
    "merbit_spmv_wave.hip": ["-mllvm", "-amdgpu-atomic-optimizer-strategy=None"],
}


def build(verbose: bool = False, jobs: int = 4) -> str:
    """Compile every source to an object file (in parallel) and link the
    shared library.  Always recompiles."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    t0 = time.time()
    pending = list(SOURCES)
    while pending or procs:
        while pending and len(procs) < jobs:
            src = pending.pop(0)
            obj = os.path.join(objdir, src.replace(".hip", ".o"))
            objs.append(obj)
            cmd = [HIPCC, *FLAGS, *FILE_FLAGS.get(src, []), "-c", os.path.join(CSRC, src),
                   "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE,
                                                stderr=subprocess.STDOUT, text=True)))
        src, pr = procs.pop(0)
        out, _ = pr.communicate()
        if pr.returncode != 0:
            for _, other in procs:
                other.kill()
            raise RuntimeError(f"hipcc failed on {src}:\n{out}")
        if verbose and out.strip():
            print(out, flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s", flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
