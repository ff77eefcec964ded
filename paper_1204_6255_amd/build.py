"""Builds the native parts of the package in-tree.

libdi.so        HIP kernels + C ABI (hipcc, gfx950 only)
graphgen/libdigen.so   seeded input generator (g++)
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")

HIP_SOURCES = ["di_kernels.hip", "di_graph.cpp", "di_solve.cpp", "di_batch.hip", "di_batch.cpp", "di_serve.cpp",
               "di_noalloc.hip", "di_window.hip"]
ARCH = "gfx950"

# -packed-fp32-ops: keep the compiler from forming packed FP32 arithmetic.
# -munsafe-fp-atomics: float/double atomicAdd become hardware atomics (the
# graph buffers come from hipMalloc, which is coarse-grained memory).
HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++20", "-fPIC", "-shared",
    "-munsafe-fp-atomics", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    raise RuntimeError("hipcc not found")


def build_di(verbose: bool = False) -> str:
    """Compiles each source to an object in _build/ (in parallel) and links
    libdi.so in-tree."""
    from concurrent.futures import ThreadPoolExecutor

    out = os.path.join(HERE, "libdi.so")
    bdir = os.path.join(ROOT, "_build", "di")
    os.makedirs(bdir, exist_ok=True)
    common = [f for f in HIPCC_FLAGS if f not in ("-shared",)]

    def compile_one(name):
        obj = os.path.join(bdir, name + ".o")
        cmd = [hipcc(), *common, f"-I{INCLUDE}", f"-I{CSRC}", "-c", "-x", "hip",
               os.path.join(CSRC, name), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    jobs = max(1, min(len(HIP_SOURCES), int(os.environ.get("MAX_JOBS", "8"))))
    with ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(compile_one, HIP_SOURCES))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", out + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


def build_all(verbose: bool = False):
    from paper_1204_6255_amd.graphgen import build as gb
    return [gb.build(verbose), build_di(verbose)]


if __name__ == "__main__":
    sys.path.insert(0, ROOT)
    for p in build_all(verbose="-v" in sys.argv):
        print(p)
