"""Build libdwtfrag.so (the HIP kernels and the C ABI) for gfx950, in-tree.

    python -m paper_1803_04880_amd.build        (from the repository root)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdwtfrag.so")
SOURCES = ["api.hip", "batch.hip", "fwd.hip", "inv.hip", "ctr.hip", "learned.hip", "se8.hip",
           "refstream.hip"]
ARCH = os.environ.get("DWTFRAG_ARCH", "gfx950")
# Per-source compiler options: the SHA-2 compressions of se8.hip are fully
# unrolled loops (their message schedule lives in registers only when every
# index is a constant), larger than the unroller's default size limit; the
# matrix-core products of learned.hip write ordinary VGPRs, so that their
# results need no copy out of the accumulator registers and the four
# products of a batch can be in flight together.
EXTRA = {"se8.hip": ["-mllvm", "-pragma-unroll-threshold=500000"],
         "learned.hip": ["-mllvm", "-amdgpu-mfma-vgpr-form"]}


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def flags() -> list[str]:
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def build(verbose: bool = False) -> str:
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:  # independent translation units: compile in parallel
        obj = os.path.join(objdir, src.replace(".hip", ".o"))
        cmd = [hipcc()] + flags() + EXTRA.get(src, []) + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), src))
        objs.append(obj)
    failed = [src for proc, src in procs if proc.wait() != 0]
    if failed:
        raise RuntimeError(f"hipcc failed on {failed}")
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
