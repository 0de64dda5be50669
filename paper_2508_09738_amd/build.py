"""Builds libgfw.so (the HIP library behind include/gfw.h) in-tree for gfx950."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgfw.so")
SOURCES = ["gfw_api.hip", "gfw_batch.hip", "gfw_gauss.hip", "gfw_active.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-function",
    "-Wno-unused-result",
    # packed FP32 instructions are not used by this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # a*b + c is two roundings, as written (no fused multiply-add contraction): the FP64
    # sums of L U then round exactly as a plain CSR loop over the operator does
    "-ffp-contract=off",
    "-fvisibility=hidden",
]


def sources() -> list:
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into paper_2508_09738_amd/libgfw.so (always rebuilds).  The
    sources compile to objects in parallel, then link."""
    import tempfile

    inc = ["-I", os.path.join(ROOT, "include")]
    compile_flags = [f for f in FLAGS if f != "-shared"]
    with tempfile.TemporaryDirectory(prefix="gfw_build_") as tmp:
        objs, procs = [], []
        for src in sources():
            obj = os.path.join(tmp, os.path.basename(src) + ".o")
            cmd = [HIPCC] + compile_flags + inc + ["-c", "-o", obj, src]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd, cwd=CSRC), cmd))
            objs.append(obj)
        for pr, cmd in procs:
            if pr.wait() != 0:
                raise subprocess.CalledProcessError(pr.returncode, cmd)
        out_tmp = LIB + ".tmp"
        cmd = [HIPCC] + FLAGS + ["-o", out_tmp] + objs
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
