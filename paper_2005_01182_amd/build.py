"""Build libotkm.so (the HIP solver library) in-tree with hipcc for gfx950.

Usage:  python -m paper_2005_01182_amd.build        (always recompiles)
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libotkm.so")
SOURCES = ["solve_one_lo.hip", "solve_one_hi.hip", "solve_batch_lo.hip", "solve_batch_hi.hip", "solve_grid.hip",
           "kernels.hip", "runtime.hip", "autotune.hip", "serve.hip", "serve_kernel.hip", "noalloc.hip", "bins.hip", "sparse.hip", "auction.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
    "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
    # packed FP32 instructions are kept out of every code object
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _obj(src: str, tag: str = "") -> str:
    return os.path.join(CSRC, "_build" + tag, os.path.splitext(src)[0] + ".o")


def _compile(src: str, extra=(), tag: str = "") -> str:
    out = _obj(src, tag)
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed on " + src)
    return out


def build(verbose: bool = True, extra=(), out: str = LIB) -> str:
    """Compile every HIP source and link libotkm.so next to this file (or, with
    extra compiler flags, a variant of it at `out`)."""
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    tag = "" if out == LIB else "_" + os.path.basename(out).replace(".", "_")
    with ThreadPoolExecutor(max_workers=min(max(2, os.cpu_count() or 2), len(srcs))) as ex:
        objs = list(ex.map(lambda src: _compile(src, extra, tag), srcs))
    LIB_OUT = out
    tmp = LIB_OUT + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link of libotkm.so failed")
    os.replace(tmp, LIB_OUT)
    if verbose:
        print("built", LIB_OUT)
    return LIB_OUT


if __name__ == "__main__":
    build()
