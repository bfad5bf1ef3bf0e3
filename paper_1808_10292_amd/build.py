"""Build step of the HIP library: compiles csrc/*.hip for gfx950 into librsort.so.

Usage: python -m paper_1808_10292_amd.build   (or __graft_entry__.build()).
Always recompiles.  The library links the HIP runtime by its soname, so inside
a process that imported torch it binds to the runtime torch already loaded.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librsort.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "--offload-arch=" + ARCH,
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Wall",
    "-Wno-unused-result",
    # Packed fp32 instructions are kept out of every kernel.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    p = os.path.join(rocm, "bin", "hipcc")
    return p if os.path.exists(p) else "hipcc"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def build(verbose: bool = True) -> str:
    srcs = sources()
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc()] + HIPCC_FLAGS + ["-I", os.path.join(os.path.dirname(HERE), "include"),
                                     "-o", tmp] + srcs
    t0 = time.time()
    if verbose:
        print("[build] " + " ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    if verbose:
        print("[build] %s (%.1f s)" % (LIB, time.time() - t0), flush=True)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
