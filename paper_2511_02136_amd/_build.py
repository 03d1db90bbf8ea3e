"""Compile the HIP library (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "liblob.so")

SOURCES = ["lob_env.hip", "ippo.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",
    "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # lane-0 LDS counter updates need no wave-level reduction of the atomic operand
    "-mllvm", "-amdgpu-atomic-optimizer-strategy=None",
    # wave-uniform branches stay plain scalar branches (no exec-mask flow blocks)
    "-mllvm", "-structurizecfg-skip-uniform-regions",
    "-Wall",
    "-Wno-unused-function",
]


def hipcc() -> str:
    for p in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if p and os.path.exists(p):
            return p
    return "hipcc"


def build_hip(verbose: bool = False, extra_flags=()) -> str:
    """Build liblob.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *extra_flags, "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", tmp, *srcs]
    if verbose:
        print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=ROOT)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_hip(verbose=True)
