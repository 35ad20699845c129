"""Build the HIP library liblcs.so in-tree for gfx950.

    python -m paper_2001_01158_amd.build

Flags: -ffp-contract=off keeps every product and sum rounded as written (the
kernels use fma() only where a fused step is intended, which makes the
marking bit-reproducible); packed FP32 instructions are disabled.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "lcs.hip")
LIB = os.path.join(HERE, "liblcs.so")
ARCH = os.environ.get("LCS_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out: str) -> list:
    return ["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            "-o", out, SRC]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
