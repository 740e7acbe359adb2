"""Builds the HIP library ``libmaclab.so`` for gfx950 in-tree with hipcc.

Usage: ``python -m paper_1901_02716_amd.build`` (or ``build_library()``).
Packed FP32 instructions are switched off for every kernel (the
``-packed-fp32-ops`` target feature); hipcc's host pass warns that it does not
know that feature, which is harmless.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libmaclab.so")
ARCH = "gfx950"


def sources() -> list[str]:
    return sorted(glob.glob(os.path.join(HERE, "csrc", "*.hip")))


def command(out: str = LIB) -> list[str]:
    return ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-I", os.path.join(ROOT, "include"), *sources(), "-o", out]


def build_library(out: str = LIB, verbose: bool = False) -> str:
    """Compiles every kernel and the C ABI into one shared library."""
    tmp = out + ".tmp"
    cmd = command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msg = "\n".join(ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + msg)
    if verbose and msg.strip():
        print(msg, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
