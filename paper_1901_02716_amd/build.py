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


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wall"]


def _run(cmd: list[str]) -> str:
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "packed-fp32-ops"
    msg = "\n".join(ln for ln in (res.stdout + res.stderr).splitlines() if noise not in ln)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + msg)
    return msg


def build_library(out: str = LIB, verbose: bool = False) -> str:
    """Compiles every kernel and the C ABI (one hipcc per source, in
    parallel) and links them into one shared library."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor

    inc = ["-I", os.path.join(ROOT, "include")]
    with tempfile.TemporaryDirectory(prefix="maclab_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in sources()]
        jobs = [["hipcc", *FLAGS, *inc, "-c", src, "-o", obj] for src, obj in zip(sources(), objs)]
        workers = min(len(jobs), max(1, min(8, os.cpu_count() or 1)))
        with ThreadPoolExecutor(workers) as ex:
            msgs = list(ex.map(_run, jobs))
        tmp = out + ".tmp"
        msgs.append(_run(["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]))
    msg = "\n".join(m for m in msgs if m.strip())
    if verbose and msg.strip():
        print(msg, file=sys.stderr)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
