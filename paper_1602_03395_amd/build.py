"""Compile the HIP library ``libfx.so`` in-tree for gfx950.

Usage: ``python paper_1602_03395_amd/build.py`` (or ``__graft_entry__.build()``); run it as a
script, since importing the package loads the library.
Packed FP32 instructions are disabled in device code
(``-target-feature -packed-fp32-ops``); hipcc's host pass warns that it does
not know the feature, which is harmless.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfx.so")
SOURCES = ["fx.cpp", "tables.cpp", "batch.cpp", "kernels.hip", "kernels_p2.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, arch: str = "gfx950") -> str:
    out_tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(HERE, "..", "include"),
           "-o", out_tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and res.stderr.strip():
        # keep warnings visible but short
        lines = [ln for ln in res.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            sys.stderr.write("\n".join(lines[:40]) + "\n")
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
