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
SOURCES = ["fx.cpp", "tables.cpp", "batch.cpp", "kernels.hip", "kernels_p2.hip", "kernels_ct.hip", "kernels_cfp.hip", "pair.hip", "farfield.hip", "brute.hip", "noalloc.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, arch: str = "gfx950") -> str:
    """Compiles every source to an object (in parallel) and links libfx.so."""
    import concurrent.futures as cf
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    common = [hipcc(), f"--offload-arch={arch}", "-O3", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]

    def compile_one(src):
        obj = os.path.join(objdir, src + ".o")
        cmd = common + ["-c", "-o", obj, os.path.join(CSRC, src)]
        res = subprocess.run(cmd, capture_output=True, text=True)
        return src, obj, cmd, res

    objs = []
    workers = min(len(SOURCES), max(1, os.cpu_count() or 1))
    with cf.ThreadPoolExecutor(max_workers=workers) as ex:
        for src, obj, cmd, res in ex.map(compile_one, SOURCES):
            if verbose:
                print(" ".join(cmd), flush=True)
            if res.returncode != 0:
                sys.stderr.write(res.stdout + res.stderr)
                raise RuntimeError(f"hipcc failed on {src}")
            objs.append(obj)
    out_tmp = LIB + ".tmp"
    link = [hipcc(), f"--offload-arch={arch}", "-shared", "-fPIC", "-o", out_tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    res = subprocess.run(link, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("link failed")
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
