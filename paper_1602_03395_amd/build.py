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


HOST_SOURCES = ["fx.cpp", "tables.cpp", "batch.cpp"]


def build_sanitized(outdir: str, arch: str = "gfx950") -> str:
    """A copy of the library whose host runtime (argument validation, plan set-up, every FP64
    table, the batch planner: ``HOST_SOURCES``) is built with AddressSanitizer and
    UndefinedBehaviorSanitizer, for CPU tests. The HIP sources are linked from the objects of
    ``build()`` (rebuilt first when missing or older than their sources); their device code is
    not instrumented. The sanitizer runtime comes from the executable that loads the library
    (link it with clang's ``-fsanitize=address,undefined``)."""
    import concurrent.futures as cf
    objdir = os.path.join(HERE, "_build")
    hip_objs = [os.path.join(objdir, s + ".o") for s in SOURCES if s not in HOST_SOURCES]
    deps = [os.path.join(CSRC, n) for n in os.listdir(CSRC)] + [os.path.join(HERE, "..", "include", "fx.h")]
    newest = max(os.path.getmtime(d) for d in deps)
    if not all(os.path.exists(o) and os.path.getmtime(o) >= newest for o in hip_objs):
        build(verbose=False, arch=arch)
    os.makedirs(outdir, exist_ok=True)
    flags = [hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-Wno-unused-command-line-argument", "-I", os.path.join(HERE, "..", "include")]

    def compile_one(src):
        obj = os.path.join(outdir, src + ".san.o")
        res = subprocess.run(flags + ["-c", "-o", obj, os.path.join(CSRC, src)], capture_output=True, text=True)
        if res.returncode != 0:
            raise RuntimeError(f"sanitized compile of {src} failed:\n{res.stdout}{res.stderr}")
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(HOST_SOURCES)) as ex:
        objs = list(ex.map(compile_one, HOST_SOURCES))
    lib = os.path.join(outdir, "libfx_san.so")
    res = subprocess.run([hipcc(), f"--offload-arch={arch}", "-shared", "-fPIC", "-o", lib] + objs + hip_objs,
                         capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link of the sanitized library failed:\n{res.stdout}{res.stderr}")
    return lib


if __name__ == "__main__":
    build(verbose=True)
