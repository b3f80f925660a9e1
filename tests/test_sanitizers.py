"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU.

* The library's host runtime (argument validation of every entry point, plan set-up with every
  FP64 table, the batch planner) rebuilt with both sanitizers and driven by a C program over
  invalid arguments and a sweep of valid problems (``tests/sanitize/abi_driver.c``); with no GPU
  present each valid plan stops at its first device allocation, after all of its host work.
* The oracle's kernel table ``oracle/gtable.c`` driven over a sweep of lengths, magnifications,
  offsets and flight times (``tests/sanitize/gtable_driver.c``).
Either run fails on the first sanitizer report (no recovery) or on any leak.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CLANG = "/opt/rocm/llvm/bin/clang"
SAN = ["-g", "-O1", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    res = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert res.returncode == 0, res.stdout[-4000:] + res.stderr[-4000:]
    return res.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_gtable_under_sanitizers(tmp_path):
    exe = str(tmp_path / "gtable_driver")
    subprocess.run(["gcc"] + SAN + [os.path.join(ROOT, "oracle", "gtable.c"), os.path.join(HERE, "gtable_driver.c"),
                                    "-lm", "-o", exe], check=True)
    assert "0 failures" in _run(exe)


@pytest.mark.skipif(not os.path.exists(CLANG) or not os.path.exists("/opt/rocm/bin/hipcc"), reason="ROCm clang not found")
def test_host_runtime_under_sanitizers(tmp_path):
    sys.path.insert(0, os.path.join(ROOT, "paper_1602_03395_amd"))
    try:
        import build
    finally:
        sys.path.pop(0)
    lib = build.build_sanitized(str(tmp_path / "lib"))
    exe = str(tmp_path / "abi_driver")
    libdir = os.path.dirname(lib)
    subprocess.run([CLANG] + SAN + ["-I", os.path.join(ROOT, "include"), os.path.join(HERE, "abi_driver.c"),
                                    "-L", libdir, "-lfx_san", f"-Wl,-rpath,{libdir}", "-lm", "-o", exe], check=True)
    out = _run(exe)
    assert "0 failures" in out
    assert int(out.split("abi driver: ")[1].split()[0]) > 300  # the sweep of valid problems ran
