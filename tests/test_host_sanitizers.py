"""Host code under AddressSanitizer + UndefinedBehaviorSanitizer (CPU only).

* The C ABI's host paths: the library's sources compiled for the host only
  (no device code), instrumented, linked into a small driver
  (tests/sanitize/host_abi.cpp) that runs argument validation, topology
  handles, the allocator hook's out-of-memory path and plan checks.
* The multithreaded C oracle loops (oracle/cpu_move.c) with edge-case sizes
  (tests/sanitize/oracle_cpu.c).
Both programs exit non-zero on a failed expectation or a sanitizer report.
"""
import os
import shutil
import subprocess

import pytest

from paper_2309_07337_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
# instrumentation applies to host code only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.mark.skipif(not os.path.exists(B.HIPCC), reason="hipcc not installed")
def test_abi_host_paths_under_asan_ubsan(tmp_path):
    import concurrent.futures as cf
    srcs = [os.path.join(B.CSRC, s) for s in B.SOURCES] + [os.path.join(SAN, "host_abi.cpp")]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        lang = ["-x", "hip"] if src.endswith(".hip") else []
        _run([B.HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC"]
             + HOST_SAN + ["-I", B.INCLUDE, "-I", B.CSRC] + lang + ["-c", src, "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_abi")
    _run([B.HIPCC, "--offload-arch=gfx950"] + HOST_SAN + objs + ["-o", exe])
    r = _run([exe], env=ENV, timeout=120)
    assert "0 failure(s)" in r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_cpu_oracle_loops_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_cpu")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", os.path.join(SAN, "oracle_cpu.c"), os.path.join(ROOT, "oracle", "cpu_move.c"),
          "-o", exe])
    r = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"), timeout=120)
    assert "0 mismatch(es)" in r.stdout
