"""Host code of the library under AddressSanitizer and UndefinedBehavior-
Sanitizer, on the CPU.

Every source is compiled with the sanitizers on the host side only (the
device code is built as usual and never launched here), linked into a
separate shared library in a temporary directory, and driven by
``tests/sanitize_driver.c`` through the status strings, layout queries,
wisdom parsing and argument checks.  The in-tree library is not touched."""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_1611_02665_amd import build as BUILD  # noqa: E402

ROCM = os.path.dirname(os.path.dirname(os.path.realpath(BUILD.HIPCC)))
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
ROCM_LIB = os.path.join(ROCM, "lib")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]
SAN_LINK = ["-fsanitize=address,undefined", "-shared-libsan"]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


@pytest.mark.skipif(not (os.path.exists(BUILD.HIPCC) and os.path.exists(CLANG)),
                    reason="hipcc / clang not installed")
def test_host_code_under_asan_and_ubsan(tmp_path):
    flags = ["-x", "hip", f"--offload-arch={BUILD.ARCH}", "-O1", "-g", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", BUILD.INCLUDE, "-I", BUILD.CSRC, *SAN_HOST]

    def compile_one(src):
        obj = str(tmp_path / (src + ".o"))
        _run([BUILD.HIPCC, *flags, "-c", os.path.join(BUILD.CSRC, src), "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(BUILD.SOURCES))) as ex:
        objs = list(ex.map(compile_one, BUILD.SOURCES))
    lib = str(tmp_path / "libbspline_san.so")
    # the shared sanitizer runtime the objects were built against
    rt = _run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"]).stdout.strip()
    rpath = ["-Wl,-rpath," + p for p in (str(tmp_path), ROCM_LIB, os.path.dirname(rt))]
    _run([CLANGXX, "-shared", *SAN_LINK, "-o", lib, *objs, "-L", ROCM_LIB, "-lamdhip64", *rpath])
    exe = str(tmp_path / "sanitize_driver")
    _run([CLANG, "-std=c99", "-g", *SAN_LINK, "-I", BUILD.INCLUDE,
          os.path.join(ROOT, "tests", "sanitize_driver.c"), "-o", exe, lib, *rpath])
    env = dict(os.environ,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env,
                       timeout=300)
    assert r.returncode == 0 and r.stdout.strip() == "ok", f"{r.stdout}\n{r.stderr}"
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    shutil.rmtree(tmp_path / "no", ignore_errors=True)
