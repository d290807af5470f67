"""Build ``libbspline.so`` (HIP for gfx950) in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libbspline.so")
OBJDIR = os.path.join(PKG, "_build")

SOURCES = ["eval_f32.hip", "eval_f16.hip", "eval_bf16.hip", "eval_launch.hip", "table.cpp",
           "layout_kernels.hip", "order_kernels.hip", "fit_kernels.hip", "autotune.cpp",
           "batch.cpp", "noalloc.hip", "stream_probe.hip"]
ARCH = os.environ.get("BSPL_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CFLAGS = [
    "-x", "hip", f"--offload-arch={ARCH}", "-O3", "-fPIC", "-std=c++17",
    "-Wall", "-Wno-unused-function",
    # generated packed FP32 arithmetic is disabled for every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", INCLUDE, "-I", CSRC,
]


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [HIPCC, *CFLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(os.cpu_count() or 4, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB




DEMO_SRC = os.path.join(ROOT, "tests", "c_abi_demo.c")
DEMO_BIN = os.path.join(ROOT, "tests", "c_abi_demo")


def build_c_demo(verbose: bool = False) -> str:
    """The plain-C use of the ABI that the tests run (host C, gcc)."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-I", INCLUDE, "-I", os.path.join(rocm, "include"),
           "-D__HIP_PLATFORM_AMD__", DEMO_SRC, "-o", DEMO_BIN, "-L", PKG, "-lbspline",
           "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN/../paper_1611_02665_amd",
           "-Wl,-rpath," + os.path.join(rocm, "lib")]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for the C demo:\n{r.stdout}\n{r.stderr}")
    if verbose:
        print(f"built {DEMO_BIN}")
    return DEMO_BIN


if __name__ == "__main__":
    build(verbose=True)
    build_c_demo(verbose=True)
    sys.exit(0)
