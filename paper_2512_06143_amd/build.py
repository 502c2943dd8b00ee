"""Build libgp2s.so (HIP kernels + C ABI) for gfx950 with hipcc, in-tree.

Usage: python paper_2512_06143_amd/build.py  (or __graft_entry__.build()). Run it
as a file: importing the package first would load the library being rebuilt.
Every call recompiles. Object files go to paper_2512_06143_amd/_build/.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libgp2s.so")

SOURCES = ["abi.hip", "batch_abi.hip", "batch.hip", "prologue.hip", "scan.hip", "assemble.hip", "spmv.hip", "pcg.hip", "slq.hip",
           "backward.hip", "predict.hip", "blockjac.hip", "farfield.hip", "grouped.hip", "bsplit.hip"]

ARCH = os.environ.get("GP2S_OFFLOAD_ARCH", "gfx950")
# Packed FP32 instructions are disabled for all device code.
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


# Host-side sanitizers for the CPU check of the runtime and validation layer (device
# code is built as usual; each -fsanitize applies to the host pass only).
SANITIZE = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer".split()
BUILD_SAN = os.path.join(PKG, "_build_asan")
LIB_SAN = os.path.join(BUILD_SAN, "libgp2s_asan.so")


def _compile(src: str, sanitize: bool = False) -> str:
    obj = os.path.join(BUILD_SAN if sanitize else BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [_hipcc(), *COMMON, *(SANITIZE if sanitize else []), "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr[-6000:]}")
    return obj


def build_sanitized(verbose: bool = False) -> str:
    """libgp2s_asan.so: the same sources with the host code under AddressSanitizer and
    UndefinedBehaviorSanitizer, for the CPU-only check of the host runtime."""
    os.makedirs(BUILD_SAN, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(lambda s: _compile(s, True), SOURCES))
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *SANITIZE, *objs, "-o", LIB_SAN]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"sanitized link failed:\n{res.stderr[-6000:]}")
    if verbose:
        print(f"built {LIB_SAN}")
    return LIB_SAN


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with ThreadPoolExecutor(max_workers=workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-6000:]}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB}")
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
