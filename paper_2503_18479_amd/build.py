"""Builds libcosim.so in-tree with hipcc for gfx950.

Every HIP source is compiled to an object under ``_build/`` (in parallel),
then linked into ``paper_2503_18479_amd/libcosim.so``.  Running this module
always recompiles.
"""
from __future__ import annotations

import concurrent.futures
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libcosim.so")
ARCH = os.environ.get("COSIM_OFFLOAD_ARCH", "gfx950")

SOURCES = ["abi.cpp", "assemble.hip", "solve.hip", "solve_big.hip", "fused.hip",
           "contract_mfma.hip", "gemm_big.hip", "optim.hip", "sparam.hip", "params.hip", "noalloc.hip"]
# the S-parameter pipeline's complex GEMMs run on rocBLAS
LIBS = ["-L/opt/rocm/lib", "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"]

COMMON = [
    "-O3", "-fPIC", "-std=c++17", f"--offload-arch={ARCH}",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    # packed FP32 VALU forms stay disabled in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found (ROCm is required to build libcosim)")


# host-side AddressSanitizer build of the same sources (device code is not
# instrumented): libcosim_asan.so, for the CPU tests of the C ABI's host code
ASAN_LIB = os.path.join(PKG, "libcosim_asan.so")
ASAN_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str:
    """The compiler's ASan runtime, to be preloaded into an uninstrumented host
    process (e.g. python) that loads libcosim_asan.so."""
    base = "/opt/rocm/llvm/lib/clang"
    for v in sorted(os.listdir(base), reverse=True) if os.path.isdir(base) else []:
        p = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
        if os.path.exists(p):
            return p
    raise RuntimeError("the ASan runtime of the ROCm compiler was not found")


def _compile(src: str, asan: bool = False) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + (".asan.o" if asan else ".o"))
    lang = ["-x", "hip"] if src.endswith(".hip") else []
    cmd = [_hipcc(), *COMMON, *(ASAN_FLAGS if asan else []), *lang, "-c",
           os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj


def build(verbose: bool = False, asan: bool = False) -> str:
    """Builds libcosim.so, or with asan=True libcosim_asan.so (host code
    under AddressSanitizer)."""
    os.makedirs(BUILD, exist_ok=True)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda src: _compile(src, asan), SOURCES))
    lib = ASAN_LIB if asan else LIB
    tmp = lib + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *(ASAN_FLAGS if asan else []),
           *objs, *LIBS, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking {os.path.basename(lib)} failed:\n{' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, lib)
    if verbose:
        print(f"built {lib}")
    return lib


if __name__ == "__main__":
    build(verbose=True, asan="--asan" in sys.argv)
    sys.exit(0)
