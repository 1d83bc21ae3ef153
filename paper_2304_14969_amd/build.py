"""Compile the HIP sources of the simulator into libqs.so (gfx950).

Usage: python -m paper_2304_14969_amd.build [-v] [--sanitize]
Objects go to paper_2304_14969_amd/_build/, the library next to this file.
--sanitize also builds _build/libqs_san.so: the host-side C++ (the C ABI's
argument checks, the circuit planner, the factorized-state bookkeeping, the
batch and network drivers) with AddressSanitizer and UndefinedBehaviorSanitizer,
linked with the ordinary device kernels. It is for CPU tests only (load it
with QS_LIB and the sanitizer runtime preloaded); the GPU code is unchanged.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libqs.so")

SOURCES = ["capi.cpp", "k_gates.hip", "k_qft.hip", "k_reduce.hip", "k_fused.hip",
           "k_fused_mfma.hip", "circuit.cpp", "k_factor.hip", "factor.cpp",
           "k_batch.hip", "batch.cpp", "k_mlp.hip", "k_tile.hip", "mlp.cpp"]

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    f"-I{INCLUDE}",
]


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def _compile(src: str, verbose: bool) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    cmd = [hipcc(), *FLAGS, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compiling {src} failed:\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, flush=True)
    return obj


# sources with host code worth sanitizing (the .hip files hold the kernels and
# their launch wrappers)
HOST_SOURCES = ["capi.cpp", "circuit.cpp", "factor.cpp", "batch.cpp", "mlp.cpp"]
SAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host",
             "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
             "-Xarch_host", "-fno-sanitize-recover=undefined"]
SAN_LIB = os.path.join(BUILD, "libqs_san.so")


def sanitizer_runtime() -> str:
    """Path of the AddressSanitizer runtime of the ROCm clang (to preload)."""
    import glob
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not hits:
        raise RuntimeError("no AddressSanitizer runtime under /opt/rocm/llvm")
    return hits[-1]


def build_sanitized(verbose: bool = False) -> str:
    """_build/libqs_san.so: HOST_SOURCES with ASan + UBSan on their host code,
    the kernel objects of the last ordinary build. Returns its path."""
    san = os.path.join(BUILD, "san")
    os.makedirs(san, exist_ok=True)
    if not all(os.path.exists(os.path.join(BUILD, os.path.splitext(x)[0] + ".o"))
               for x in SOURCES if x not in HOST_SOURCES):
        build(verbose)

    def comp(src):
        obj = os.path.join(san, os.path.splitext(src)[0] + ".o")
        flags = [f for f in FLAGS if f != "-O3"] + SAN_FLAGS
        cmd = [hipcc(), *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"compiling {src} (sanitized) failed:\n{r.stdout}\n{r.stderr}")
        return obj

    jobs = min(len(HOST_SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(comp, HOST_SOURCES))
    objs += [os.path.join(BUILD, os.path.splitext(x)[0] + ".o") for x in SOURCES
             if x not in HOST_SOURCES]
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-Xarch_host",
           "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-shared-libsan",
           *objs, "-o", SAN_LIB]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libqs_san.so failed:\n{r.stdout}\n{r.stderr}")
    return SAN_LIB


def build(verbose: bool = False) -> str:
    """Compile every source and link libqs.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    jobs = min(len(SOURCES), int(os.environ.get("MAX_JOBS", "8")))
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"linking libqs.so failed:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
