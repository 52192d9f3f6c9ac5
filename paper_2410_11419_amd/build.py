"""Build libgs3.so (the HIP kernels and the C-ABI) for gfx950, in-tree.

    python -m paper_2410_11419_amd.build [--jobs N] [--debug] [--host-check]

Each ``csrc/*.hip`` is compiled to an object under ``_build/`` at the repo
root and the objects are linked into ``paper_2410_11419_amd/libgs3.so``.
Packed-FP32 instructions are disabled for all device code.

``--host-check`` (``build_host_check``) also builds, under ``_build_san/``,
a copy of the library whose host code carries AddressSanitizer and
UndefinedBehaviorSanitizer instrumentation (the device code is built as
usual) and ``tests/host_abi_check.c`` linked against it: a program that
drives every host-side decision of the C-ABI without a GPU.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libgs3.so")
ARCH = "gfx950"

# - no packed fp32 instructions (plain float code only);
# - no atomic optimizer: the kernels reduce a value across the wave (or a
#   16-lane row) before one lane adds it, and the optimizer would wrap each
#   such single-lane atomic in a scan loop over the active lanes.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-mllvm", "-amdgpu-atomic-optimizer-strategy=None"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: install ROCm or set HIPCC")


BUILD_SAN = os.path.join(ROOT, "_build_san")
LIB_SAN = os.path.join(BUILD_SAN, "libgs3_san.so")
HOST_CHECK = os.path.join(BUILD_SAN, "host_abi_check")
HOST_CHECK_SRC = os.path.join(ROOT, "tests", "host_abi_check.c")
# host-code sanitizers only: each flag goes to the host compilation (the
# device code cannot carry them); vptr checks need the C++ runtime of the
# sanitizers, which a C test program does not link
SAN_HOST_FLAGS = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                  "-Xarch_host", "-fno-sanitize=vptr", "-Xarch_host", "-fno-sanitize-recover=undefined",
                  "-Xarch_host", "-fno-omit-frame-pointer"]


def compile_one(src: str, debug: bool, out_dir: str = BUILD, extra=()) -> str:
    obj = os.path.join(out_dir, os.path.basename(src).replace(".hip", ".o"))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-std=c++17", "-fPIC", "-c", src, "-o", obj,
           "-I", os.path.join(ROOT, "include"), "-Wall", "-Wno-unused-function"]
    cmd += ["-O1", "-g"] if debug else ["-O3"]
    cmd += DEVICE_FLAGS + list(extra)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops' is not a recognized feature" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{out}")
    if out.strip():
        print(out, file=sys.stderr)
    return obj


def build(jobs: int = 8, debug: bool = False, verbose: bool = True) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: compile_one(s, debug), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}{r.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} from {len(srcs)} sources")
    return LIB


def clang() -> str:
    for cand in (os.environ.get("CLANG"), "/opt/rocm/llvm/bin/clang", shutil.which("clang")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("clang not found: install ROCm or set CLANG")


def build_host_check(jobs: int = 8, verbose: bool = True) -> str:
    """The sanitizer-instrumented library and the host check program."""
    os.makedirs(BUILD_SAN, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    with cf.ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(lambda s: compile_one(s, True, BUILD_SAN, SAN_HOST_FLAGS), srcs))
    cmd = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", LIB_SAN] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}{r.stderr}")
    # the C program is built by clang alone (no HIP source on this line),
    # which links the sanitizer runtimes the library's host code calls
    cmd = [clang(), "-std=c11", "-Wall", "-Werror", "-g", "-O1", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"),
           HOST_CHECK_SRC, "-L", BUILD_SAN, "-lgs3_san", f"-Wl,-rpath,{BUILD_SAN}", "-o", HOST_CHECK]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"host check build failed: {' '.join(cmd)}\n{r.stdout}{r.stderr}")
    if verbose:
        print(f"built {HOST_CHECK} against {LIB_SAN}")
    return HOST_CHECK


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=8)
    ap.add_argument("--debug", action="store_true")
    ap.add_argument("--host-check", action="store_true")
    a = ap.parse_args()
    build(a.jobs, a.debug)
    if a.host_check:
        build_host_check(a.jobs)
