"""Compile the HIP library for gfx950: one translation unit, no relocatable
device code, FP contraction off and no fast math (bit-reproducible hit
placement), packed FP32 instructions disabled."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
SRC = os.path.join(PKG, "csrc", "fcs_runtime.hip")
LIB = os.path.join(PKG, "libfcs.so")
# measured ceilings of the chip (atomics, HBM copy, VALU, launches): benchmark only
CEIL_SRC = os.path.join(PKG, "csrc", "fcs_ceilings.hip")
CEIL_LIB = os.path.join(PKG, "libfcs_ceilings.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
]


def _compile(src: str, lib: str, verbose: bool, libs=()) -> str:
    tmp = lib + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
           src, "-o", tmp, *libs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile libfcs.so (the C ABI) and libfcs_ceilings.so (the benchmark's
    ceiling measurements); returns the path of libfcs.so."""
    _compile(CEIL_SRC, CEIL_LIB, verbose)
    # roctx ranges around the entry points (rocprofv3 --marker-trace)
    return _compile(SRC, LIB, verbose, libs=("-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"))


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
