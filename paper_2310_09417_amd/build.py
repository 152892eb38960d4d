"""Build of the HIP shared library (gfx950) in-tree: ``librid.so`` next to
this file.  Called by ``__graft_entry__.build()``; runs hipcc on the CPU."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librid.so")
SOURCES = [os.path.join(CSRC, "rid_api.hip")]  # the library (the driver below links it)
DEPS = SOURCES + [os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hpp", ".h"))] + [
    os.path.join(ROOT, "include", "rid.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


NATIVE = os.path.join(HERE, "rid_bench_native")
NATIVE_SRC = os.path.join(CSRC, "rid_bench_native.hip")


def build_native(verbose: bool = False) -> str:
    """Native profiling driver linked against librid.so (no Python)."""
    tmp = NATIVE + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-o", tmp, NATIVE_SRC,
           "-L", HERE, "-lrid", "-Wl,-rpath,$ORIGIN"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, NATIVE)
    return NATIVE


def build(force: bool = True, verbose: bool = False) -> str:
    if not force and os.path.exists(LIB) and all(
            os.path.getmtime(LIB) >= os.path.getmtime(d) for d in DEPS):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_native(verbose)
    return LIB


if __name__ == "__main__":
    print(build(force=True, verbose=True))
