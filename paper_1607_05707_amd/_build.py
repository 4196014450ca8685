"""Compile the HIP sources into the in-tree shared library for gfx950.

Produces ``paper_1607_05707_amd/_lib/libirgl.so`` (the C ABI declared in
``include/irgl.h``).  Always recompiles; callers that only need the library
load what is built.
"""
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIBDIR = os.path.join(PKG, "_lib")
LIB = os.path.join(LIBDIR, "libirgl.so")
RUNNER = os.path.join(LIBDIR, "irgl_run")
ARCH = os.environ.get("IRGL_OFFLOAD_ARCH", "gfx950")

SOURCES = ["irgl.hip", "irgl_mst.hip", "irgl_pipe.hip", "irgl_dmr.hip"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the HIP library)")


def build(verbose: bool = False, extra=()) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           # no packed-FP32 instructions anywhere in device code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    cmd += list(extra)
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    cmd += ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    # native runner over the C ABI (timing / profiling without Python)
    rcmd = [hipcc(), "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
            os.path.join(CSRC, "irgl_run.cpp"), "-L", LIBDIR, "-lirgl",
            "-Wl,-rpath,$ORIGIN", "-o", RUNNER + ".tmp"]
    if verbose:
        print(" ".join(rcmd), flush=True)
    subprocess.check_call(rcmd)
    os.replace(RUNNER + ".tmp", RUNNER)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=sys.argv[1:]))
