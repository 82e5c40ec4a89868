"""Build the gfx950 shared library libcofem.so in-tree with hipcc.

Usage: python -m paper_2105_10439_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(PKG, "libcofem.so")

SOURCES = ["kernels.hip", "conv.hip", "dct.hip", "cofem.hip", "serve.hip", "noalloc.hip"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-fvisibility=hidden",
    # keep the compiler from forming packed FP32 instructions (v_pk_*_f32)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-result",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, "-I", INCLUDE, "-I", CSRC, "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    # the host pass warns that it does not know the packed-FP32 feature: harmless
    msgs = [l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + "\n".join(msgs))
    if verbose and msgs:
        print("\n".join(msgs))
    os.replace(tmp, LIB)
    build_c_caller(verbose)
    build_layout_check(verbose)
    return LIB


C_CALLER_SRC = os.path.join(ROOT, "tests", "c", "fit_smoke.c")
C_CALLER = os.path.join(ROOT, "tests", "c", "fit_smoke")


def build_c_caller(verbose: bool = False) -> str:
    """The plain-C test caller of the library (gcc, C99, links libcofem.so and the HIP
    runtime): proves the boundary is usable from C without the Python binding."""
    rocm = os.path.dirname(os.path.dirname(hipcc()))
    cmd = ["gcc", "-std=c99", "-O2", "-Wall", "-I", INCLUDE, "-I", os.path.join(rocm, "include"),
           "-D__HIP_PLATFORM_AMD__", C_CALLER_SRC, "-L", PKG, "-lcofem", "-L", os.path.join(rocm, "lib"),
           "-lamdhip64", f"-Wl,-rpath,{PKG}:{os.path.join(rocm, 'lib')}", "-o", C_CALLER]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("gcc failed for the C caller:\n" + res.stdout + res.stderr)
    return C_CALLER


LAYOUT_CHECK_SRC = os.path.join(ROOT, "tests", "c", "layout_check.hip")
LAYOUT_CHECK = os.path.join(ROOT, "tests", "c", "layout_check")


def build_layout_check(verbose: bool = False) -> str:
    """A host program that checks the FIR signal-slice layout function of the device helpers
    (it runs on the CPU; no device code is launched)."""
    flags = [f for f in HIPCC_FLAGS if f not in ("-fPIC", "-shared", "-fvisibility=hidden")]
    cmd = [hipcc(), *flags, "-I", INCLUDE, "-I", CSRC, "-o", LAYOUT_CHECK, LAYOUT_CHECK_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        msgs = [l for l in (res.stdout + res.stderr).splitlines() if "packed-fp32-ops" not in l]
        raise RuntimeError("hipcc failed for the layout check:\n" + "\n".join(msgs))
    return LAYOUT_CHECK


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
