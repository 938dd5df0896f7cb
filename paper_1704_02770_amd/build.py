"""Builds libqkrylov.so in-tree for gfx950 with hipcc.

Usage: python paper_1704_02770_amd/build.py   (or call build()).
Run it by path, not as a module of the package: importing the package loads
the library this script produces.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libqkrylov.so")
SOURCES = ["qk_kernels.hip", "qk_blocked.hip", "qk_split.hip", "qk_batch.hip", "qk_persist.hip", "qk_grad.hip",
           "qk_abi.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-fvisibility=hidden",
    # packed FP32 instructions stay off in every HIP translation unit
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only where one source expression holds both, so
    # a kernel body gives the same bits in every kernel it is inlined into
    # (the plain launches and the persistent step) and in every variant of it
    "-ffp-contract=on",
    "-Wno-unused-command-line-argument",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libqkrylov.so (always recompiles)."""
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed building libqkrylov.so")
    os.replace(tmp, LIB)
    build_c_demo(verbose)
    return LIB


DEMO_SRC = os.path.join(ROOT, "tests", "c_abi", "qk_demo.c")
DEMO = os.path.join(ROOT, "tests", "c_abi", "qk_demo")


def build_c_demo(verbose: bool = False) -> str:
    """The plain C user of the ABI (tests/c_abi/qk_demo.c), linked against the
    in-tree library and the HIP runtime with gcc."""
    rocm = os.path.dirname(os.path.dirname(os.path.realpath(HIPCC)))
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(rocm, "include"), DEMO_SRC,
           "-L", HERE, "-lqkrylov", "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_1704_02770_amd", "-Wl,-rpath," + os.path.join(rocm, "lib"), "-o", DEMO]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("gcc failed building tests/c_abi/qk_demo")
    return DEMO


if __name__ == "__main__":
    print(build(verbose=True))
