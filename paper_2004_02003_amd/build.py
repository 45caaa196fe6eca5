"""Build the HIP library ``libbto.so`` for gfx950 (in-tree, next to this file)."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libbto.so")
SOURCES = ["advect.hip", "tiles.hip", "seed_flowmap.hip", "adjoint.hip", "grad_reduce.hip", "rebin.hip", "reconstruct.hip",
           "touched.hip", "radix.hip", "api.hip"]
ARCH = os.environ.get("BTO_OFFLOAD_ARCH", "gfx950")


DEMO_SRC = os.path.join(HERE, "c_abi_demo.c")
DEMO = os.path.join(HERE, "bto_c_abi_demo")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_demo(verbose: bool = False) -> str:
    """Plain C consumer of the C-ABI (gcc, HIP runtime API, links libbto.so)."""
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-I", os.path.join(ROOT, "include"), DEMO_SRC, "-o", DEMO + ".tmp", "-L", HERE, "-lbto",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath,$ORIGIN",
           "-Wl,-rpath," + os.path.join(ROCM, "lib"), "-lm"]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(DEMO + ".tmp", DEMO)
    return DEMO


def build(verbose: bool = False) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-o", LIB + ".tmp"] + srcs
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    build_demo(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
