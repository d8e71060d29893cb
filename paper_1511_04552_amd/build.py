"""Build step of the HIP library ``libmclbm.so`` for gfx950 (hipcc, in-tree)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(HERE, "csrc", "mclbm.hip"), os.path.join(HERE, "csrc", "nn.hip")]
SO = os.path.join(HERE, "libmclbm.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    "--offload-arch=gfx950",
    # packed FP32 instructions are not emitted (v_pk_* FP32 forms)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # multiply-adds are fused only within one expression, so a kernel's
    # arithmetic does not depend on the code it is inlined into: every
    # kernel that runs the node update gives the same bits
    "-ffp-contract=on",
    "-Wall", "-Wno-unused-function",
]


DRIVER_SRC = os.path.join(ROOT, "tests", "c_abi", "cavity_driver.c")
DRIVER = os.path.join(ROOT, "tests", "c_abi", "cavity_driver")


def build_c_driver(verbose: bool = False) -> str:
    """The plain C program on the C ABI (gcc, host code only; it finds the
    in-tree library through an rpath relative to itself)."""
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), DRIVER_SRC, "-L", HERE, "-lmclbm",
           "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,$ORIGIN/../../paper_1511_04552_amd",
           "-Wl,-rpath,/opt/rocm/lib", "-lm", "-o", DRIVER]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return DRIVER


def build(verbose: bool = False) -> str:
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), "-o", SO + ".tmp", *SRCS]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SO + ".tmp", SO)
    return SO


if __name__ == "__main__":
    print(build(verbose=True))
