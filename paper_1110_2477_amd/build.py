"""Builds ``libbtprice.so`` (HIP kernels + C ABI) for gfx950 with hipcc.

Flags that matter for results: ``-ffp-contract=off`` (every product and sum
rounds separately, as the method's canonical operations require) and no
fast-math; IEEE-correct binary64 division is hipcc's default.  Packed FP32
instructions are disabled for all HIP code.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libbtprice.so")
SOURCES = [os.path.join(CSRC, "bt_kernels.hip")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"


def hip_flags():
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
        "-ffp-contract=off", "-fno-fast-math",
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
        "-I" + os.path.join(ROOT, "include"),
    ]


CPU_LIB = os.path.join(HERE, "libbtcpu.so")
CPU_SOURCES = [os.path.join(CSRC, "bt_cpu_alg1.cpp")]


def build_cpu(verbose: bool = False) -> str:
    """libbtcpu.so: the paper's Algorithm 1 on host threads (include/bt_cpu.h),
    built with the host compiler from the same per-node code as the kernels
    (contraction off, so its results are the kernels' bits)."""
    tmp = CPU_LIB + ".tmp"
    cmd = ["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-pthread", "-ffp-contract=off", "-fno-fast-math",
           "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
           "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-o", tmp, *CPU_SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build(verbose: bool = False, extra=()) -> str:
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *hip_flags(), *extra, "-shared", "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_cpu(verbose)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True, extra=[a for a in sys.argv[1:] if a != "-v"]))
