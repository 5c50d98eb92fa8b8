"""Builds the CPU oracle library ``oracle/liboracle.so`` with gcc.

Test infrastructure only: the product path never links or loads it.
The source is compiled twice -- values only (``*_v`` symbols) and with four
forward-mode tangents (``*_g`` symbols) -- with contraction off so that every
product and sum is a separately rounded IEEE binary64 operation.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "btoracle.c")
LIB = os.path.join(HERE, "liboracle.so")
FLAGS = ["-O2", "-fPIC", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
         "-Wall", "-Wno-unused-function"]


def build(verbose: bool = False) -> str:
    objs = []
    for nt in (0, 4):
        obj = os.path.join(HERE, f"btoracle_nt{nt}.o")
        cmd = ["gcc", *FLAGS, f"-DNT={nt}", "-c", SRC, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
