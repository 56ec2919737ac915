"""Compile the C oracle (test infrastructure) into oracle/liblbm_oracle.so.

Plain gcc, -O2 with FP contraction off so the arithmetic is exactly the
order written in lbm_oracle.c; OpenMP only splits the z loop of a step
(nodes are independent within a step, so the result does not depend on the
thread count).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIB = os.path.join(HERE, "liblbm_oracle.so")


def build(verbose=False):
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-std=c99", "-D_DEFAULT_SOURCE", "-Wall",
           "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
