"""Build the HIP library liblbm.so (gfx950) in-tree with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["kernels.hip", "runtime.hip", "probes.hip"]
ARCH = os.environ.get("LBM_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
    "-Wall", "-Wno-unused-function",
    # packed FP32 (v_pk_*_f32) stays off in all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no multiply-add fusion: each operation rounds as written, so the same
    # arithmetic gives the same bits in every kernel it is inlined into
    # (AA vs AB, alone vs batched, checkpoint at either parity)
    "-ffp-contract=off",
]


def build(verbose=False, extra=()):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc] + FLAGS + list(extra) + ["-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


C_ABI_TEST = os.path.join(os.path.dirname(HERE), "tests", "c_abi")


def build_c_abi_test(verbose=False):
    """The plain-C program that drives the library through include/lbm.h
    only (tests/c_abi/lid_cavity.c), linked against liblbm.so with a
    relative run path."""
    src = os.path.join(C_ABI_TEST, "lid_cavity.c")
    out = os.path.join(C_ABI_TEST, "lid_cavity")
    rel = os.path.relpath(HERE, C_ABI_TEST)
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", src, "-o", out + ".tmp", "-L" + HERE,
           "-llbm", "-Wl,-rpath,$ORIGIN/" + rel]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
