"""Compile the host-only FP64 oracle (test infrastructure) with gcc.

The oracle is a separate shared library, libvkt_oracle.so, built from
vkt_oracle.c alone; it never links or includes any GPU-library source.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "vkt_oracle.c")
LIB = os.path.join(HERE, "libvkt_oracle.so")


def build_oracle(verbose: bool = False) -> str:
    """Always recompile; returns the path of the built library."""
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-D_POSIX_C_SOURCE=200809L", "-Wall",
           "-Wextra", "-fPIC", "-shared", "-pthread", "-o", tmp, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_oracle(verbose=True))
