"""Build the FP64 CPU oracle (test infrastructure) with gcc.

The oracle is plain C99 + optional OpenMP.  No architecture-specific flags are
used so that a library built on one x86-64 host runs on another.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cg_oracle.c")
LIB = os.path.join(HERE, "libcgoracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-std=c99", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
           "-o", LIB, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    lib_t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > lib_t for f in ("cg_oracle.c", "cg_oracle.h"))


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
