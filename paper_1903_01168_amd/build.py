"""Build the HIP library ``libcglbm.so`` for gfx950 with hipcc.

Compiles every HIP/C++ source under ``csrc/`` into one shared object next to
this file.  Runs on a machine without a GPU (hipcc cross-compiles).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcglbm.so")
SOURCES = ["cg_kernels.hip", "cg_capi.cpp", "cg_server.cpp"]
HEADERS = ["cg_device.hpp", "cg_kernels.hpp", "cg_capi_internal.hpp", "cg_schedule.hpp"]

# -packed-fp32-ops: no packed FP32 instructions (v_pk_*_f32) in device code.
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def sources():
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    return [s for s in srcs if os.path.exists(s)]


def build(verbose: bool = False, extra=()) -> str:
    cmd = ["hipcc", *FLAGS, *extra, "-o", LIB + ".tmp", *sources(), "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def is_stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    deps = sources() + [os.path.join(CSRC, h) for h in HEADERS] + \
        [os.path.join(ROOT, "include", h) for h in ("cglbm.h", "cglbm_serve.h")]
    return any(os.path.exists(d) and os.path.getmtime(d) > t for d in deps)


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
