"""Build libips4o.so (the HIP library behind include/ips4o.h) for gfx950.

    python paper_1705_02257_amd/build.py        # or build_library() from Python

hipcc cross-compiles here; no GPU is needed to build.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libips4o.so")
SOURCES = [os.path.join(HERE, "csrc", "driver.hip")]
HEADERS = [os.path.join(HERE, "csrc", "kernels.hpp"), os.path.join(HERE, "csrc", "traits.hpp"),
           os.path.join(HERE, "csrc", "planner.hpp"), os.path.join(HERE, "csrc", "wrword.hpp"),
           os.path.join(ROOT, "include", "ips4o.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # packed fp32 instructions are kept out of every kernel
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


def build_library(force: bool = True, verbose: bool = False) -> str:
    """Compile the library (always when force, else only when missing)."""
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + ["-o", tmp] + SOURCES
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build_library(force=True, verbose=True)
    sys.exit(0)
