"""Build libcosmo.so (the HIP kernels and the C ABI of include/cosmo.h) for gfx950.

    python -m paper_2212_01937_amd.build     (or: python paper_2212_01937_amd/build.py)

The library is built in-tree next to this file.  All device code is compiled with
packed-FP32 instruction selection disabled.  The stand-alone measurement of the
vector-ALU ceiling of code built this way (tools/valu_ceiling.hip) is not part of the
library and is built only on request:

    python -m paper_2212_01937_amd.build --valu-ceiling
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "cosmo.hip")
LIB = os.path.join(HERE, "libcosmo.so")
DEPS = [os.path.join(HERE, "csrc", f) for f in ("cmath.hpp", "carlson.hpp", "setup.hpp", "lane.hpp", "adjoint.hpp", "between.hpp", "cosmo.hip")] + [
    os.path.join(ROOT, "include", "cosmo.h")]
TOOL_SRC = os.path.join(HERE, "tools", "valu_ceiling.hip")
TOOL = os.path.join(HERE, "tools", "valu_ceiling")
ARCH = os.environ.get("COSMO_OFFLOAD_ARCH", "gfx950")
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-command-line-argument"]


def command(out):
    return ["hipcc"] + FLAGS + ["-fPIC", "-shared", "-I", os.path.join(ROOT, "include"), "-o", out, SRC]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def build_tool(verbose: bool = False) -> str:
    tmp = TOOL + ".tmp"
    cmd = ["hipcc"] + FLAGS + ["-o", tmp, TOOL_SRC]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, TOOL)
    return TOOL


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    if "--valu-ceiling" in sys.argv:
        print(build_tool(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
