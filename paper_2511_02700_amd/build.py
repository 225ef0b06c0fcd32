"""Build the native library ``liblpide.so`` (HIP for gfx950 + host C++) in-tree.

    python -m paper_2511_02700_amd.build

Compiles csrc/lpide.hip (device kernels and the C ABI of include/lpide.h) and
csrc/host_plan.cpp (host-side discretization) with hipcc into one shared
library next to this file.
"""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblpide.so")

SOURCES = ["lpide.hip", "host_plan.cpp"]
HEADERS = ["fft.hpp", "kernels.hpp", "host_plan.hpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LPIDE_ARCH", "gfx950")


def build(verbose=False):
    """Compile every source (always) and link liblpide.so; returns its path."""
    objs = []
    common = ["-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC]
    for src in SOURCES:
        obj = os.path.join(CSRC, src + ".o")
        cmd = [HIPCC] + common
        if src.endswith(".hip"):
            # packed FP32 instructions are kept out of all device code
            cmd += ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-x", "hip"]
        cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
