"""Build the native library ``liblpide.so`` (HIP for gfx950 + host C++) in-tree.

    python -m paper_2511_02700_amd.build

Compiles, in parallel, csrc/lpide.hip (plans, groups, batches, the adjoint
driver and the C ABI of include/lpide.h), csrc/march_L.hip once per transform
size L (the launch sequences of the march kernels for that size),
csrc/host_plan.cpp (host-side discretization), and the price-space plan
(csrc/ps.hip, csrc/ps_host.cpp, csrc/ps_L.hip once per size) with hipcc, and
links them into one shared library next to this file.
"""

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "liblpide.so")

SIZES = [64, 128, 256, 512, 768, 1024, 1536, 2048, 3072, 4096]
# the price-space plan's transform sides: also 7-smooth sides 2^m p (p = 5, 7, 9) and the two-level sides
PS_SIZES = SIZES + [640, 896, 1152, 1280, 1792, 2304, 2560, 3584, 4608, 5120, 6144, 7168, 8192, 12288, 16384, 24576]
# (source, object, extra flags)
UNITS = ([("lpide.hip", "lpide.o", []), ("host_plan.cpp", "host_plan.o", []), ("ps.hip", "ps.o", []),
          ("ps_host.cpp", "ps_host.o", [])] +
         [("march_L.hip", "march_L%d.o" % L, ["-DLPIDE_L=%d" % L]) for L in SIZES] +
         [("ps_L.hip", "ps_L%d.o" % L, ["-DLPIDE_L=%d" % L]) for L in PS_SIZES])

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("LPIDE_ARCH", "gfx950")


def _compile(src, obj, extra, verbose):
    cmd = [HIPCC, "-O3", "-std=c++17", "-fPIC", "-I", INCLUDE, "-I", CSRC] + extra
    if src.endswith(".hip"):
        # packed FP32 instructions are kept out of all device code
        cmd += ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-x", "hip"]
    cmd += ["-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return obj


def build(verbose=False, jobs=None):
    """Compile every translation unit (always) and link liblpide.so; returns its path."""
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    # a failed build leaves no library behind, so nothing runs stale code
    if os.path.exists(LIB):
        os.remove(LIB)
    objs = [os.path.join(CSRC, o) for _, o, _ in UNITS]
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        futs = [ex.submit(_compile, src, obj, extra, verbose) for (src, _, extra), obj in zip(UNITS, objs)]
        for f in futs:
            f.result()
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
