"""Native code checked on the CPU under AddressSanitizer and UBSan (no GPU):

* the workgroup FFT of csrc/fft.hpp, unchanged, compiled for the host against
  a small emulation of the HIP facilities it uses (tests/cpu/emu: one OS thread
  per GPU thread, a barrier for __syncthreads), at every transform side and
  elements-per-thread choice the library instantiates, FP64 and FP32, forward
  and inverse, against the DFT in long double (tests/cpu/fft_emu.cpp), with the
  LDS buffer and the twiddle tables in exactly sized heap arrays;
* the host discretization csrc/host_plan.cpp (density, weights, diffusion,
  folded kernel, initial grids of every pay-off, line factors, semi-Lagrangian
  tables) on the nig64 workload, its derived quantities against the oracle's.
"""

import math
import os
import shutil
import subprocess

import pytest

import workloads
from oracle import integral, levy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_02700_amd", "csrc")
CPU = os.path.join(ROOT, "tests", "cpu")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _gxx():
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    return gxx


def _run(cmd, **kw):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run(cmd, capture_output=True, text=True, env=env, **kw)


def test_workgroup_fft_emulated_under_sanitizers(tmp_path):
    # the cases are compiled as PARTS programs in parallel (one translation unit
    # takes about 100 s under the sanitizers), each run after its build
    PARTS = 4
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    exes = [str(tmp_path / ("fft_emu%d" % q)) for q in range(PARTS)]
    builds = [subprocess.Popen([_gxx(), "-std=c++20"] + SAN +
                               ["-DFFT_EMU_PARTS=%d" % PARTS, "-DFFT_EMU_PART=%d" % q, "-I", os.path.join(CPU, "emu"),
                                "-I", CSRC, os.path.join(CPU, "fft_emu.cpp"), "-o", exes[q], "-lpthread"],
                               stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True, env=env)
              for q in range(PARTS)]
    for b in builds:
        _, err = b.communicate(timeout=900)
        assert b.returncode == 0, err[-3000:]
    cases = []
    for exe in exes:
        r = _run([exe], timeout=600)
        assert r.returncode == 0 and "ALL OK" in r.stdout, (r.stdout[-2000:], r.stderr[-3000:])
        assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
        cases += [line for line in r.stdout.splitlines() if " ok" in line]
    assert len(cases) >= 160          # sides x radices x {fp64, fp32} x {forward, inverse}


def test_host_plan_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_plan_check")
    r = _run([_gxx(), "-std=c++17"] + SAN + ["-I", os.path.join(ROOT, "include"), "-I", CSRC,
                                             os.path.join(CSRC, "host_plan.cpp"), os.path.join(CPU, "host_plan_check.cpp"),
                                             "-o", exe, "-lpthread"])
    assert r.returncode == 0, r.stderr[-3000:]
    w = workloads.workload("nig64")
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    rho = p["rho"]
    args = [p["alpha"], p["delta"], p["lam"], p["eta"][0], p["eta"][1], rho[0][0], rho[0][1], rho[1][1], w["r"],
            w["n"], w["y_lo"], w["y_hi"]]
    r = _run([exe] + ["%.17g" % float(a) for a in args], timeout=600)
    assert r.returncode == 0 and r.stdout.rstrip().endswith("OK"), (r.stdout[-2000:], r.stderr[-3000:])
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    got = dict(line.split() for line in r.stdout.splitlines() if " " in line)
    h = (w["y_hi"] - w["y_lo"]) / (w["n"] - 1)
    d = integral.discretize(p, h, w["r"])
    assert int(got["N_z"]) == d["N_z"] and int(got["M2"]) == d["M2"]
    assert math.isclose(float(got["sum_omega"]), d["sum_omega"], rel_tol=1e-13)
    assert math.isclose(float(got["r_omega"]), d["r_omega"], rel_tol=1e-13)
    assert math.isclose(float(got["kappa1"]), d["kappa"][0], rel_tol=1e-12, abs_tol=1e-15)
    assert math.isclose(float(got["kappa2"]), d["kappa"][1], rel_tol=1e-12, abs_tol=1e-15)
    for q in (1, 2):
        assert 4 <= int(got["sl_transpose_width_%d" % (q - 1)]) <= 8
