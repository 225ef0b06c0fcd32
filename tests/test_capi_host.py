"""CPU-side checks of the native library: it loads, exports every symbol that
include/lpide.h declares, and its host-side discretization (no device work)
agrees with the oracle.  No GPU compute calls are made here."""

import math
import os
import re

import numpy as np
import pytest

import workloads
from oracle import integral, levy, scheme

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    from paper_2511_02700_amd import _lib as L
    if not os.path.exists(L.LIB_PATH):
        pytest.skip("liblpide.so not built (run __graft_entry__.build())")
    return L


def test_header_symbols_exported():
    """Every function declared in include/lpide.h is exported by liblpide.so and
    bound by the Python layer."""
    L = _lib()
    text = open(os.path.join(ROOT, "include", "lpide.h")).read()
    decl = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(lpide_\w+)\s*\(", text, re.M))
    assert len(decl) >= 12
    lib = L.lib()
    for name in decl:
        assert hasattr(lib, name), name
        assert name in L.SIGNATURES, name


def _std(w):
    m = w["model"]
    return (m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])


@pytest.mark.parametrize("name", ["nig64", "fv512"])
def test_host_discretization_matches_oracle(name):
    """z-grid sizes, weights, S, kappa, r_omega from the C++ plan agree with the
    oracle's independent computation (libstdc++ vs SciPy/AMOS Bessel functions,
    tanh-sinh vs QUADPACK for S)."""
    import paper_2511_02700_amd as lp
    _lib()
    w = workloads.workload(name)
    lv = lp.levy_from_std(*_std(w), w["r"])
    g = lp.make_grid(w["n"], w["y_lo"], w["y_hi"])
    info, om, _ = lp.discretize_host(g, lv, want_omega=True)
    p = levy.nts_from_std(*_std(w))
    h = (w["y_hi"] - w["y_lo"]) / (w["n"] - 1)
    d = integral.discretize(p, h, w["r"])
    assert info["N_z"] == d["N_z"] and info["M2"] == d["M2"] and info["M1"] == d["M1"]
    assert info["z_star"] == pytest.approx(d["z_star"], rel=1e-12)
    assert np.max(np.abs(om - d["W"])) <= 1e-13 * np.max(d["W"])
    assert info["sum_omega"] == pytest.approx(d["sum_omega"], rel=1e-13)
    assert np.allclose(info["kappa"], d["kappa"], rtol=1e-12, atol=1e-15)
    assert info["r_omega"] == pytest.approx(d["r_omega"], rel=1e-13)
    S = np.array([d["S"][0, 0], d["S"][0, 1], d["S"][1, 1]])
    assert np.allclose(info["S"], S, rtol=1e-11, atol=0)
    # FFT side: no wrap-around onto the kept outputs for the cubic T^in
    # the smallest automatic transform side (2^m, or 3 * 2^m at 1536 and 3072) without wrap-around
    sides = sorted([2 ** q for q in range(6, 13)] + [1536, 3072])
    need = w["n"] + d["N_z"] + 1
    assert info["L"] == min(s for s in sides if s >= need)


@pytest.mark.parametrize("kind", ["put_avg", "call_avg", "put_1", "call_1", "exchange", "spread"])
def test_host_initial_values_match_oracle(kind):
    """Cell-averaged V^0: closed-form inner integrals (C++) vs root-split
    Gauss-Legendre (oracle)."""
    import paper_2511_02700_amd as lp
    _lib()
    n, lo, hi = 37, -1.1, 0.9
    lv = lp.levy_from_std(0.2, 0.25, 0.3, -0.1, -0.1, 0.2, 0.5, 0.03)
    g = lp.make_grid(n, lo, hi)
    _, _, v0 = lp.discretize_host(g, lv, lp.make_payoff(kind, 100.0, 1.0), want_v0=True)
    h = (hi - lo) / (n - 1)
    y = lo + h * np.arange(n)
    ref = scheme.initial_values(kind, 100.0, y, y, h, True)
    assert np.max(np.abs(v0 - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_host_parameter_validation():
    import paper_2511_02700_amd as lp
    L = _lib()
    g = lp.make_grid(64, -3, 3)
    bad = [
        lp.levy_nts(1.2, 1.0, 1.0, (0, 0), (0.04, 0.0, 0.04), 0.0),      # alpha >= 1
        lp.levy_nts(0.5, -1.0, 1.0, (0, 0), (0.04, 0.0, 0.04), 0.0),     # delta <= 0
        lp.levy_nts(0.5, 1.0, 1.0, (0, 0), (0.04, 0.05, 0.04), 0.0),     # rho not PD
        lp.levy_nts(0.5, 1.0, 0.01, (0.5, 0), (0.04, 0.0, 0.04), 0.0),   # no exponential moment
    ]
    for lv in bad:
        with pytest.raises(L.LpideError) as ei:
            lp.discretize_host(g, lv)
        assert ei.value.code == -1
    lv = lp.levy_from_std(0.2, 0.25, 0.3, -0.1, -0.1, 0.2, 0.5, 0.03)
    uneven = lp.make_grid(64, -3, 3)
    uneven.y_hi[1] = 4.0
    for gg in (lp.make_grid(4, -3, 3), lp.make_grid(64, -3, 3, sl_order=2), uneven):
        with pytest.raises(L.LpideError):
            lp.discretize_host(gg, lv)
    with pytest.raises(L.LpideError):
        lp.levy_from_std(0.2, 0.25, 1.5, -0.1, -0.1, 0.2, 0.5, 0.03)


def test_levy_from_std_matches_oracle_mapping():
    import paper_2511_02700_amd as lp
    _lib()
    for w in ("nig64", "fv512", "nts1024"):
        ww = workloads.workload(w)
        lv = lp.levy_from_std(*_std(ww), 0.0)
        p = levy.nts_from_std(*_std(ww))
        assert lv.delta == pytest.approx(p["delta"], rel=1e-14)
        assert lv.lambda_ == pytest.approx(p["lam"], rel=1e-14)
        assert list(lv.eta) == pytest.approx(list(p["eta"]))
        assert list(lv.rho) == pytest.approx([p["rho"][0, 0], p["rho"][0, 1], p["rho"][1, 1]])


def test_binding_structs_match_header(tmp_path):
    """The ctypes structures of the binding have the size of the header's C
    structures, and the timing-class list its length (a C program built with
    gcc prints sizeof of each)."""
    import ctypes as C
    import shutil
    import subprocess
    L = _lib()
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pairs = [("lpide_grid", L.Grid), ("lpide_levy", L.Levy), ("lpide_payoff", L.Payoff), ("lpide_opts", L.Opts),
             ("lpide_info", L.Info), ("lpide_adjoint_info", L.AdjInfo), ("lpide_batch_opts", L.BatchOpts),
             ("lpide_group_info", L.GroupInfo)]
    src = tmp_path / "sizes.c"
    src.write_text('#include <stdio.h>\n#include "lpide.h"\nint main(void) {\n' +
                   "".join('    printf("%%zu\\n", sizeof(%s));\n' % c for c, _ in pairs) +
                   '    printf("%d\\n", LPIDE_KCLASSES);\n    return 0;\n}\n')
    exe = tmp_path / "sizes"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    for (cname, py), size in zip(pairs, out):
        assert C.sizeof(py) == size, cname
    assert len(L.KCLASSES) == out[-1]
