"""Host side of the price-space plan through the C ABI (lpide_ps_discretize_host,
no device touched) against the oracle's price-space module: the grid, the
y-grid sizes with the 7-smooth shift N_y^*, the weights, kappa_omega, r_omega,
the small-jump covariance and the cell-averaged pay-off, on the Table 1 sets
with the grids of Sec. 4; and the validation errors."""

import csv
import os

import numpy as np
import pytest

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
PRINTED_C = {"VG0": 21.6164, "VG1": 67.1487, "NIG0": 55.0673, "NIG1": 45.0189}     # Sec. 4
X_MAX = {"VG0": 5700.0, "VG1": 500.0, "NIG0": 600.0, "NIG1": 700.0}                 # Sec. 4


def _params(name):
    with open(os.path.join(GOLD, "table1_params.csv")) as f:
        rows = list(csv.DictReader(line for line in f if not line.startswith("#")))
    return {q["name"]: q for q in rows}[name]


@pytest.fixture(scope="module")
def lp():
    import paper_2511_02700_amd as m
    m.lib()
    return m


@pytest.mark.parametrize("name,N_x,payoff", [("VG1", 24, "put_avg"), ("NIG1", 16, "put_avg"), ("VG0", 20, "put_1"),
                                             ("NIG0", 12, "put_avg")])
def test_ps_discretization_matches_oracle(lp, name, N_x, payoff):
    from oracle import levy
    from oracle import price_space as ps
    q = _params(name)
    eta = (float(q["eta1"]), float(q["eta2"]))
    lv = lp.levy_nts(float(q["alpha"]), float(q["delta"]), float(q["lambda"]), eta,
                     (float(q["rho11"]), float(q["rho12"]), float(q["rho22"])), float(q["r"]))
    pay = lp.make_payoff(payoff, float(q["K"]), float(q["T"]))
    info, x, v0, om = lp.ps_discretize_host(lp.make_ps_grid(N_x, X_MAX[name], c=PRINTED_C[name]), lv, pay,
                                            want_v0=True, want_omega=True)
    p = levy.nts_params(float(q["alpha"]), float(q["delta"]), float(q["lambda"]), eta,
                        ((float(q["rho11"]), float(q["rho12"])), (float(q["rho12"]), float(q["rho22"]))))
    prob = ps.PriceSpaceProblem(p, N_x, float(q["K"]), X_MAX[name], float(q["T"]), N_x // 2, float(q["r"]),
                                payoff=payoff, c=PRINTED_C[name])
    assert np.max(np.abs(x - prob.x)) <= 1e-12 * prob.x_max
    assert (info["N_z"], info["n_in"], info["N_ym"], info["N_yp"], info["N_ystar"]) == (
        prob.N_z, prob.n_in, prob.N_ym, prob.N_yp, prob.N_ystar)
    assert info["n_out"] == len(prob.y_out)
    assert info["h_z"] == pytest.approx(prob.h_z, rel=1e-12)
    assert np.max(np.abs(om - prob.W)) <= 1e-13 * np.max(np.abs(prob.W))
    assert np.allclose(info["kappa"], prob.kappa, rtol=0, atol=1e-13)
    assert info["r_omega"] == pytest.approx(prob.r_omega, rel=1e-13)
    assert np.allclose(info["S"], [prob.S[0, 0], prob.S[0, 1], prob.S[1, 1]], rtol=1e-10, atol=1e-15)
    assert np.max(np.abs(v0 - prob.V0())) < 1e-13 * prob.K
    # the y^in nodes inside [0, x_max]: the rows of T^in that are not zero
    assert info["n_nz"] == int(np.count_nonzero(prob.y_in <= prob.x_max))


def test_ps_grid_constant_from_the_relation(lp):
    """c = 0 asks for the root of the relation for F: the nodes then put a
    fraction F of themselves in [0, x_int], as the oracle's root does."""
    from oracle import price_space as ps
    lv = lp.levy_black_scholes(0.0, (0.04, 0.0, 0.04))
    info, x, _, _ = lp.ps_discretize_host(lp.make_ps_grid(400, 500.0), lv, lp.make_payoff("put_avg", 100.0, 1.0))
    xo, c = ps.x_grid(400, 100.0, 500.0)
    assert info["c"] == pytest.approx(c, rel=1e-10)
    assert np.max(np.abs(x - xo)) < 1e-9
    assert abs(np.count_nonzero(x <= 250.0) / 401 - 0.65) < 2.0 / 400


def test_ps_validation(lp):
    lv = lp.levy_black_scholes(0.0, (0.04, 0.0, 0.04))
    pay = lp.make_payoff("put_avg", 100.0, 1.0)
    for bad in (dict(N_x=4), dict(x_max=200.0), dict(fraction=1.5), dict(nz_per_nx=0)):
        g = lp.make_ps_grid(32, 500.0)
        for k, v in bad.items():
            setattr(g, k, v)
        with pytest.raises(lp.LpideError):
            lp.ps_discretize_host(g, lv, pay)
    with pytest.raises(lp.LpideError):
        lp.ps_discretize_host(lp.make_ps_grid(32, 500.0), lv, lp.make_payoff("exchange", 100.0, 1.0), want_v0=True)


def test_accel_option_validated_before_any_device_work(lp):
    """lpide_opts.accel: the price-space plan takes -1 (automatic), 0 (the
    paper's iteration) or an Anderson depth 1..6 and refuses anything else;
    the log plan refuses any value but 0.  Both are checked before a device is
    touched, so the refusal is seen here."""
    import ctypes as C
    from paper_2511_02700_amd import _lib as L
    lib = L.lib()
    lv = lp.levy_black_scholes(0.0, (0.04, 0.0, 0.04))
    pay = lp.make_payoff("put_avg", 100.0, 1.0)
    g = lp.make_ps_grid(32, 500.0)
    for bad in (-2, 7, 100):
        o = L.Opts()
        lib.lpide_opts_default(C.byref(o))
        o.accel = bad
        h = C.c_void_p()
        rc = lib.lpide_ps_plan_create(C.byref(g), C.byref(lv), C.byref(pay), 0.5, 16, C.byref(o), C.byref(h))
        assert L.ERRORS.get(rc) == "LPIDE_E_PARAM" and not h.value
        assert b"accel" in lib.lpide_last_error()
    o = L.Opts()
    lib.lpide_opts_default(C.byref(o))
    assert o.accel == 0                   # the default is the paper's iteration
    o.accel = 4
    lg = lp.make_grid(32, -2.0, 2.0)
    h = C.c_void_p()
    rc = lib.lpide_plan_create(C.byref(lg), C.byref(lv), C.byref(pay), 0.5, 8, C.byref(o), C.byref(h))
    assert L.ERRORS.get(rc) == "LPIDE_E_PARAM" and not h.value
    assert b"accel" in lib.lpide_last_error()
