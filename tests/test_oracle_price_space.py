"""Pins of the oracle's price-space discretization (oracle/price_space.py, the
paper's own grid and operators, Sec. 3.2, 3.3 and the Sec. 4 settings)
against what the paper and the mathematics fix: grid structure, exactness of
the difference and interpolation formulas on polynomials, the summation
operator on constants and linear functions (the e^z geometry of the y grids),
direct sum = FFT, the 7-smooth side, closed-form cell averages, the
Black-Scholes limit, and the paper's Table 3 prices reached at second order
under refinement.
"""

import csv
import math
import os

import numpy as np
import pytest

from oracle import levy
from oracle import price_space as ps

GOLD = os.path.join(os.path.dirname(__file__), "golden")
PRINTED_C = {"VG0": 21.6164, "VG1": 67.1487, "NIG0": 55.0673, "NIG1": 45.0189}     # Sec. 4
X_MAX = {"VG0": 5700.0, "VG1": 500.0, "NIG0": 600.0, "NIG1": 700.0}                 # Sec. 4


def _rows(name):
    with open(os.path.join(GOLD, name)) as f:
        return list(csv.DictReader(line for line in f if not line.startswith("#")))


def _table1(name):
    r = {q["name"]: q for q in _rows("table1_params.csv")}[name]
    p = levy.nts_params(float(r["alpha"]), float(r["delta"]), float(r["lambda"]), (float(r["eta1"]), float(r["eta2"])),
                        ((float(r["rho11"]), float(r["rho12"])), (float(r["rho12"]), float(r["rho22"]))))
    return p, float(r["r"]), float(r["T"]), float(r["K"])


def test_grid_structure():
    """Uniform on [0, x_int] with x_int = 5K/2, graded (increasing spacing)
    beyond, x_N = x_max; the fraction of nodes in [0, x_int] tends to F."""
    for N in (50, 400, 4000):
        x, c = ps.x_grid(N, 100.0, 500.0)
        h = np.diff(x)
        inner = x[1:] <= 250.0 + 1e-9
        assert x[0] == 0.0 and x[-1] == 500.0 and np.all(h > 0)
        assert np.allclose(h[inner], h[0], rtol=1e-12)
        assert np.all(np.diff(h[~inner][1:]) > 0)
        frac = np.count_nonzero(x <= 250.0) / (N + 1)
        assert abs(frac - 0.65) < 2.0 / N
    assert ps.fraction_in_uniform_part(ps.c_for_fraction(250.0, 500.0, 0.65), 250.0, 500.0) == pytest.approx(0.65,
                                                                                                            rel=1e-13)


def test_printed_c_values_nearly_satisfy_the_relation():
    """Sec. 4 prints c for each parameter set; with x_int = 5K/2 and the printed
    x_max they give F within 1.6% of 65% (the stated target), and the exact
    roots lie within 7% of them (reading P5: the oracle uses the printed c
    where it reproduces the paper's runs)."""
    for name, c in PRINTED_C.items():
        F = ps.fraction_in_uniform_part(c, 250.0, X_MAX[name])
        assert abs(F - 0.65) < 0.016, (name, F)
        assert abs(ps.c_for_fraction(250.0, X_MAX[name], 0.65) / c - 1.0) < 0.07


def test_seven_smooth_side():
    """#in = N_y^- + N_y^+ + 2 N_z has no prime factor above 7, and N_y^* is the
    least such shift; y^out covers [x_1, x_max]."""
    p, r, T, K = _table1("VG1")
    prob = ps.PriceSpaceProblem(p, 40, K, 500.0, T, 20, r, c=PRINTED_C["VG1"])
    assert ps.largest_prime_factor(prob.n_in) <= 7
    base = prob.n_in - 2 * prob.N_ystar
    assert all(ps.largest_prime_factor(base + 2 * s) > 7 for s in range(prob.N_ystar))
    assert prob.y_out[0] <= prob.x[1] and prob.y_out[-1] >= prob.x[-1]
    assert len(prob.y_in) == prob.n_in and len(prob.y_out) == prob.n_in - 2 * prob.N_z + 1


def test_diffusion_exact_on_quadratics():
    """Three-point formulas on a nonuniform grid are exact for quadratics:
    D u = 1/2 a11 x1^2 u_11 + a12 x1 x2 u_12 + 1/2 a22 x2^2 u_22 away from x_max."""
    x, _ = ps.x_grid(30, 100.0, 500.0)
    a = np.array([[0.04, 0.012], [0.012, 0.09]])
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    u = 3.0 + 0.5 * X1 - 0.2 * X2 + 1e-3 * X1 ** 2 - 2e-3 * X1 * X2 + 3e-3 * X2 ** 2
    want = 0.5 * a[0, 0] * X1 ** 2 * 2e-3 + a[0, 1] * X1 * X2 * (-2e-3) + 0.5 * a[1, 1] * X2 ** 2 * 6e-3
    got = (ps.build_D(x, a) @ u.ravel()).reshape(u.shape)
    # exact on every node off the x_max rows (where v is taken linear); on the
    # x_i = 0 rows only the derivatives in x_i vanish, as the x factors do
    sl = slice(0, -1)
    assert np.allclose(got[sl, sl], want[sl, sl], rtol=1e-10, atol=1e-10)
    assert got[0, 0] == 0.0 and np.max(np.abs(got[0, 1:-1])) > 0.0


def test_interpolation_exact_on_cubics():
    x, _ = ps.x_grid(25, 100.0, 600.0)
    t = np.linspace(0.0, 600.0 * math.exp(0.01), 77)
    f = lambda s: 2.0 - s + 1e-3 * s * s - 1e-6 * s ** 3
    got = ps.interp_matrix(x, t) @ f(x)
    assert np.allclose(got, f(t), rtol=1e-11, atol=1e-9)


@pytest.fixture(scope="module")
def vg1_small():
    p, r, T, K = _table1("VG1")
    return ps.PriceSpaceProblem(p, 32, K, 500.0, T, 16, r, c=PRINTED_C["VG1"])


def test_summation_direct_equals_fft(vg1_small):
    """The direct correlation sum and the FFT agree within the FFT's rounding
    bound (a few eps log2(n) sum|omega| max|v^in|), amplified on the x = 0 rows
    by the linear extrapolation there (coefficients about 1/h_z per axis)."""
    prob = vg1_small
    V = np.random.default_rng(3).standard_normal((33, 33))
    a = prob.B(V, "direct")
    b = prob.B(V, "fft")
    vin = (prob.T_in @ (prob.T_in @ V).T).T
    t_out = float(np.max(np.abs(prob.T_out).sum(axis=1)))
    bound = 8 * np.finfo(float).eps * math.log2(prob.n_in ** 2) * np.abs(prob.W).sum() * np.abs(vin).max()
    assert np.max(np.abs(a - b)) < bound * t_out ** 2
    assert np.max(np.abs(a - b)[1:, 1:]) < bound * 4.0                 # no extrapolation off the x = 0 rows


def test_summation_on_constants_and_linear_functions(vg1_small):
    """Where every y^in sample stays inside [0, x_max], B 1 = sum omega and
    B x_1 = x_1 sum_l omega_l e^{z_l^(1)} (the interpolations reproduce linear
    functions, x e^{z_l} = y^in_{m+l}); at x = 0 the linear extrapolation gives
    B x_1 = 0.  A shift of the y grids by one node or half a cell fails this."""
    prob = vg1_small
    x = prob.x
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    l = (np.arange(-prob.N_z, prob.N_z) + 0.5) * prob.h_z
    s0 = prob.W.sum()
    s1 = np.sum(prob.W * np.exp(l)[:, None])
    ok = x <= prob.x_max * math.exp(-prob.N_z * prob.h_z - 4 * prob.h_z) * 0.95
    sel = np.ix_(ok, ok)
    assert ok.sum() >= 5
    B1 = prob.B(np.ones_like(X1))
    assert np.allclose(B1[sel], s0, rtol=1e-11)
    Bx = prob.B(X1)
    assert np.allclose(Bx[sel], X1[sel] * s1, rtol=1e-9, atol=1e-9)
    assert np.all(np.abs(Bx[0, :][ok]) < 1e-9)


def _clip_below_line(poly, c):
    """The part of a convex polygon with x + y <= c (one half-plane clip)."""
    out = []
    for (x0, y0), (x1, y1) in zip(poly, poly[1:] + poly[:1]):
        f0, f1 = x0 + y0 - c, x1 + y1 - c
        if f0 <= 0:
            out.append((x0, y0))
        if f0 * f1 < 0:
            t = f0 / (f0 - f1)
            out.append((x0 + t * (x1 - x0), y0 + t * (y1 - y0)))
    return out


def test_cell_average_put_avg_vs_polygon():
    """The pay-off is linear where it is positive, so its cell integral is the
    area of {x1 + x2 <= 2K} inside the cell times the pay-off at that polygon's
    centroid (shoelace formulas), independent of the oracle's quadrature."""
    K = 100.0
    for a1, b1, a2, b2 in ((95.0, 103.0, 96.0, 101.5), (99.0, 100.5, 99.2, 101.1), (60.0, 140.0, 90.0, 120.0),
                           (40.0, 60.0, 70.0, 90.0), (120.0, 130.0, 95.0, 99.0)):
        # local coordinates u = x1 - a1, v = x2 - a2 keep the shoelace sums free of cancellation
        P = _clip_below_line([(0.0, 0.0), (b1 - a1, 0.0), (b1 - a1, b2 - a2), (0.0, b2 - a2)], 2.0 * K - a1 - a2)
        area = cx = cy = 0.0
        for (x0, y0), (x1, y1) in zip(P, P[1:] + P[:1]):
            cr = x0 * y1 - x1 * y0
            area += 0.5 * cr
            cx += (x0 + x1) * cr / 6.0
            cy += (y0 + y1) * cr / 6.0
        ref = 0.0 if area == 0.0 else area * (K - 0.5 * (a1 + a2) - 0.5 * (cx + cy) / area) / ((b1 - a1) * (b2 - a2))
        got = ps._cell_avg_put_avg(K, a1, b1, a2, b2)
        assert got == pytest.approx(ref, rel=1e-13, abs=1e-13), (a1, b1, a2, b2)


def test_black_scholes_put_price_space():
    """Zero Levy measure, Brownian covariance, put on asset 1: the price-space
    march converges to the Black-Scholes price at second order."""
    from closed_forms import bs_put
    s1, s2, c = 0.25, 0.2, 0.4
    cov = np.array([[s1 * s1, c * s1 * s2], [c * s1 * s2, s2 * s2]])
    errs = []
    for N in (32, 64):
        prob = ps.PriceSpaceProblem(None, N, 100.0, 500.0, 1.0, N // 2, 0.03, payoff="put_1", sigma_bs=cov)
        V, _ = ps.solve(prob, tol=1e-12)
        P = prob.prices(V, [(100.0, 100.0), (90.0, 110.0)])
        errs.append(max(abs(P[0] - bs_put(100, 100, 1, 0.03, s1)), abs(P[1] - bs_put(90, 100, 1, 0.03, s1))))
    assert errs[1] < 2e-2 and math.log2(errs[0] / errs[1]) > 1.7, errs


@pytest.mark.parametrize("name", ["VG1", "NIG1"])
def test_table3_reached_at_second_order(name):
    """The paper's printed grid (x_max, c of Sec. 4) with N_x = 32 and 64:
    the nine prices of Table 3 (N_x = 800 in the paper) are approached at an
    observed order of at least 1.8.  Measured: VG1 0.28 -> 0.070 -> 0.016 at
    N_x = 32, 64, 128; NIG1 0.095 -> 0.026 -> 0.0040."""
    p, r, T, K = _table1(name)
    gold = _rows("table3_prices.csv")
    spots = [(float(g["x1"]), float(g["x2"])) for g in gold]
    want = np.array([float(g[name]) for g in gold])
    errs = []
    for N in (32, 64):
        prob = ps.PriceSpaceProblem(p, N, K, X_MAX[name], T, N // 2, r, c=PRINTED_C[name])
        V, _ = ps.solve(prob, tol=1e-10)
        errs.append(float(np.max(np.abs(prob.prices(V, spots) - want))))
    assert errs[1] < 0.08 and math.log2(errs[0] / errs[1]) > 1.8, errs


def test_greeks_exact_on_quadratics():
    """The Greek stencils are those of D (Sec. 3.2.1): exact for quadratics at
    the inner nodes; on the x_i = 0 rows the derivatives in x_i are zero by the
    scheme's convention, on the x_max rows Gamma in x_i is zero and Delta is the
    backward difference (exact for the linear part)."""
    x, _ = ps.x_grid(30, 100.0, 500.0)
    X1, X2 = np.meshgrid(x, x, indexing="ij")
    u = 3.0 + 0.5 * X1 - 0.2 * X2 + 1e-3 * X1 ** 2 - 2e-3 * X1 * X2 + 3e-3 * X2 ** 2
    d1, d2, g11, g12, g22 = ps.greeks(x, u)
    inner = (slice(1, -1), slice(1, -1))
    assert np.allclose(d1[inner], (0.5 + 2e-3 * X1 - 2e-3 * X2)[inner], rtol=1e-10, atol=1e-10)
    assert np.allclose(d2[inner], (-0.2 - 2e-3 * X1 + 6e-3 * X2)[inner], rtol=1e-10, atol=1e-10)
    assert np.allclose(g11[inner], 2e-3, rtol=1e-9) and np.allclose(g22[inner], 6e-3, rtol=1e-9)
    assert np.allclose(g12[inner], -2e-3, rtol=1e-9)
    assert np.all(d1[0, :] == 0.0) and np.all(g11[0, :] == 0.0) and np.all(g11[-1, :] == 0.0)
    lin = 3.0 + 0.5 * X1 - 0.2 * X2
    assert np.allclose(ps.greeks(x, lin)[0][-1, :], 0.5, rtol=1e-12)


def test_greeks_black_scholes_put_price_space():
    """Zero Levy measure, put on asset 1: Delta_1 and Gamma_11 of the price-space
    march at the nodes near the money approach the Black-Scholes put Delta and
    Gamma at second order (and do not depend on x_2).  Measured: Delta 6.1e-3,
    1.5e-3, 3.7e-4 and Gamma 1.6e-4, 3.9e-5, 1.2e-5 at N_x = 32, 64, 128."""
    from closed_forms import bs_put_delta_gamma
    s1 = 0.25
    cov = np.array([[s1 * s1, 0.02], [0.02, 0.04]])
    errs = []
    for N in (32, 64):
        prob = ps.PriceSpaceProblem(None, N, 100.0, 500.0, 1.0, N // 2, 0.03, payoff="put_1", sigma_bs=cov)
        V, _ = ps.solve(prob, tol=1e-12)
        d1, _, g11, _, _ = ps.greeks(prob.x, V)
        sel = [m for m in range(len(prob.x)) if 80.0 <= prob.x[m] <= 125.0]
        e = 0.0
        for m in sel:
            dlt, gam = bs_put_delta_gamma(prob.x[m], 100.0, 1.0, 0.03, s1)
            e = max(e, abs(d1[m, 5] - dlt), 100.0 * abs(g11[m, 5] - gam))
            assert np.allclose(d1[m, 1:-1], d1[m, 5], rtol=0, atol=1e-9)
        errs.append(e)
    assert errs[1] < 5e-3 and math.log2(errs[0] / errs[1]) > 1.7, errs
