"""The paper's own discretization in price space -- oracle side (test
infrastructure only; see the package docstring).

The log-moneyness modules (``scheme``, ``output``) restate the method on a
uniform grid in y = ln(S/K).  This module restates it as the paper computes it
(Sec. 3.2, Sec. 3.3, Sec. 4 settings), on a graded grid in the prices
themselves:

* the x grid: x_m = phi(xi_max m / N_x) per axis with the piecewise linear /
  sinh map phi (uniform on [0, x_int], graded beyond) and the constant c chosen
  so that the fraction F of the points in [0, x_int] is max(65%, x_int/x_max);
* D: second-order central differences on the nonuniform grid, no derivative
  terms at x = 0, no second derivative and a backward first difference at
  x_max, assembled as Kronecker products with the diagonal x factors;
* B_omega = T^out I~ C T^in: cubic interpolation from the x grid to the
  log-uniform grid y^in (zero outside [0, x_max]^2), the correlation with the
  weights omega on the y grids (by FFT, or by direct sum), cubic interpolation
  back from y^out to the x grid, linear extrapolation at x = 0;
* N_y^-, N_y^+ from x_1 and x_max, and the least N_y^* that makes the side
  N_y^- + N_y^+ + 2 N_z a 7-smooth number;
* the semi-Lagrangian theta-method with departure points x e^{kappa h_t},
  the damped start, extrapolated start values and the fixed-point iteration
  of Algorithm 1 (exact sparse LU for the implicit systems);
* cell averages of the pay-off on the cells [x_{m-1/2}, x_{m+1/2}]^2 that meet
  its kink.

Readings taken where the paper is silent (also listed in the design doc):
P1 interpolation (T^in, T^out, T^SL, prices off the grid) is cubic Lagrange in
   the price variable on the four nearest nodes of the respective grid, the
   stencil clamped to the grid's ends (polynomial extrapolation beyond them,
   except the linear extrapolation to x = 0 that Sec. 4 prescribes for T^out);
P2 N_y^* is the least non-negative integer with the 7-smooth property;
P3 z_max^III is the level-1e-14 maximum (the printed values; reading A2) and
   h_z = z_max^III / N_z with N_z = 2 N_x (Sec. 4 settings);
P4 the regions R_I, R_II, R_III and the weights follow the log-grid oracle
   (``integral``) with this h_z: the weights do not depend on the x grid;
P5 the constant c of the grid: the root of the stated relation for F, unless
   given (the printed values give F between 0.640 and 0.650 instead of 0.65).
"""

import math

import numpy as np
import scipy.optimize as so
import scipy.signal as ssig
import scipy.sparse as ssp
import scipy.sparse.linalg as sla

from . import integral
from .scheme import extrapolated_start, step_list


# --------------------------------------------------------------------------- #
# x grid (Sec. 4: the map phi and the constant c)
# --------------------------------------------------------------------------- #
def fraction_in_uniform_part(c, x_int, x_max):
    """F = xi_int / xi_max: the limit fraction of points in [0, x_int] (Sec. 4)."""
    return 1.0 / (1.0 + (c / x_int) * math.asinh((x_max - x_int) / c))


def c_for_fraction(x_int, x_max, F):
    """The c > 0 with fraction_in_uniform_part(c) = F; F decreases from 1 to
    x_int / x_max as c grows, so the root is unique for x_int/x_max < F < 1."""
    f = lambda c: fraction_in_uniform_part(c, x_int, x_max) - F
    return so.brentq(f, 1e-9 * x_max, 1e9 * x_max, xtol=1e-14 * x_max, rtol=1e-15, maxiter=500)


def x_grid(N_x, K, x_max, fraction=0.65, c=None):
    """Nodes x_0 = 0 < ... < x_N = x_max and the constant c (inf: uniform grid):
    x_int = 5K/2, F = max(fraction, x_int/x_max) (Sec. 4).  A given c is used
    as it is (the values printed in Sec. 4 satisfy the relation for F only to
    about 1.5%, reading P5); otherwise c is its root."""
    x_int = 2.5 * K
    F = max(fraction, x_int / x_max)
    if c is None and F <= x_int / x_max:
        return np.linspace(0.0, x_max, N_x + 1), math.inf
    if c is None:
        c = c_for_fraction(x_int, x_max, F)
    xi_int = x_int / c
    xi_max = xi_int + math.asinh((x_max - x_int) / c)
    xi = xi_max * np.arange(N_x + 1) / N_x
    x = np.where(xi <= xi_int, c * xi, x_int + c * np.sinh(xi - xi_int))
    x[-1] = x_max
    return x, c


# --------------------------------------------------------------------------- #
# Diffusion matrix D (Sec. 3.2.1)
# --------------------------------------------------------------------------- #
def fd_matrices(x):
    """First- and second-derivative matrices D1, D2 on the nonuniform grid x:
    central three-point formulas inside; row 0 zero (both derivative terms
    vanish at x = 0); at x_max no second derivative and the backward first
    difference (v linear in x there)."""
    n = len(x)
    hx = np.diff(x)                      # hx[m-1] = x_m - x_{m-1}
    D1 = ssp.lil_matrix((n, n))
    D2 = ssp.lil_matrix((n, n))
    for m in range(1, n - 1):
        hm, hp = hx[m - 1], hx[m]
        D1[m, m - 1] = -hp / (hm * (hm + hp))
        D1[m, m] = (hp - hm) / (hm * hp)
        D1[m, m + 1] = hm / (hp * (hm + hp))
        D2[m, m - 1] = 2.0 / (hm * (hm + hp))
        D2[m, m] = -2.0 / (hm * hp)
        D2[m, m + 1] = 2.0 / (hp * (hm + hp))
    D1[n - 1, n - 2] = -1.0 / hx[-1]
    D1[n - 1, n - 1] = 1.0 / hx[-1]
    return D1.tocsr(), D2.tocsr()


def build_D(x, a):
    """D = 1/2 a11 X^2 D2 (axis 1) + a12 (X D1) (x) (X D1) + 1/2 a22 X^2 D2 (axis 2)
    on V[m1, m2] flattened row-major (m1 slow), a = sigma_omega sigma_omega^T."""
    n = len(x)
    D1, D2 = fd_matrices(x)
    X = ssp.diags(x)
    I = ssp.identity(n, format="csr")
    A1, A2 = X @ D1, X @ X @ D2
    return (0.5 * a[0, 0] * ssp.kron(A2, I) + a[0, 1] * ssp.kron(A1, A1) + 0.5 * a[1, 1] * ssp.kron(I, A2)).tocsr()


# --------------------------------------------------------------------------- #
# Interpolation (reading P1)
# --------------------------------------------------------------------------- #
def lagrange_row(nodes, t, P=3):
    """Stencil start s and the P+1 Lagrange weights of t on nodes[s..s+P]: the
    P+1 nodes nearest to t in index order, clamped to the ends of the grid."""
    n = len(nodes)
    j = int(np.searchsorted(nodes, t, side="right")) - 1   # nodes[j] <= t < nodes[j + 1]
    s = min(max(j - (P - 1) // 2, 0), n - 1 - P)
    pts = nodes[s:s + P + 1]
    w = np.empty(P + 1)
    for i in range(P + 1):
        v = 1.0
        for k in range(P + 1):
            if k != i:
                v *= (t - pts[k]) / (pts[i] - pts[k])
        w[i] = v
    return s, w


def interp_matrix(nodes, targets, P=3, zero_above=None):
    """Sparse matrix of cubic interpolation from values on `nodes` to `targets`
    (rows of targets above zero_above are zero: v = 0 outside R_x)."""
    rows, cols, vals = [], [], []
    for r, t in enumerate(targets):
        if zero_above is not None and t > zero_above:
            continue
        s, w = lagrange_row(nodes, t, P)
        rows += [r] * (P + 1)
        cols += list(range(s, s + P + 1))
        vals += list(w)
    return ssp.csr_matrix((vals, (rows, cols)), shape=(len(targets), len(nodes)))


# --------------------------------------------------------------------------- #
# Summation term B_omega (Sec. 3.2.2, Sec. 4 settings)
# --------------------------------------------------------------------------- #
def largest_prime_factor(m):
    p, f = 2, 1
    while m > 1:
        while m % p == 0:
            f, m = p, m // p
        p += 1
    return f


def y_sizes(x1, x_max, h_z, N_z):
    """N_y^-, N_y^+ and N_y^* (Sec. 4): N_y^- = ceil(-ln x_1 / h_z) + N_y^*,
    N_y^+ = ceil(ln x_max / h_z) + N_y^*, N_y^* the least with a 7-smooth
    #in = N_y^- + N_y^+ + 2 N_z (reading P2)."""
    base_m = math.ceil(-math.log(x1) / h_z)
    base_p = math.ceil(math.log(x_max) / h_z)
    star = 0
    while largest_prime_factor(base_m + base_p + 2 * N_z + 2 * star) > 7:
        star += 1
    return base_m + star, base_p + star, star


class PriceSpaceProblem:
    """Everything Algorithm 1 needs on the paper's price-space grid.

    model: output of levy.nts_params / levy.nts_from_std (None: zero Levy
    measure); sigma_bs: Brownian covariance; payoff "put_avg" or "put_1".
    """

    def __init__(self, model, N_x, K, x_max, T, N_t, r, payoff="put_avg", theta=0.5, sigma_bs=None,
                 damping=True, ell_cut=1e-14, frac2=math.sqrt(0.1), m1=2, ng=8, fraction=0.65, c=None):
        self.N_x, self.K, self.x_max, self.T, self.N_t, self.r = int(N_x), float(K), float(x_max), float(T), \
            int(N_t), float(r)
        self.payoff, self.theta, self.damping = payoff, float(theta), bool(damping)
        self.x, self.c = x_grid(self.N_x, self.K, self.x_max, fraction, c)
        sbs = np.zeros((2, 2)) if sigma_bs is None else np.asarray(sigma_bs, dtype=np.float64)
        if model is None:
            self.N_z, self.h_z, self.W, self.S = 0, 0.0, np.zeros((0, 0)), np.zeros((2, 2))
            self.kappa, self.r_omega, self.sum_omega, self.z_star = np.array([r, r]), r, 0.0, 0.0
        else:
            self.z_star = integral.z_star(model, ell_cut)
            self.N_z = 2 * self.N_x                                   # Sec. 4: N_z = 2 N_x
            self.h_z = self.z_star / self.N_z                         # h_z = z_max^III / N_z
            M2 = int(math.ceil(frac2 * self.N_z - 0.5))               # z_max^II = h_z ceil(...)
            self.W = integral.weights(model, self.h_z, self.N_z, m1, M2, ng)
            self.S = integral.small_jump_cov(model, self.h_z, m1)
            self.kappa, self.r_omega, self.sum_omega = integral.drift_and_rate(self.W, self.h_z, self.N_z, r)
        self.a = sbs + self.S                                         # sigma_omega sigma_omega^T
        if self.N_z:
            self.N_ym, self.N_yp, self.N_ystar = y_sizes(self.x[1], self.x_max, self.h_z, self.N_z)
            m_out = np.arange(-self.N_ym, self.N_yp + 1)
            m_in = np.arange(-self.N_z - self.N_ym, self.N_z + self.N_yp)
            self.y_out = np.exp(m_out * self.h_z)
            self.y_in = np.exp((m_in + 0.5) * self.h_z)
            self.T_in = interp_matrix(self.x, self.y_in, zero_above=self.x_max)
            self.T_out = self._t_out()

    @property
    def n_in(self):
        return self.N_ym + self.N_yp + 2 * self.N_z

    def _t_out(self):
        """Cubic interpolation from y^out to the x nodes; x_0 = 0 lies below
        y^out and is extrapolated linearly from its first two nodes (Sec. 4)."""
        M = interp_matrix(self.y_out, self.x).tolil()
        y0, y1 = self.y_out[0], self.y_out[1]
        M[0, :] = 0.0
        M[0, 0] = (y1 - 0.0) / (y1 - y0)
        M[0, 1] = (0.0 - y0) / (y1 - y0)
        return M.tocsr()

    def B(self, V, method="fft"):
        """B_omega V = T^out I~ C T^in V on the (N_x+1)^2 grid V[m1, m2]."""
        if not self.N_z:
            return np.zeros_like(V)
        vin = (self.T_in @ (self.T_in @ V).T).T                       # T_in V T_in^T on y^in
        # (C v)_m = sum_l omega_l v^in_{m+l} on the y^out nodes: the "valid" part
        # of the correlation (the rows I~ keeps), by FFT or by direct sum
        if method == "direct":
            out = ssig.correlate2d(vin, self.W, mode="valid")
        else:
            out = ssig.fftconvolve(vin, self.W[::-1, ::-1], mode="valid")
        return (self.T_out @ (self.T_out @ out).T).T                 # T_out out T_out^T

    def D(self):
        return build_D(self.x, self.a)

    def sl_matrix(self, dt):
        """T^SL: interpolation at the departure points x_m e^{kappa_omega^(i) dt} (Sec. 3.3)."""
        T1 = interp_matrix(self.x, self.x * math.exp(self.kappa[0] * dt))
        T2 = interp_matrix(self.x, self.x * math.exp(self.kappa[1] * dt))
        return ssp.kron(T1, T2).tocsr()

    def V0(self):
        """Pay-off at the nodes, cell averaged on the cells that meet its kink (Sec. 3.2.3)."""
        x, K = self.x, self.K
        xm = np.empty(len(x) + 1)                                     # x_{m - 1/2}, m = 0..N_x+1
        xm[1:-1] = 0.5 * (x[1:] + x[:-1])
        xm[0] = -xm[1]
        xm[-1] = 2.0 * x[-1] - xm[-2]
        X1, X2 = np.meshgrid(x, x, indexing="ij")
        if self.payoff == "put_avg":
            V = np.maximum(K - 0.5 * (X1 + X2), 0.0)
            for i in range(len(x)):
                for j in range(len(x)):
                    a1, b1, a2, b2 = xm[i], xm[i + 1], xm[j], xm[j + 1]
                    if a1 + a2 < 2 * K < b1 + b2:
                        V[i, j] = _cell_avg_put_avg(K, a1, b1, a2, b2)
        elif self.payoff == "put_1":
            V = np.maximum(K - X1, 0.0) + 0.0 * X2
            for i in range(len(x)):
                a1, b1 = xm[i], xm[i + 1]
                if a1 < K < b1:
                    V[i, :] = 0.5 * (K - a1) ** 2 / (b1 - a1)
        else:
            raise ValueError(self.payoff)
        return V

    def prices(self, V, spots):
        """Cubic interpolation of V at spot pairs (Sec. 4, reading P1)."""
        out = []
        for s1, s2 in np.asarray(spots, dtype=np.float64).reshape(-1, 2):
            a, w1 = lagrange_row(self.x, s1)
            b, w2 = lagrange_row(self.x, s2)
            out.append(w1 @ V[a:a + 4, b:b + 4] @ w2)
        return np.array(out)


def greeks(x, V):
    """Delta and Gamma surfaces on the price grid by the difference schemes of
    D (Sec. 3.2.1; the paper plots them in Sec. 4): Delta_i = D1 along axis i,
    Gamma_ii = D2 along axis i, Gamma_12 = D1 along both axes, with D1, D2 of
    fd_matrices (their rows at x = 0 and, for D2, at x_max are zero).  Returns
    (delta1, delta2, gamma11, gamma12, gamma22), each (N_x+1) x (N_x+1)."""
    D1, D2 = fd_matrices(np.asarray(x, dtype=np.float64))
    V = np.asarray(V, dtype=np.float64)
    d1 = np.asarray(D1 @ V)                       # axis 1 (rows, m1)
    d2 = np.asarray((D1 @ V.T).T)                 # axis 2 (columns, m2)
    g11 = np.asarray(D2 @ V)
    g22 = np.asarray((D2 @ V.T).T)
    g12 = np.asarray(D1 @ d2)                     # D1 along axis 1 of D1 along axis 2
    return d1, d2, g11, g12, g22


def _cell_avg_put_avg(K, a1, b1, a2, b2, nq=8):
    """(1 / cell area) * integral over [a1, b1] x [a2, b2] of max(K - (x1 + x2)/2, 0):
    the inner integral in x2 in closed form, the outer one by Gauss-Legendre on
    the pieces between the kinks x1 = 2K - b2 and x1 = 2K - a2, where the
    inner integral is a polynomial of degree two."""
    def inner(x1):
        c = K - 0.5 * x1
        up = min(b2, 2.0 * c)
        if up <= a2:
            return 0.0
        return (up - a2) * (c - 0.25 * (up + a2))                    # c (up - a2) - (up^2 - a2^2) / 4

    t, wq = np.polynomial.legendre.leggauss(nq)
    cuts = sorted({a1, b1} | {v for v in (2 * K - b2, 2 * K - a2) if a1 < v < b1})
    tot = 0.0
    for lo, hi in zip(cuts[:-1], cuts[1:]):
        xs = 0.5 * (hi - lo) * t + 0.5 * (hi + lo)
        tot += 0.5 * (hi - lo) * sum(wi * inner(xi) for wi, xi in zip(wq, xs))
    return tot / ((b1 - a1) * (b2 - a2))


def solve(prob, tol=1e-12, max_iter=200, n_steps=None):
    """Algorithm 1 on the price-space grid: returns V^{N_t} (or after the first
    n_steps entries of the step list) and the fixed-point iteration counts.
    Each step: E = V + dt (1 - theta)(D + B - r_omega) V, W = T^SL E, Y^0 by
    extrapolation over the main steps (the damped sub-steps form main step 1),
    then (I - dt theta (D - r_omega)) Y^k = dt theta B Y^{k-1} + W (sparse LU)
    until max |Y^k - Y^{k-1}| / max(1, |Y^k|) < tol."""
    n = prob.N_x + 1
    N = n * n
    D = prob.D()
    I = ssp.identity(N, format="csr")
    r_om = prob.r_omega
    steps = step_list(prob.theta, prob.T, prob.N_t, prob.damping)
    if n_steps is not None:
        steps = steps[:n_steps]
    V = prob.V0()
    hist = [V.copy()]
    cache = {}
    iters = []
    n_sub = 4 if prob.damping else 1
    for s, (th, dt) in enumerate(steps):
        if (th, dt) not in cache:
            cache[(th, dt)] = (sla.splu((I - dt * th * (D - r_om * I)).tocsc()), prob.sl_matrix(dt))
        lu, TSL = cache[(th, dt)]
        v = V.ravel()
        E = v + dt * (1.0 - th) * (D @ v - r_om * v + prob.B(V).ravel()) if th < 1.0 else v
        Wv = TSL @ E
        Y = V.ravel().copy() if (prob.damping and s < n_sub) else extrapolated_start(hist).ravel()
        prev = np.inf
        for k in range(1, max_iter + 1):
            Yn = lu.solve(dt * th * prob.B(Y.reshape(n, n)).ravel() + Wv)
            err = float(np.max(np.abs(Yn - Y) / np.maximum(1.0, np.abs(Yn))))
            Y = Yn
            if err < tol or (err < 1e-13 and err >= prev):
                break
            prev = err
        else:
            raise RuntimeError("fixed-point iteration did not converge in %d iterations" % max_iter)
        iters.append(k)
        V = Y.reshape(n, n)
        if (not prob.damping) or s >= n_sub - 1:
            hist.append(V.copy())
            if len(hist) > 4:
                hist.pop(0)
    return V, iters
