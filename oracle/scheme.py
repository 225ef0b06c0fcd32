"""Spatial and temporal discretization -- oracle side (test infrastructure).

Log-moneyness form of Sec. 3.2 and Sec. 3.3 on the uniform grid
y_j = y_lo + j h (j = 0..n-1, both axes, same h), values stored row-major as
V[j1, j2].  Each function states the passage it follows and, where the paper is
silent about the log grid, the reading taken.

Coordinates.  With y_i = ln(x_i / K):
  * x_i^2 d^2/dx_i^2 = d^2/dy_i^2 - d/dy_i and x_1 x_2 d^2/dx_1 dx_2 = d^2/dy_1 dy_2,
    so the diffusion operator of Sec. 3.2.1 becomes
    1/2 a11 (d11 - d1) + a12 d12 + 1/2 a22 (d22 - d2), a = sigma_omega sigma_omega^T;
  * x (e^z - 1) jumps become shifts y -> y + z, so B_omega u(y) = sum_l omega_l u(y + z_l)
    (Sec. 3.1, summation operator), and with h_z = h the points y_m + z_l are the
    half-shifted nodes y_{m+l} + h/2, i.e. the y^in grid of Sec. 3.2.2 while the
    y^out grid is the solution grid itself (T^out = identity);
  * the characteristic x_t = -mu_omega(x) of Sec. 3.3 has departure points
    x e^{kappa h_t}, i.e. y + kappa h_t: a constant shift.
"""

import math

import numpy as np
import scipy.fft as sfft
import scipy.sparse as ssp
import scipy.sparse.linalg as sla


# --------------------------------------------------------------------------- #
# Lagrange interpolation helpers (Sec. 3.2.2 and Sec. 3.3 use Lagrange
# interpolation; Sec. 4 takes cubic polynomials)
# --------------------------------------------------------------------------- #
def lagrange_weights(nodes, x):
    """Lagrange basis values at x for the given nodes (plain product formula)."""
    nodes = [float(t) for t in nodes]
    w = []
    for i, ti in enumerate(nodes):
        v = 1.0
        for j, tj in enumerate(nodes):
            if j != i:
                v *= (x - tj) / (ti - tj)
        w.append(v)
    return np.array(w)


def lagrange_dweights(nodes, x):
    """Derivatives of the Lagrange basis at x (product rule, term by term)."""
    nodes = [float(t) for t in nodes]
    d = []
    for i, ti in enumerate(nodes):
        tot = 0.0
        for k, tk in enumerate(nodes):
            if k == i:
                continue
            v = 1.0 / (ti - tk)
            for j, tj in enumerate(nodes):
                if j != i and j != k:
                    v *= (x - tj) / (ti - tj)
            tot += v
        d.append(tot)
    return np.array(d)


def stencil_start(xi, n, P):
    """First node of the P+1 point stencil around the (fractional) index xi.

    Reading (the paper is silent on departure points outside the grid): the
    stencil is centred, floor(xi) - (P-1)/2, and clamped into [0, n-1-P], i.e.
    polynomial extrapolation near the ends.
    """
    s = int(math.floor(xi)) - (P - 1) // 2
    return min(max(s, 0), n - 1 - P)


# --------------------------------------------------------------------------- #
# Summation operator B (Sec. 3.1 summation operator, Sec. 3.2.2)
# --------------------------------------------------------------------------- #
def half_shift_taps(P):
    """Offsets j and weights of the order-P Lagrange interpolant at y_k + h/2 from
    nodes y_{k+j} (the T^in interpolation of Sec. 3.2.2 from the solution grid to
    the half-shifted y^in grid)."""
    offs = list(range(-(P - 1) // 2, (P + 1) // 2 + 1))
    return offs, lagrange_weights(offs, 0.5)


def interp_to_half_grid(v, P, N_z):
    """v^in on the half-shifted nodes k = -N_z .. n+N_z-2 of both axes, stored
    with offset N_z (entry [k1+N_z, k2+N_z]).

    Reading of "v = 0 outside the truncated domain" (Sec. 4 settings) on the log
    grid: node values outside [0, n-1] are zero on every side, both inside the
    interpolation stencil and for the summation.
    """
    n1, n2 = v.shape
    offs, w = half_shift_taps(P)
    pad = N_z + max(abs(o) for o in offs) + 1
    vp = np.zeros((n1 + 2 * pad, n2 + 2 * pad))
    vp[pad:pad + n1, pad:pad + n2] = v
    m1 = n1 + 2 * N_z - 1
    m2 = n2 + 2 * N_z - 1
    # axis 1 then axis 2 (tensor-product interpolation)
    t = np.zeros((m1, n2 + 2 * pad))
    for o, wo in zip(offs, w):
        a = pad - N_z + o
        t += wo * vp[a:a + m1, :]
    out = np.zeros((m1, m2))
    for o, wo in zip(offs, w):
        a = pad - N_z + o
        out += wo * t[:, a:a + m2]
    return out


def correlate_half_grid(vin, W, n1, n2, method="fft"):
    """out[m] = sum_{a,b} W[a, b] vin[m1 + a, m2 + b], m in [0,n1) x [0,n2): the
    cross-correlation of Sec. 3.2.2 with vin indexed from its first half-grid node
    k = -N_z (entry a of W is l = a - N_z).

    method="direct": the plain double sum over the (2 N_z)^2 weights.
    method="fft":    the same correlation through zero-padded real FFTs of a size
                     with no wrap-around onto the kept outputs (Sec. 3.2.2: the
                     circulant matrix C applied with fft, conjugate, ifft and the
                     row selection I~), computed with scipy.fft.
    """
    na, nb = W.shape
    if method == "direct":
        out = np.zeros((n1, n2))
        for a in range(na):
            for b in range(nb):
                w = W[a, b]
                if w != 0.0:
                    out += w * vin[a:a + n1, b:b + n2]
        return out
    if method != "fft":
        raise ValueError(method)
    L1 = sfft.next_fast_len(vin.shape[0], real=True)
    L2 = sfft.next_fast_len(vin.shape[1], real=True)
    Fw = sfft.rfft2(W, s=(L1, L2))
    Fv = sfft.rfft2(vin, s=(L1, L2))
    c = sfft.irfft2(np.conj(Fw) * Fv, s=(L1, L2))
    return c[:n1, :n2]


def apply_B(v, W, N_z, P=3, method="fft"):
    """(B v)_m = sum_l omega_l v^in_{m+l}, m in [0, n-1]^2: the summation operator
    over the y-grids of Sec. 3.2.2 (T^in = order-P interpolation to the
    half-shifted grid, then the cross-correlation with Omega; T^out = identity).
    The direct O(n^2 N_z^2) sum and the FFT evaluation are both available.
    """
    n1, n2 = v.shape
    if N_z == 0:
        return np.zeros_like(v)
    vin = interp_to_half_grid(v, P, N_z)
    return correlate_half_grid(vin, W, n1, n2, method)


# --------------------------------------------------------------------------- #
# Diffusion operator D (Sec. 3.2.1, matrix D as a Kronecker sum)
# --------------------------------------------------------------------------- #
def second_order_1d(n, h):
    """d^2/dy^2 - d/dy by central differences on interior nodes; zero rows at
    j = 0 and j = n-1.

    Reading of the boundary rules of Sec. 3.2.1 on the log grid: "v linear in x"
    (the rule at x_max) means x^2 v_xx = 0, i.e. (d^2/dy^2 - d/dy) v = 0, and is
    applied at both ends of the truncated log domain.
    """
    lo = np.full(n - 1, 1.0 / (h * h) + 0.5 / h)   # coefficient of v_{j-1} in row j
    di = np.full(n, -2.0 / (h * h))
    up = np.full(n - 1, 1.0 / (h * h) - 0.5 / h)   # coefficient of v_{j+1} in row j
    di[0] = di[-1] = 0.0
    up[0] = 0.0
    lo[-1] = 0.0
    return ssp.diags([lo, di, up], [-1, 0, 1], shape=(n, n), format="csr")


def first_order_1d(n, h):
    """d/dy used by the mixed term: central in the interior, first-order forward at
    j = 0 and backward at j = n-1 (Sec. 3.2.1 takes the backward scheme at the
    upper boundary; the lower log boundary mirrors it)."""
    A = ssp.lil_matrix((n, n))
    for j in range(1, n - 1):
        A[j, j - 1] = -0.5 / h
        A[j, j + 1] = 0.5 / h
    A[0, 0] = -1.0 / h
    A[0, 1] = 1.0 / h
    A[n - 1, n - 2] = -1.0 / h
    A[n - 1, n - 1] = 1.0 / h
    return A.tocsr()


def build_D(n, h, a):
    """D = 1/2 a11 (L (x) I) + a12 (G (x) G) + 1/2 a22 (I (x) L) for row-major
    V[j1, j2] (axis 1 = slow index), the log-grid form of the Kronecker-sum matrix
    D of Sec. 3.2.1, where L = second_order_1d and G = first_order_1d."""
    L = second_order_1d(n, h)
    G = first_order_1d(n, h)
    I = ssp.identity(n, format="csr")
    D = 0.5 * a[0, 0] * ssp.kron(L, I) + a[0, 1] * ssp.kron(G, G) + 0.5 * a[1, 1] * ssp.kron(I, L)
    return D.tocsr()


# --------------------------------------------------------------------------- #
# Semi-Lagrangian interpolation T^SL (Sec. 3.3)
# --------------------------------------------------------------------------- #
def sl_matrix_1d(n, shift_cells, P):
    """Interpolation from the grid to the departure points y_j + kappa h_t
    (shift_cells = kappa h_t / h), order-P Lagrange with clamped stencils."""
    A = ssp.lil_matrix((n, n))
    for j in range(n):
        xi = j + shift_cells
        s = stencil_start(xi, n, P)
        w = lagrange_weights(range(s, s + P + 1), xi)
        for t in range(P + 1):
            A[j, s + t] = w[t]
    return A.tocsr()


def sl_matrix(n, kappa, h, dt, P):
    """T^SL = T_1 (x) T_2 for row-major grids: departure points
    y + kappa_omega dt, one constant shift per axis (Sec. 3.3)."""
    T1 = sl_matrix_1d(n, kappa[0] * dt / h, P)
    T2 = sl_matrix_1d(n, kappa[1] * dt / h, P)
    return ssp.kron(T1, T2).tocsr()


# --------------------------------------------------------------------------- #
# Pay-offs and cell-averaged initial data (Sec. 3.2.3, Sec. 4)
# --------------------------------------------------------------------------- #
PAYOFFS = ("put_avg", "call_avg", "put_1", "call_1", "exchange", "spread")


def payoff_g(kind):
    """g with pay-off = K max(g(y1, y2), 0), y_i = ln(S_i / K).

    put_avg is the put-on-the-average of Sec. 4; spread is the spread call
    max(S1 - S2 - K, 0) named among the extensions of Sec. 5; the others are
    used for checks (call-on-the-average, single-asset put / call on asset 1,
    exchange S1 - S2).
    Each g is monotone in each variable, so its kink set {g = 0} meets a cell
    iff g changes sign over the cell's corners.
    """
    if kind == "put_avg":
        return lambda y1, y2: 1.0 - 0.5 * (np.exp(y1) + np.exp(y2))
    if kind == "call_avg":
        return lambda y1, y2: 0.5 * (np.exp(y1) + np.exp(y2)) - 1.0
    if kind == "put_1":
        return lambda y1, y2: 1.0 - np.exp(y1) + 0.0 * y2
    if kind == "call_1":
        return lambda y1, y2: np.exp(y1) - 1.0 + 0.0 * y2
    if kind == "exchange":
        return lambda y1, y2: np.exp(y1) - np.exp(y2)
    if kind == "spread":
        return lambda y1, y2: np.exp(y1) - np.exp(y2) - 1.0
    raise ValueError(kind)


def _roots_in(f, a, b):
    """Sign-change root of a monotone f in the open interval (a, b), if any."""
    import scipy.optimize as spo
    fa, fb = f(a), f(b)
    if fa == 0.0 or fb == 0.0 or (fa > 0) == (fb > 0):
        return []
    return [spo.brentq(f, a, b, xtol=1e-300, rtol=1e-15)]


def _gl(f, a, b, nq=24):
    x, w = np.polynomial.legendre.leggauss(nq)
    t = 0.5 * (b - a) * x + 0.5 * (a + b)
    return 0.5 * (b - a) * float(np.dot(w, [f(ti) for ti in t]))


def cell_average(g, a1, b1, a2, b2, nq=24):
    """(1 / |cell|) * integral over [a1,b1]x[a2,b2] of max(g, 0): the cell average of
    Sec. 3.2.3, taken in the y variables (reading: on the log grid the averaging
    measure is dy1 dy2).

    The integral is split where the positive part of g has a kink: the inner
    (y2) integral at the root of g(y1, .), the outer (y1) integral where that
    root crosses a2 or b2; Gauss-Legendre on each smooth piece.
    """
    def inner(y1):
        pts = [a2] + _roots_in(lambda y2: g(y1, y2), a2, b2) + [b2]
        tot = 0.0
        for s, t in zip(pts[:-1], pts[1:]):
            mid = g(y1, 0.5 * (s + t))
            if mid > 0.0:
                tot += _gl(lambda y2: g(y1, y2), s, t, nq)
        return tot

    bps = sorted(set(_roots_in(lambda y1: g(y1, a2), a1, b1) + _roots_in(lambda y1: g(y1, b2), a1, b1)))
    pts = [a1] + bps + [b1]
    tot = 0.0
    for s, t in zip(pts[:-1], pts[1:]):
        tot += _gl(inner, s, t, nq)
    return tot / ((b1 - a1) * (b2 - a2))


def initial_values(kind, K, y1, y2, h, cell_avg=True):
    """V^0: the pay-off at the nodes, replaced by its cell average on the cells
    [y_j1 +- h/2] x [y_j2 +- h/2] that meet the kink set (Sec. 3.2.3).  A cell
    meets the kink set when g takes both signs (or zero) at its corners."""
    g = payoff_g(kind)
    Y1, Y2 = np.meshgrid(y1, y2, indexing="ij")
    V = K * np.maximum(g(Y1, Y2), 0.0)
    if not cell_avg:
        return V
    hh = 0.5 * h
    c = [g(Y1 + s1 * hh, Y2 + s2 * hh) for s1 in (-1, 1) for s2 in (-1, 1)]
    cmin = np.minimum.reduce(c)
    cmax = np.maximum.reduce(c)
    hit = (cmin <= 0.0) & (cmax >= 0.0)
    for j1, j2 in np.argwhere(hit):
        V[j1, j2] = K * cell_average(g, y1[j1] - hh, y1[j1] + hh, y2[j2] - hh, y2[j2] + hh)
    return V


# --------------------------------------------------------------------------- #
# Time march (Sec. 3.3, Algorithm 1)
# --------------------------------------------------------------------------- #
def step_list(theta, T, N_t, damping=True):
    """(theta, dt) of every step: N_t uniform steps of size T/N_t; with damping the
    first one is replaced by four steps of size dt/4 with theta = 1 (Sec. 3.3)."""
    dt = T / N_t
    if damping:
        return [(1.0, dt / 4.0)] * 4 + [(theta, dt)] * (N_t - 1)
    return [(theta, dt)] * N_t


def extrapolated_start(hist):
    """Starting value Y^{n,0} from V^{n-1}, V^{n-2}, ... (Sec. 3.3, extrapolated
    starting value): orders 0..3 as the history allows.  hist[-1] = V^{n-1}."""
    m = len(hist)
    if m == 1:
        return hist[-1].copy()
    if m == 2:
        return 2.0 * hist[-1] - hist[-2]
    if m == 3:
        return 3.0 * hist[-1] - 3.0 * hist[-2] + hist[-3]
    return 4.0 * hist[-1] - 6.0 * hist[-2] + 4.0 * hist[-3] - hist[-4]


class Problem:
    """Everything Algorithm 1 needs, on an n x n uniform log grid.

    disc     : output of ``integral.discretize`` (weights W, N_z, a, kappa, r_omega)
    y_lo, h  : grid origin (2,) and mesh width; y_i,j = y_lo[i] + j h
    sl_order : Lagrange order P of T^SL (1 or 3; Sec. 4 takes cubic)
    in_order : Lagrange order of T^in (1 or 3; Sec. 4 takes cubic)
    """

    def __init__(self, n, y_lo, h, disc, payoff="put_avg", K=100.0, T=1.0, N_t=32,
                 theta=0.5, sl_order=3, in_order=3, damping=True, cell_avg=True):
        self.n, self.h = int(n), float(h)
        self.y_lo = np.asarray(y_lo, dtype=np.float64).reshape(2)
        self.disc = disc
        self.payoff, self.K, self.T, self.N_t = payoff, float(K), float(T), int(N_t)
        self.theta, self.sl_order, self.in_order = float(theta), int(sl_order), int(in_order)
        self.damping, self.cell_avg = bool(damping), bool(cell_avg)
        self.y1 = self.y_lo[0] + self.h * np.arange(self.n)
        self.y2 = self.y_lo[1] + self.h * np.arange(self.n)

    def V0(self):
        return initial_values(self.payoff, self.K, self.y1, self.y2, self.h, self.cell_avg)

    def B(self, v, method=None):
        d = self.disc
        if method is None:
            method = "direct" if self.n <= 24 and d["N_z"] <= 24 else "fft"
        return apply_B(v, d["W"], d["N_z"], self.in_order, method)


def solve(prob, tol=1e-14, max_iter=200, inner="lu", B_method=None, n_steps=None,
          record=None, on_step=None):
    """Algorithm 1 in log coordinates: returns V after the step list (or after its
    first ``n_steps`` entries) and per-step fixed-point iteration counts.

    Each step (theta, dt):
      1. BV = B V (skipped when theta = 1, where it is not used);
      2. W = T^SL (V + dt (1-theta)((D - r_omega) V + BV));
      3. Y^0 by extrapolation over the main steps (reading: the four damped
         sub-steps form main step n = 1 and each starts from the previous
         sub-step's value);
      4. iterate (I - dt theta (D - r_omega I)) Y^k = dt theta B Y^{k-1} + W, each
         system solved exactly (sparse LU, or BiCGSTAB + ILU to 1e-15 as in
         Sec. 3.3), until max |Y^k - Y^{k-1}| / max(1, |Y^k|) < tol
         (Sec. 3.3 stopping rule).  If rounding stalls the increments before
         tol is met, the loop stops once they stop decreasing below 1e-13.
    ``record``, if a list, receives (step, theta, dt, iterations, last increment).
    ``on_step``, if given, is called as on_step(s, V) with the grid after step-list
    entry s (0-based); it only observes the march.
    """
    d = prob.disc
    n = prob.n
    N = n * n
    D = build_D(n, prob.h, d["a"])
    I = ssp.identity(N, format="csr")
    r_om = d["r_omega"]
    steps = step_list(prob.theta, prob.T, prob.N_t, prob.damping)
    if n_steps is not None:
        steps = steps[:n_steps]
    V = prob.V0()
    hist = [V.copy()]                     # V^0, V^1, ... at main-step ends
    cache = {}
    iters = []
    n_sub = 4 if prob.damping else 1
    for s, (th, dt) in enumerate(steps):
        key = (th, dt)
        if key not in cache:
            A = (I - dt * th * (D - r_om * I)).tocsc()
            TSL = sl_matrix(n, d["kappa"], prob.h, dt, prob.sl_order)
            if inner == "lu":
                fac = sla.splu(A)
                solver = lambda b, fac=fac: fac.solve(b)
            else:
                ilu = sla.spilu(A, drop_tol=1e-8, fill_factor=10)
                M = sla.LinearOperator(A.shape, ilu.solve)

                def solver(b, A=A, M=M):
                    x, info = sla.bicgstab(A, b, rtol=1e-15, atol=0.0, M=M, maxiter=1000)
                    if info != 0:
                        raise RuntimeError("BiCGSTAB did not converge")
                    return x
            cache[key] = (TSL, solver)
        TSL, solver = cache[key]
        v = V.ravel()
        if th < 1.0:
            BV = prob.B(V, B_method).ravel()
            E = v + dt * (1.0 - th) * (D @ v - r_om * v + BV)
        else:
            E = v
        Wv = TSL @ E
        # starting value
        in_damping = prob.damping and s < n_sub
        Y = V.ravel().copy() if in_damping else extrapolated_start(hist).ravel()
        prev_err = np.inf
        for k in range(1, max_iter + 1):
            rhs = dt * th * prob.B(Y.reshape(n, n), B_method).ravel() + Wv
            Yn = solver(rhs)
            err = float(np.max(np.abs(Yn - Y) / np.maximum(1.0, np.abs(Yn))))
            Y = Yn
            if err < tol or (err < 1e-13 and err >= prev_err):
                break
            prev_err = err
        else:
            raise RuntimeError("fixed-point iteration did not converge in %d iterations" % max_iter)
        iters.append(k)
        if record is not None:
            record.append((s, th, dt, k, err))
        V = Y.reshape(n, n)
        if on_step is not None:
            on_step(s, V)
        if (not prob.damping) or s >= n_sub - 1:
            hist.append(V.copy())
            if len(hist) > 4:
                hist.pop(0)
    return V, iters
