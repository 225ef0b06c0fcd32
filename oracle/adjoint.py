"""Reverse-mode derivative of the discrete time march -- oracle side.

TEST INFRASTRUCTURE ONLY (see the package header): plain dense linear algebra
in FP64 for small grids.

Each entry (theta, dt) of the step list (Sec. 3.3) maps V^s to the exact
solution Y = V^{s+1} of the theta-scheme equation

    (I - dt theta A) Y = T^SL (I + dt (1 - theta) A) V^s,   A = D + B - r_omega I

(Sec. 3.3, the equation the fixed-point iteration of Algorithm 1 solves;
D from Sec. 3.2.1, B from Sec. 3.2.2, T^SL the semi-Lagrangian interpolation).
For a scalar J of V^{N} with gradient vbar, the exact discrete adjoint runs the
steps backwards:

    lam = (I - dt theta A)^{-T} Ybar,  mu = (T^SL)^T lam,
    Vbar^s = (I + dt (1 - theta) A)^T mu,

and the derivative of J with respect to any quantity q the step matrices
depend on is sum_s lam^T [d(T^SL)/dq E_s + dt (1 - theta) T^SL (dA/dq) V^s
+ dt theta (dA/dq) Y], with E_s = (I + dt (1 - theta) A) V^s.  The quantities
taken here are the coefficients a11, a12, a22 of D, the kill rate r_omega, the
drift coefficients kappa_omega (through the departure points of T^SL) and the
weights omega (through B).  Everything is assembled as dense matrices, so this
is meant for grids of a few hundred nodes.
"""

import numpy as np

from . import scheme


def _dense_B(prob):
    """B as a dense N x N matrix, column by column (B applied to unit grids)."""
    n = prob.n
    N = n * n
    Bm = np.zeros((N, N))
    e = np.zeros((n, n))
    for m in range(N):
        e.flat[m] = 1.0
        Bm[:, m] = prob.B(e, "fft").ravel()
        e.flat[m] = 0.0
    return Bm


def _sl_1d_derivative(n, shift_cells, P):
    """d T_1d / d xi at departure points j + shift_cells, stencil starts fixed."""
    M = np.zeros((n, n))
    for j in range(n):
        xi = j + shift_cells
        s = scheme.stencil_start(xi, n, P)
        dw = scheme.lagrange_dweights(range(s, s + P + 1), xi)
        M[j, s:s + P + 1] = dw
    return M


class Dense:
    """Dense step matrices of a Problem (shared across steps of one kind)."""

    def __init__(self, prob):
        d = prob.disc
        n = prob.n
        self.prob = prob
        self.N = n * n
        self.I = np.eye(self.N)
        self.D = scheme.build_D(n, prob.h, d["a"]).toarray()
        unit = [np.array([[1.0, 0.0], [0.0, 0.0]]), np.array([[0.0, 1.0], [1.0, 0.0]]),
                np.array([[0.0, 0.0], [0.0, 1.0]])]
        # D is linear in (a11, a12, a22); a12 enters through the symmetric off-diagonal
        self.Dc = [scheme.build_D(n, prob.h, u).toarray() for u in unit]
        self.B = _dense_B(prob) if d["N_z"] > 0 else np.zeros((self.N, self.N))
        self.A = self.D + self.B - d["r_omega"] * self.I
        self.steps = scheme.step_list(prob.theta, prob.T, prob.N_t, prob.damping)
        self._cache = {}

    def mats(self, th, dt):
        key = (th, dt)
        if key not in self._cache:
            prob, d = self.prob, self.prob.disc
            n, P = prob.n, prob.sl_order
            s1, s2 = d["kappa"][0] * dt / prob.h, d["kappa"][1] * dt / prob.h
            T1 = scheme.sl_matrix_1d(n, s1, P).toarray()
            T2 = scheme.sl_matrix_1d(n, s2, P).toarray()
            dT1 = _sl_1d_derivative(n, s1, P) * dt / prob.h
            dT2 = _sl_1d_derivative(n, s2, P) * dt / prob.h
            MI = self.I - dt * th * self.A
            ME = self.I + dt * (1.0 - th) * self.A
            self._cache[key] = dict(MI=MI, ME=ME, TSL=np.kron(T1, T2), dTk1=np.kron(dT1, T2), dTk2=np.kron(T1, dT2))
        return self._cache[key]


def forward(prob, dense=None, n_steps=None):
    """States V^0..V^S and explicit parts E_s of the exact theta-scheme march."""
    dense = dense or Dense(prob)
    steps = dense.steps if n_steps is None else dense.steps[:n_steps]
    V = [prob.V0().ravel()]
    E = []
    for th, dt in steps:
        m = dense.mats(th, dt)
        e = m["ME"] @ V[-1]
        E.append(e)
        V.append(np.linalg.solve(m["MI"], m["TSL"] @ e))
    return V, E, dense


def adjoint(prob, vbar, n_steps=None):
    """Reverse march for dJ/dV^S = vbar (n x n).  Returns a dict with
    V0bar (n x n), native = dJ/d(a11, a12, a22, r_omega, kappa1, kappa2) and
    omega = dJ/d omega (2 N_z x 2 N_z, indexed like disc['W'])."""
    V, E, dense = forward(prob, n_steps=n_steps)
    d = prob.disc
    n, Nz = prob.n, d["N_z"]
    steps = dense.steps if n_steps is None else dense.steps[:n_steps]
    ybar = np.asarray(vbar, dtype=np.float64).ravel().copy()
    native = np.zeros(6)
    gw = np.zeros((2 * Nz, 2 * Nz)) if Nz > 0 else np.zeros((0, 0))
    for s in range(len(steps) - 1, -1, -1):
        th, dt = steps[s]
        m = dense.mats(th, dt)
        lam = np.linalg.solve(m["MI"].T, ybar)
        mu = m["TSL"].T @ lam
        Y, Vs, Es = V[s + 1], V[s], E[s]
        ci, ce = dt * th, dt * (1.0 - th)
        for c in range(3):
            native[c] += ci * lam @ (dense.Dc[c] @ Y) + ce * mu @ (dense.Dc[c] @ Vs)
        native[3] -= ci * lam @ Y + ce * mu @ Vs
        native[4] += lam @ (m["dTk1"] @ Es)
        native[5] += lam @ (m["dTk2"] @ Es)
        if Nz > 0:
            # dB v / d omega[a, b] at m = vin[m1 + a, m2 + b] (B = correlation of the
            # half-shifted interpolant with Omega, Sec. 3.2.2)
            yin = scheme.interp_to_half_grid(Y.reshape(n, n), prob.in_order, Nz)
            vin = scheme.interp_to_half_grid(Vs.reshape(n, n), prob.in_order, Nz)
            L2 = lam.reshape(n, n)
            M2 = mu.reshape(n, n)
            for a in range(2 * Nz):
                for b in range(2 * Nz):
                    gw[a, b] += ci * np.sum(L2 * yin[a:a + n, b:b + n]) + ce * np.sum(M2 * vin[a:a + n, b:b + n])
        ybar = m["ME"].T @ mu
    return dict(V0bar=ybar.reshape(n, n), native=native, omega=gw, VN=V[-1].reshape(n, n))
