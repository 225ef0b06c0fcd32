"""Prices and deltas at spot pairs, and Greeks on the grid -- oracle side (test
infrastructure).

Sec. 4 evaluates the grid solution off the grid by cubic interpolation; here the
tensor-product cubic Lagrange interpolant in the log variables y_i = ln(S_i/K),
with the clamped stencil of ``scheme.stencil_start``.  Deltas are the
derivatives of the same interpolant: dP/dS_i = (dP/dy_i) / S_i.

The Delta and Gamma surfaces of Sec. 4 (its figure of the Greeks over the
spot plane) are finite differences of the grid solution: see greeks_on_grid.
"""

import math

import numpy as np

from .scheme import lagrange_dweights, lagrange_weights, stencil_start


def prices(V, y_lo, h, K, spots, with_delta=False):
    """Interpolated prices (and deltas) at spot pairs spots[k] = (S1, S2)."""
    n = V.shape[0]
    spots = np.asarray(spots, dtype=np.float64).reshape(-1, 2)
    P = np.empty(len(spots))
    Dl = np.empty((len(spots), 2))
    for k, (s1, s2) in enumerate(spots):
        xi1 = (math.log(s1 / K) - y_lo[0]) / h
        xi2 = (math.log(s2 / K) - y_lo[1]) / h
        a = stencil_start(xi1, n, 3)
        b = stencil_start(xi2, n, 3)
        w1 = lagrange_weights(range(a, a + 4), xi1)
        w2 = lagrange_weights(range(b, b + 4), xi2)
        blk = V[a:a + 4, b:b + 4]
        P[k] = w1 @ blk @ w2
        if with_delta:
            d1 = lagrange_dweights(range(a, a + 4), xi1) / h
            d2 = lagrange_dweights(range(b, b + 4), xi2) / h
            Dl[k, 0] = (d1 @ blk @ w2) / s1
            Dl[k, 1] = (w1 @ blk @ d2) / s2
    return (P, Dl) if with_delta else P


def _d1(V, h, axis):
    """dV/dy along axis: central differences inside, second-order one-sided
    differences (-3, 4, -1) / 2h on the two edges."""
    V = np.moveaxis(V, axis, 0)
    D = np.empty_like(V)
    D[1:-1] = (V[2:] - V[:-2]) / (2.0 * h)
    D[0] = (-3.0 * V[0] + 4.0 * V[1] - V[2]) / (2.0 * h)
    D[-1] = (3.0 * V[-1] - 4.0 * V[-2] + V[-3]) / (2.0 * h)
    return np.moveaxis(D, 0, axis)


def _d2(V, h, axis):
    """d2V/dy2 along axis: (1, -2, 1) / h^2 inside, the second-order one-sided
    stencil (2, -5, 4, -1) / h^2 on the two edges."""
    V = np.moveaxis(V, axis, 0)
    D = np.empty_like(V)
    D[1:-1] = (V[2:] - 2.0 * V[1:-1] + V[:-2]) / (h * h)
    D[0] = (2.0 * V[0] - 5.0 * V[1] + 4.0 * V[2] - V[3]) / (h * h)
    D[-1] = (2.0 * V[-1] - 5.0 * V[-2] + 4.0 * V[-3] - V[-4]) / (h * h)
    return np.moveaxis(D, 0, axis)


def greeks_on_grid(V, y_lo, h, K):
    """Delta and Gamma surfaces at the grid nodes.  With S_i = K e^{y_i}:
    dV/dS_i = V_{y_i} / S_i, d2V/dS_i^2 = (V_{y_i y_i} - V_{y_i}) / S_i^2 and
    d2V/dS_1 dS_2 = V_{y_1 y_2} / (S_1 S_2), the y-derivatives by the stencils
    of _d1 and _d2 (the mixed one as _d1 along axis 0 of _d1 along axis 1).
    Returns (delta1, delta2, gamma11, gamma12, gamma22), each n x n."""
    V = np.asarray(V, dtype=np.float64)
    n = V.shape[0]
    S1 = K * np.exp(y_lo[0] + h * np.arange(n))[:, None]
    S2 = K * np.exp(y_lo[1] + h * np.arange(n))[None, :]
    v1, v2 = _d1(V, h, 0), _d1(V, h, 1)
    v11, v22 = _d2(V, h, 0), _d2(V, h, 1)
    v12 = _d1(_d1(V, h, 1), h, 0)
    return (v1 / S1, v2 / S2, (v11 - v1) / (S1 * S1), v12 / (S1 * S2), (v22 - v2) / (S2 * S2))
