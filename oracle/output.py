"""Prices and deltas at spot pairs -- oracle side (test infrastructure).

Sec. 4 evaluates the grid solution off the grid by cubic interpolation; here the
tensor-product cubic Lagrange interpolant in the log variables y_i = ln(S_i/K),
with the clamped stencil of ``scheme.stencil_start``.  Deltas are the
derivatives of the same interpolant: dP/dS_i = (dP/dy_i) / S_i.
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
