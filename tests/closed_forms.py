"""Closed-form and independent reference prices used to pin the oracle.

These are not part of the oracle: they are textbook formulas (Black-Scholes
prices and Greeks, Margrabe, the spread call as a one-dimensional integral of
Black-Scholes calls) and a one-dimensional Fourier-inversion price built from the NTS
characteristic exponent of Appendix A (Table 5), used to check the oracle's
two-dimensional march from outside.
"""

import math

import numpy as np
import scipy.integrate as spi
from scipy.stats import norm


def bs_put(S, K, T, r, sigma):
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    d2 = d1 - sigma * math.sqrt(T)
    return K * math.exp(-r * T) * norm.cdf(-d2) - S * norm.cdf(-d1)


def bs_put_delta_gamma(S, K, T, r, sigma):
    """Delta and Gamma of the Black-Scholes put."""
    d1 = (math.log(S / K) + (r + 0.5 * sigma * sigma) * T) / (sigma * math.sqrt(T))
    return norm.cdf(d1) - 1.0, norm.pdf(d1) / (S * sigma * math.sqrt(T))


def bs_spread_call(S1, S2, K, T, r, sig1, sig2, corr, nodes=100):
    """Spread call max(S1 - S2 - K, 0) under 2D geometric Brownian motion.
    Conditional on the standard normal z that drives asset 2, asset 1 is
    lognormal with conditional mean F(z) and log-volatility v, so the price is
    e^{-rT} E_z[Black(F(z), S2_T(z) + K, v)], taken by Gauss-Hermite quadrature
    in z (the conditional call price is smooth in z)."""
    x, w = np.polynomial.hermite_e.hermegauss(nodes)       # weight exp(-z^2 / 2)
    w = w / math.sqrt(2.0 * math.pi)
    sT = math.sqrt(T)
    S2T = S2 * np.exp((r - 0.5 * sig2 * sig2) * T + sig2 * sT * x)
    v = sig1 * math.sqrt(1.0 - corr * corr) * sT
    F = S1 * np.exp((r - 0.5 * sig1 * sig1) * T + sig1 * sT * corr * x + 0.5 * v * v)
    X = S2T + K
    d1 = (np.log(F / X) + 0.5 * v * v) / v
    d2 = d1 - v
    return math.exp(-r * T) * float(np.dot(w, F * norm.cdf(d1) - X * norm.cdf(d2)))


def margrabe(S1, S2, T, sig1, sig2, corr):
    """Exchange option max(S1 - S2, 0) under 2D geometric Brownian motion."""
    s = math.sqrt(sig1 * sig1 + sig2 * sig2 - 2.0 * corr * sig1 * sig2)
    d1 = (math.log(S1 / S2) + 0.5 * s * s * T) / (s * math.sqrt(T))
    d2 = d1 - s * math.sqrt(T)
    return S1 * norm.cdf(d1) - S2 * norm.cdf(d2)


def fourier_put_1d(S, K, T, r, psi):
    """European put on one asset whose log-price is ln S + (r - psi(-i)) T + L(T),
    L a compensated Levy process with characteristic exponent psi (so that
    E[e^{i u L(T)}] = exp(T psi(u))).  Gil-Pelaez inversion of the two exercise
    probabilities (under Q and under the share measure)."""
    drift = r - psi(-1j).real
    x0 = math.log(S) + drift * T
    lk = math.log(K)

    def phi(u):
        return np.exp(1j * u * x0 + T * psi(u))

    phi_mi = phi(-1j).real  # = S e^{rT}

    def f_q(u):
        return (np.exp(-1j * u * lk) * phi(u) / (1j * u)).real

    def f_s(u):
        return (np.exp(-1j * u * lk) * phi(u - 1j) / (1j * u * phi_mi)).real

    opts = dict(limit=2000, epsabs=1e-13, epsrel=1e-12)
    iq = spi.quad(f_q, 0.0, np.inf, **opts)[0]
    is_ = spi.quad(f_s, 0.0, np.inf, **opts)[0]
    p_q = 0.5 - iq / math.pi
    p_s = 0.5 - is_ / math.pi
    return K * math.exp(-r * T) * p_q - S * p_s
