"""2D Normal Tempered Stable (NTS) Levy measure -- oracle side (test infrastructure).

Follows Sec. 4 (the NTS Levy density used in the experiments) and Appendix A
(Tables 4 and 5: subordinator quantities, NTS characteristic exponent and
variance).  Plain NumPy/SciPy in FP64.
"""

import math

import numpy as np
import scipy.special as sps


def nts_params(alpha, delta, lam, eta, rho):
    """Validated NTS parameter set (Sec. 4: 0 <= alpha < 1, delta > 0, lambda > 0,
    eta in R^2, rho symmetric positive definite).

    Also requires the exponential moment E[exp(L_i(1))] to exist for both
    coordinates (needed by the drift correction kappa_omega of Sec. 3.1 and by
    the characteristic exponent at u = -i e_i, Table 5): the subordinator Laplace
    argument lambda - eta_i - rho_ii / 2 must be positive.
    """
    eta = np.asarray(eta, dtype=np.float64).reshape(2)
    rho = np.asarray(rho, dtype=np.float64).reshape(2, 2)
    if not (0.0 <= alpha < 1.0):
        raise ValueError("alpha must lie in [0, 1)")
    if not (delta > 0.0 and lam > 0.0):
        raise ValueError("delta and lambda must be positive")
    if abs(rho[0, 1] - rho[1, 0]) > 1e-15 * max(1.0, abs(rho[0, 1])):
        raise ValueError("rho must be symmetric")
    det = rho[0, 0] * rho[1, 1] - rho[0, 1] * rho[1, 0]
    if not (rho[0, 0] > 0.0 and det > 0.0):
        raise ValueError("rho must be positive definite")
    for i in range(2):
        if not (lam - eta[i] - 0.5 * rho[i, i] > 0.0):
            raise ValueError("exponential moment of L_%d(1) does not exist" % (i + 1))
    rinv = np.array([[rho[1, 1], -rho[0, 1]], [-rho[1, 0], rho[0, 0]]]) / det
    eta_rn2 = float(eta @ rinv @ eta)            # ||eta||_rho^2
    c1 = math.sqrt(eta_rn2 + 2.0 * lam)           # sqrt(||eta||_rho^2 + 2 lambda)
    return dict(alpha=float(alpha), delta=float(delta), lam=float(lam), eta=eta,
                rho=rho, det=det, rinv=rinv, c1=c1, rinv_eta=rinv @ eta)


def nts_from_std(sigma1, sigma2, corr, theta1, theta2, kappa, alpha):
    """Map (sigma_1, sigma_2, correlation, skews theta_1, theta_2, subordinator
    variance kappa, index alpha) to the paper's NTS parameters.

    Reading (not fixed by the paper): the subordinator G of Appendix A is taken
    with unit mean and variance kappa.  From Table 4, E[G(1)] = delta
    Gamma(1-alpha) / lambda^(1-alpha) and V[G(1)] = delta Gamma(2-alpha) /
    lambda^(2-alpha); setting them to 1 and kappa gives lambda = (1-alpha)/kappa
    and delta = lambda^(1-alpha) / Gamma(1-alpha).  The Brownian motion that is
    subordinated has drift eta = (theta_1, theta_2) and covariance
    rho = [[s1^2, c s1 s2], [c s1 s2, s2^2]] (Appendix A.2).
    """
    if not (kappa > 0.0):
        raise ValueError("kappa must be positive")
    lam = (1.0 - alpha) / kappa
    delta = lam ** (1.0 - alpha) / math.gamma(1.0 - alpha)
    rho = np.array([[sigma1 * sigma1, corr * sigma1 * sigma2],
                    [corr * sigma1 * sigma2, sigma2 * sigma2]])
    return nts_params(alpha, delta, lam, (theta1, theta2), rho)


def _rho_norm(p, z1, z2):
    ri = p["rinv"]
    q2 = ri[0, 0] * z1 * z1 + 2.0 * ri[0, 1] * z1 * z2 + ri[1, 1] * z2 * z2
    return np.sqrt(q2)


def log_density(p, z1, z2):
    """log of the NTS Levy density (Sec. 4, the Bessel-K_{1+alpha} form):

        l(z) = delta/pi * sqrt(c1^(2(1+alpha)) / det rho) * K_{1+alpha}(c1 ||z||_rho)
               * ||z||_rho^(-1-alpha) * exp(<eta, z>_rho),
        c1 = sqrt(||eta||_rho^2 + 2 lambda), <x, y>_rho = x^T rho^{-1} y.

    Evaluated through the exponentially scaled Bessel function so that large
    arguments do not underflow.
    """
    z1 = np.asarray(z1, dtype=np.float64)
    z2 = np.asarray(z2, dtype=np.float64)
    a = p["alpha"]
    nu = 1.0 + a
    q = _rho_norm(p, z1, z2)
    x = p["c1"] * q
    logpref = (math.log(p["delta"] / math.pi)
               + 0.5 * (2.0 * nu * math.log(p["c1"]) - math.log(p["det"])))
    e = p["rinv_eta"]
    return (logpref + np.log(sps.kve(nu, x)) - x - nu * np.log(q)
            + e[0] * z1 + e[1] * z2)


def density(p, z1, z2):
    """The NTS Levy density l(z) of Sec. 4 (see ``log_density``)."""
    return np.exp(log_density(p, z1, z2))


def variance(p):
    """Closed-form covariance of L(1) (Appendix A, Table 5):

        V[L(1)] = delta Gamma(2-alpha)/lambda^(2-alpha) (rho lambda/(1-alpha) + eta eta^T).

    The variance printed in Sec. 4 carries the factor rho lambda^(1-alpha); only
    the Table 5 form reproduces Table 2, so Table 5 is taken.
    """
    a, d, lam, eta, rho = p["alpha"], p["delta"], p["lam"], p["eta"], p["rho"]
    return d * math.gamma(2.0 - a) / lam ** (2.0 - a) * (rho * lam / (1.0 - a) + np.outer(eta, eta))


def subordinator_mean(p):
    """E[G(1)] of the tempered stable subordinator (Appendix A, Table 4)."""
    a = p["alpha"]
    return p["delta"] * math.gamma(1.0 - a) / p["lam"] ** (1.0 - a)


def char_exponent(p, u):
    """Characteristic exponent psi_L(u) = log E[exp(i u^T L(1))] of the
    compensated NTS process (Appendix A, Table 5), for complex u of shape (..., 2):

        alpha = 0:     -delta ln((lambda - i u^T eta + u^T rho u / 2)/lambda) - i u^T c
        alpha in (0,1): delta Gamma(-alpha) ((lambda - i u^T eta + u^T rho u / 2)^alpha
                         - lambda^alpha) - i u^T c,
        c = delta Gamma(1-alpha)/lambda^(1-alpha) eta  (Appendix A.2).
    """
    u = np.asarray(u, dtype=np.complex128)
    a, d, lam, eta, rho = p["alpha"], p["delta"], p["lam"], p["eta"], p["rho"]
    c = subordinator_mean(p) * eta
    ueta = u[..., 0] * eta[0] + u[..., 1] * eta[1]
    urho = (u[..., 0] * (rho[0, 0] * u[..., 0] + rho[0, 1] * u[..., 1])
            + u[..., 1] * (rho[1, 0] * u[..., 0] + rho[1, 1] * u[..., 1]))
    arg = lam - 1j * ueta + 0.5 * urho
    uc = u[..., 0] * c[0] + u[..., 1] * c[1]
    if a == 0.0:
        return -d * np.log(arg / lam) - 1j * uc
    return d * math.gamma(-a) * (arg ** a - lam ** a) - 1j * uc
