"""Integral discretization -- oracle side (test infrastructure).

Follows Sec. 3.1 (the partition R_I / R_II / R_III of the truncated jump domain,
the cell-centred z-grid, the artificial diffusion over R_I, the weights omega and
the modified drift and kill rate) and the scheme settings of Sec. 4 (z_max^I,
z_max^II and z_max^III rules), on a z-grid whose mesh width equals the
log-price mesh width h.
"""

import math

import numpy as np
import scipy.integrate as spi
import scipy.optimize as spo

from . import levy


def _ray_root(p, u1, u2, log_cut):
    """Radius r > 0 with l(r u) = cut along the unit direction u.

    Along a ray the NTS density strictly decreases (d/dr log l <= -(c1 - ||eta||_rho)
    ||u||_rho < 0 because K_{nu+1} >= K_nu), so the root is unique.
    """
    f = lambda r: float(levy.log_density(p, r * u1, r * u2)) - log_cut
    lo = 1e-12
    hi = 1e-3
    while f(hi) > 0.0:
        lo = hi
        hi *= 2.0
        if hi > 1e6:
            raise RuntimeError("level set of the Levy density not found")
    return spo.brentq(f, lo, hi, xtol=1e-300, rtol=1e-15, maxiter=500)


def z_star(p, ell_cut=1e-14, n_angles=4096):
    """z_max^III before rounding to the z-grid (Sec. 4 settings): the largest
    infinity norm over the level set {l(z) = ell_cut}.

    Reading: the paper states the level 1e-8 but prints values (11.5010, 2.1410,
    0.4172, 0.8807) that are those of the level 1e-14; ``ell_cut`` is therefore a
    parameter, default 1e-14.  Computed by a root along each of ``n_angles`` rays,
    then a bounded maximisation over the angle around the best ray.
    """
    log_cut = math.log(ell_cut)

    def g(phi):
        c, s = math.cos(phi), math.sin(phi)
        r = _ray_root(p, c, s, log_cut)
        return r * max(abs(c), abs(s))

    phis = np.arange(n_angles) * (2.0 * math.pi / n_angles)
    vals = np.array([g(ph) for ph in phis])
    k = int(np.argmax(vals))
    d = 2.0 * math.pi / n_angles
    res = spo.minimize_scalar(lambda ph: -g(ph), bounds=(phis[k] - d, phis[k] + d),
                              method="bounded", options=dict(xatol=1e-12))
    return max(float(vals[k]), -float(res.fun))


def grid_sizes(p, h, ell_cut=1e-14, m1=2, frac2=math.sqrt(0.1)):
    """Integer sizes of the z-grid (Sec. 3.1 z-grid and Sec. 4 settings) with h_z = h:

        N_z = ceil(z* / h)             (so z_max^III = N_z h >= z*),
        z_max^I  = m1 h                (paper: m1 = 2),
        z_max^II = M2 h,  M2 = ceil(frac2 N_z - 1/2)   (paper: frac2 = sqrt(0.1)).
    """
    zs = z_star(p, ell_cut)
    nz = int(math.ceil(zs / h))
    m2 = int(math.ceil(frac2 * nz - 0.5))
    return dict(z_star=zs, N_z=nz, M1=int(m1), M2=m2)


def cell_norm_inf(N_z):
    """c_l = max(|l1 + 1/2|, |l2 + 1/2|) for l in [-N_z, N_z-1]^2: the infinity
    norm of the cell centre z_l in units of h (Sec. 3.1 z-grid)."""
    l = np.arange(-N_z, N_z) + 0.5
    return np.maximum(np.abs(l)[:, None], np.abs(l)[None, :])


def weights(p, h, N_z, M1, M2, ng=8):
    """Quadrature weights omega_l on the cells R_l, l in [-N_z, N_z-1]^2
    (Sec. 3.1, the omega definition):

        z_l in R_I   (c_l <= M1):       0
        z_l in R_II  (M1 < c_l <= M2):  ||z_l||^-2 * integral over R_l of ||z||^2 l(z) dz
        z_l in R_III (c_l > M2):        l(z_l) h^2          (midpoint rule)

    with the Euclidean norm (Proposition 3.1 takes the Euclidean norm).  The
    cell integrals over R_II use a tensor Gauss-Legendre rule with ``ng`` nodes
    per axis; the integrand is analytic on each R_II cell, which is at least 2h
    from the origin.  Returned as an array W[l1 + N_z, l2 + N_z].
    """
    c = cell_norm_inf(N_z)
    W = np.zeros((2 * N_z, 2 * N_z))
    zc = (np.arange(-N_z, N_z) + 0.5) * h
    Z1, Z2 = np.meshgrid(zc, zc, indexing="ij")
    r3 = c > M2
    W[r3] = levy.density(p, Z1[r3], Z2[r3]) * h * h
    r2 = (c > M1) & (c <= M2)
    idx = np.argwhere(r2)
    xg, wg = np.polynomial.legendre.leggauss(ng)
    off = 0.5 * h * xg                       # nodes relative to the cell centre
    w2 = np.outer(wg, wg).ravel() * (0.25 * h * h)
    o1 = np.repeat(off, ng)
    o2 = np.tile(off, ng)
    chunk = 20000
    for s in range(0, len(idx), chunk):
        ii = idx[s:s + chunk]
        c1 = zc[ii[:, 0]]
        c2 = zc[ii[:, 1]]
        q1 = c1[:, None] + o1[None, :]
        q2 = c2[:, None] + o2[None, :]
        f = (q1 * q1 + q2 * q2) * levy.density(p, q1, q2)
        integ = f @ w2
        W[ii[:, 0], ii[:, 1]] = integ / (c1 * c1 + c2 * c2)
    return W


def small_jump_cov(p, h, M1, epsrel=1e-13):
    """Artificial diffusion matrix S = integral over R_I of z z^T l(z) dz
    (Sec. 3.1, the small-jump replacement), R_I = [-M1 h, M1 h]^2.

    Computed in polar coordinates: S = int_phi u u^T I(phi) dphi with
    I(phi) = int_0^{R(phi)} r^3 l(r u) dr and R(phi) = M1 h / max(|cos|, |sin|).
    The radial integrand behaves like r^(1 - 2 alpha) at the origin, so the
    inner integral uses QUADPACK's algebraic-endpoint-weight rule, the outer
    one an adaptive vector rule over the eight octants.
    """
    a = p["alpha"]
    half = M1 * h

    def inner(phi):
        u1, u2 = math.cos(phi), math.sin(phi)
        R = half / max(abs(u1), abs(u2))
        g = lambda r: r ** (2.0 + 2.0 * a) * float(levy.density(p, r * u1, r * u2)) if r > 0 else \
            _small_r_limit(p, u1, u2)
        val, _ = spi.quad(g, 0.0, R, weight="alg", wvar=(1.0 - 2.0 * a, 0.0),
                          epsabs=0.0, epsrel=epsrel, limit=200)
        return np.array([u1 * u1, u1 * u2, u2 * u2]) * val

    tot = np.zeros(3)
    for k in range(8):
        v, _ = spi.quad_vec(inner, k * math.pi / 4.0, (k + 1) * math.pi / 4.0,
                            epsabs=0.0, epsrel=epsrel, limit=200)
        tot += v
    return np.array([[tot[0], tot[1]], [tot[1], tot[2]]])


def _small_r_limit(p, u1, u2):
    """lim_{r->0} r^(2+2 alpha) l(r u), used only if QUADPACK samples r = 0:
    K_nu(x) ~ Gamma(nu) 2^(nu-1) x^-nu as x -> 0 (nu = 1 + alpha > 0)."""
    a = p["alpha"]
    nu = 1.0 + a
    q = math.sqrt(p["rinv"][0, 0] * u1 * u1 + 2 * p["rinv"][0, 1] * u1 * u2 + p["rinv"][1, 1] * u2 * u2)
    pref = p["delta"] / math.pi * math.sqrt(p["c1"] ** (2 * nu) / p["det"])
    return pref * math.gamma(nu) * 2.0 ** (nu - 1.0) * p["c1"] ** (-nu) * q ** (-2.0 * nu)


def drift_and_rate(W, h, N_z, r):
    """Modified drift coefficients and kill rate of the approximating operator
    A_omega (Sec. 3.1):

        kappa_omega^(i) = r - sum_l omega_l (exp(z_l^(i)) - 1),
        r_omega         = r + sum_l omega_l.

    Summed exactly (math.fsum).  Returns (kappa (2,), r_omega, sum omega).
    """
    zc = (np.arange(-N_z, N_z) + 0.5) * h
    em1 = np.expm1(zc)
    k1 = r - math.fsum((W * em1[:, None]).ravel())
    k2 = r - math.fsum((W * em1[None, :]).ravel())
    s = math.fsum(W.ravel())
    return np.array([k1, k2]), r + s, s


def discretize(p, h, r, sigma_bs=None, ell_cut=1e-14, m1=2, frac2=math.sqrt(0.1), ng=8):
    """All plan-time quantities of the integral discretization for mesh width h:
    sizes, weights, S, a = sigma sigma^T + S, kappa_omega, r_omega (Sec. 3.1).

    ``sigma_bs`` is the Brownian covariance sigma sigma^T (zero in the paper's
    experiments, Sec. 4).  ``p=None`` means a zero Levy measure (pure
    Black-Scholes), for which N_z = 0 and every jump quantity vanishes.
    """
    sbs = np.zeros((2, 2)) if sigma_bs is None else np.asarray(sigma_bs, dtype=np.float64)
    if p is None:
        return dict(z_star=0.0, N_z=0, M1=m1, M2=0, W=np.zeros((0, 0)), S=np.zeros((2, 2)),
                    a=sbs.copy(), kappa=np.array([r, r]), r_omega=r, sum_omega=0.0)
    sz = grid_sizes(p, h, ell_cut, m1, frac2)
    W = weights(p, h, sz["N_z"], sz["M1"], sz["M2"], ng)
    S = small_jump_cov(p, h, sz["M1"])
    kappa, r_om, s = drift_and_rate(W, h, sz["N_z"], r)
    out = dict(sz)
    out.update(W=W, S=S, a=sbs + S, kappa=kappa, r_omega=r_om, sum_omega=s)
    return out
