"""Seeded synthetic workloads shared by the oracle-side tests, the GPU tests and
the benchmark.

This module holds data only: contract and model parameters, grid sizes and
seeded random draws.  It contains none of the method's arithmetic (no Levy
density, no weights, no operators), so both the oracle (``oracle/``) and the
HIP path (``paper_2511_02700_amd``) can take their inputs from it without
sharing any computation.

The workloads follow the paper's experiments (Sec. 4): a European
put-on-the-average option max(K - (S1+S2)/2, 0) under a pure-jump 2D Normal
Tempered Stable model, here parameterised by (sigma1, sigma2, corr, theta1,
theta2, kappa, alpha) of the subordinated Brownian motion, on a uniform
log-price grid y_i = ln(S_i / K).
"""

import numpy as np

# Model parameters in the subordinated-Brownian-motion form: Brownian
# volatilities and correlation, drifts (skews), subordinator variance kappa and
# index alpha.
NIG_BASE = dict(sigma1=0.2, sigma2=0.25, corr=0.3, theta1=-0.1, theta2=-0.1, kappa=0.2, alpha=0.5)
FV_BASE = dict(sigma1=0.2, sigma2=0.25, corr=0.3, theta1=-0.05, theta2=-0.15, kappa=0.15, alpha=0.3)

CONTRACT = dict(payoff="put_avg", K=100.0, T=1.0, r=0.03)

# name -> workload.  n nodes per axis, both ends included; N_t time steps;
# theta of the theta-method; tol of the fixed-point stopping rule.
WORKLOADS = {
    # NIG (alpha = 1/2), 64 x 64 on [-3, 3]^2, 32 steps.
    "nig64": dict(model=NIG_BASE, n=64, y_lo=-3.0, y_hi=3.0, N_t=32, theta=0.5, tol=1e-12,
                  **CONTRACT),
    # finite-variation NTS (alpha = 0.3), 512 x 512 on [-4, 4]^2, 256 steps.
    "fv512": dict(model=FV_BASE, n=512, y_lo=-4.0, y_hi=4.0, N_t=256, theta=0.5, tol=1e-12,
                  **CONTRACT),
    # large grids, 2048 x 2048 on [-5, 5]^2, 1024 steps, alpha in {0.5, 0.3}, corr in {-0.5, 0.5}.
    "nig2048_m": dict(model=dict(NIG_BASE, corr=-0.5), n=2048, y_lo=-5.0, y_hi=5.0, N_t=1024,
                      theta=0.5, tol=1e-12, **CONTRACT),
    "nig2048_p": dict(model=dict(NIG_BASE, corr=0.5), n=2048, y_lo=-5.0, y_hi=5.0, N_t=1024,
                      theta=0.5, tol=1e-12, **CONTRACT),
    "fv2048_m": dict(model=dict(FV_BASE, corr=-0.5), n=2048, y_lo=-5.0, y_hi=5.0, N_t=1024,
                     theta=0.5, tol=1e-12, **CONTRACT),
    "fv2048_p": dict(model=dict(FV_BASE, corr=0.5), n=2048, y_lo=-5.0, y_hi=5.0, N_t=1024,
                     theta=0.5, tol=1e-12, **CONTRACT),
    # adjoint-sized grid: 1024 x 1024 on [-4, 4]^2, 512 steps, alpha = 0.4.
    "nts1024": dict(model=dict(NIG_BASE, alpha=0.4), n=1024, y_lo=-4.0, y_hi=4.0, N_t=512,
                    theta=0.5, tol=1e-12, **CONTRACT),
}


def workload(name, **over):
    """A copy of a named workload with fields overridden."""
    w = dict(WORKLOADS[name])
    w["model"] = dict(w["model"])
    for k, v in over.items():
        if k in w["model"]:
            w["model"][k] = v
        else:
            w[k] = v
    return w


def spot_pairs(count=64, seed=1, lo=80.0, hi=120.0):
    """Seeded spot pairs, uniform in [lo, hi]^2."""
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=(count, 2))


def random_grid(n, seed=0, kind="normal"):
    """A seeded n x n test grid (FP64).  kind='normal' draws N(0,1) values;
    kind='smooth' draws a smooth bump plus noise, closer to option values."""
    rng = np.random.default_rng(seed)
    if kind == "normal":
        return rng.standard_normal((n, n))
    y = np.linspace(-1.0, 1.0, n)
    Y1, Y2 = np.meshgrid(y, y, indexing="ij")
    return np.exp(-(Y1 ** 2 + Y2 ** 2)) + 1e-3 * rng.standard_normal((n, n))


def batch_draw(count=256, seed=3):
    """The batched workload: per solve, n ~ U{128, 256, 512, 1024}, alpha ~ U[0.2, 0.6],
    sigma_i ~ U[0.1, 0.4], corr ~ U[-0.7, 0.7], K ~ U[80, 120], T ~ U[0.25, 2],
    N_t = n / 2; skews, kappa, r and the domain [-4, 4]^2 fixed."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n = int(rng.choice([128, 256, 512, 1024]))
        out.append(dict(
            model=dict(sigma1=float(rng.uniform(0.1, 0.4)), sigma2=float(rng.uniform(0.1, 0.4)),
                       corr=float(rng.uniform(-0.7, 0.7)), theta1=-0.1, theta2=-0.1, kappa=0.2,
                       alpha=float(rng.uniform(0.2, 0.6))),
            n=n, y_lo=-4.0, y_hi=4.0, N_t=n // 2, theta=0.5, tol=1e-12, payoff="put_avg",
            K=float(rng.uniform(80.0, 120.0)), T=float(rng.uniform(0.25, 2.0)), r=0.03))
    return out
