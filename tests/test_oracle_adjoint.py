"""Pins of the oracle's discrete adjoint (oracle/adjoint.py) against things
other than itself: central finite differences of the oracle's own forward
march, the linearity of the march in V^0, and the agreement of its dense exact
march with the iterative Algorithm 1 of oracle/scheme.py."""

import copy

import numpy as np
import pytest

import workloads
from oracle import adjoint as oadj
from oracle import integral, levy, scheme


def _problem(n=18, N_t=5, half=2.0, alpha=0.5, corr=0.3, theta=0.5):
    w = workloads.workload("nig64", n=n, N_t=N_t, y_lo=-half, y_hi=half, alpha=alpha, corr=corr, theta=theta)
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    return scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"])


@pytest.fixture(scope="module")
def case():
    prob = _problem()
    rng = np.random.default_rng(5)
    vbar = rng.standard_normal((prob.n, prob.n))
    res = oadj.adjoint(prob, vbar)
    return prob, vbar, res


def _J(prob, vbar):
    V, _, _ = oadj.forward(prob)
    return float(np.sum(vbar.ravel() * V[-1]))


def test_dense_march_equals_algorithm_1(case):
    """The dense exact march is the fixed point that Algorithm 1 iterates to."""
    prob, _, res = case
    Vo, _ = scheme.solve(prob, tol=1e-14)
    assert np.max(np.abs(res["VN"] - Vo)) < 1e-11


def test_linear_in_initial_values(case):
    """For fixed coefficients the march is linear in V^0, so J = vbar . V^N
    equals V0bar . V^0."""
    prob, vbar, res = case
    J = np.sum(vbar * res["VN"])
    assert abs(J - np.sum(res["V0bar"] * prob.V0())) < 1e-10 * max(1.0, abs(J))


def _perturbed(prob, which, eps):
    q = copy.copy(prob)
    d = dict(prob.disc)
    if which in ("a11", "a12", "a22"):
        a = np.array(d["a"], dtype=np.float64)
        i, j = {"a11": (0, 0), "a12": (0, 1), "a22": (1, 1)}[which]
        a[i, j] += eps
        if i != j:
            a[j, i] += eps
        d["a"] = a
    elif which == "r_omega":
        d["r_omega"] = d["r_omega"] + eps
    elif which in ("kappa1", "kappa2"):
        k = np.array(d["kappa"], dtype=np.float64)
        k[0 if which == "kappa1" else 1] += eps
        d["kappa"] = k
    else:
        W = np.array(d["W"], dtype=np.float64)
        W[which] += eps
        d["W"] = W
    q.disc = d
    return q


@pytest.mark.parametrize("which,idx", [("a11", 0), ("a12", 1), ("a22", 2), ("r_omega", 3), ("kappa1", 4),
                                       ("kappa2", 5)])
def test_native_gradient_vs_central_differences(case, which, idx):
    prob, vbar, res = case
    eps = 1e-6
    fd = (_J(_perturbed(prob, which, eps), vbar) - _J(_perturbed(prob, which, -eps), vbar)) / (2 * eps)
    g = res["native"][idx]
    assert abs(g - fd) < 1e-6 * max(1.0, abs(fd)), (which, g, fd)


def test_omega_gradient_vs_central_differences(case):
    """Three weights: one in R_II next to R_I, one in R_II, one in R_III."""
    prob, vbar, res = case
    Nz, M1, M2 = prob.disc["N_z"], prob.disc["M1"], prob.disc["M2"]
    picks = [(Nz + M1, Nz), (Nz - M2 + 1, Nz + 1), (1, 2 * Nz - 3)]
    scale = np.max(np.abs(res["omega"]))
    for a, b in picks:
        eps = 1e-6
        fd = (_J(_perturbed(prob, (a, b), eps), vbar) - _J(_perturbed(prob, (a, b), -eps), vbar)) / (2 * eps)
        assert abs(res["omega"][a, b] - fd) < 1e-6 * max(scale, 1e-3), ((a, b), res["omega"][a, b], fd)
