"""GPU edge cases of the march, through the C ABI, against the oracle on the
same inputs: the end points of theta (fully implicit theta = 1, where the
explicit part and its correlation vanish; fully explicit theta = 0, where the
implicit operator is the identity and the fixed point is reached at once),
the march without damping, a single time step, plans without jumps whose grid
fills the row transform (n equal to its side, the largest row buffer of the
line-row kernel), an empty spot list, the Greeks on the smallest grid and the
one-shot solve helper.

Bar: |a - b| / max(1, |b|) within 1e-10, as for the other marches.
"""

import sys

import numpy as np
import pytest

import workloads
from oracle import integral, levy, scheme

pytestmark = pytest.mark.gpu


def _note(msg):
    print("[gpu-case] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def lp():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no HIP device visible")
    import paper_2511_02700_amd as m
    m.lib()
    return m


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


def _oracle(w, damping=True):
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    prob = scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"], damping=damping)
    return scheme.solve(prob, tol=1e-14)[0]


@pytest.mark.parametrize("theta,damping", [(1.0, True), (1.0, False), (0.0, True), (0.5, False)])
def test_theta_end_points_and_damping(lp, theta, damping):
    w = workloads.workload("nig64", n=40, N_t=8, y_lo=-2.5, y_hi=2.5, theta=theta)
    _note("theta=%g damping=%s" % (theta, damping))
    plan = lp.plan_from_workload(w, damping=damping)
    assert plan.info()["n_steps"] == (w["N_t"] + 3 if damping else w["N_t"])
    assert _rel(plan.solve().cpu().numpy(), _oracle(w, damping)) < 1e-10


def test_single_time_step(lp):
    """M = 1: the step list is the damped block alone (four theta = 1 quarter steps)."""
    w = workloads.workload("nig64", n=40, N_t=1, y_lo=-2.5, y_hi=2.5)
    _note("single time step")
    plan = lp.plan_from_workload(w)
    assert plan.info()["n_steps"] == 4
    assert _rel(plan.solve().cpu().numpy(), _oracle(w)) < 1e-10


@pytest.mark.parametrize("n", [64, 256])
def test_no_jumps_grid_fills_the_row_transform(lp, n):
    """Without jumps the row kernels take the power of two >= n, here n itself:
    the line-row kernel's row buffer (n + T/2 + 1 values per row at E = 4) is
    at its largest."""
    s1, s2, c = 0.3, 0.2, 0.4
    cov = np.array([[s1 * s1, c * s1 * s2], [c * s1 * s2, s2 * s2]])
    _note("no jumps, n = %d" % n)
    g = lp.make_grid(n, -2.0, 2.0)
    plan = lp.Plan(g, lp.levy_black_scholes(0.03, (cov[0, 0], cov[0, 1], cov[1, 1])),
                   lp.make_payoff("put_1", 100.0, 1.0), theta=0.5, M=12)
    Vg = plan.solve().cpu().numpy()
    h = 4.0 / (n - 1)
    disc = integral.discretize(None, h, 0.03, sigma_bs=cov)
    prob = scheme.Problem(n, (-2.0, -2.0), h, disc, payoff="put_1", K=100.0, T=1.0, N_t=12, theta=0.5)
    Vo, _ = scheme.solve(prob, tol=1e-14)
    assert _rel(Vg, Vo) < 1e-10


def test_empty_spot_list_and_smallest_greeks(lp):
    """The smallest grid (n = 8): the march is finite, an empty spot list gives
    empty prices and a zero price cotangent, and the Greeks of a seeded grid
    equal the oracle's."""
    import torch
    from oracle import output
    w = workloads.workload("nig64", n=8, N_t=4, y_lo=-1.0, y_hi=1.0)
    _note("empty spot list, n = 8")
    plan = lp.plan_from_workload(w)
    V = plan.solve()
    assert torch.isfinite(V).all()
    assert plan.price(V, np.zeros((0, 2))).numel() == 0
    vb = plan.price_adjoint(np.zeros((0, 2)), np.zeros(0))
    assert vb.shape == (8, 8) and float(vb.abs().max()) == 0.0
    G = workloads.random_grid(8, seed=8)
    got = plan.greeks(torch.from_numpy(G).cuda()).cpu().numpy()
    ref = output.greeks_on_grid(G, (-1.0, -1.0), 2.0 / 7, 100.0)
    for q in range(5):
        assert np.max(np.abs(got[q] - ref[q])) <= 1e-12 * np.max(np.abs(ref[q]))


def test_one_shot_solve_helper(lp):
    """lp.solve (plan, march, destroy in one call) gives the oracle's grid."""
    w = workloads.workload("nig64", n=40, N_t=8, y_lo=-2.5, y_hi=2.5)
    _note("one-shot solve helper")
    m = w["model"]
    lv = lp.levy_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"],
                          w["r"])
    g = lp.make_grid(w["n"], w["y_lo"], w["y_hi"])
    pay = lp.make_payoff(w["payoff"], w["K"], w["T"])
    v = lp.solve(g, lv, pay, theta=w["theta"], M=w["N_t"], tol=w["tol"])
    assert tuple(v.shape) == (w["n"], w["n"])
    assert _rel(v.cpu().numpy(), _oracle(w)) < 1e-10


@pytest.mark.parametrize("damping", [True, False])
def test_products_without_the_correlation(lp, damping):
    """The FP64 march with the two products taken without the correlation
    (the default: the explicit part from the previous step's implicit equation,
    B Y^0 of the first iteration by linearity from the stored B V of the
    history) and with every product by the correlation (all_correlations) both
    give the oracle's grid.  The timing classes show which kernels ran: the
    explicit correlation in the first step of the march only, the identity
    kernel in every later step with theta < 1, and iteration 1 without the
    transform once every grid of the start value came from the march (damped
    sub-steps 1-3 and steps 7 on; without damping steps 4 on)."""
    w = workloads.workload("nig64", N_t=16)
    _note("products without the correlation, damping=%s" % damping)
    Vo = _oracle(w, damping)
    res = {}
    for allc in (False, True):
        plan = lp.plan_from_workload(w, damping=damping, all_correlations=allc)
        plan.solve()
        plan.set_timing(["expl_cols", "expl_id", "rows_lin"])
        V = plan.solve().cpu().numpy()
        st = plan.kernel_stats()
        n_steps = plan.info()["n_steps"]
        first_cn = 4 if damping else 0          # first theta = 1/2 step of the step list
        if allc:
            assert st["expl_cols"][0] == n_steps - first_cn and st["expl_id"][0] == 0
            assert st["rows_lin"][0] == 0
        else:
            assert st["expl_cols"][0] == (0 if damping else 1)
            assert st["expl_id"][0] == n_steps - first_cn - (0 if damping else 1)
            assert st["rows_lin"][0] == (3 + n_steps - 7 if damping else n_steps - 4)
        e = _rel(V, Vo)
        _note("all_correlations=%s: grid %.2e" % (allc, e))
        assert e < 1e-10
        res[allc] = V
    assert _rel(res[False], res[True]) < 1e-11
