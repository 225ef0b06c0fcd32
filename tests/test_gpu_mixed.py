"""GPU parity of the mixed form (FP32 iteration correlations on increments,
everything else FP64) against the FP64 oracle and the plain FP64 GPU path.

Bar: prices and the grid within 1e-6 in the relative metric
|a - b| / max(1, |b|); deltas within 1e-6 absolute.  The FP32 rounding enters
only through increments (Y^0 - V^{n-1}, then delta^k), whose size is
O(dt |A V|), so the expected error is about eps32 * T * |B V| ~ 1e-8: the tests
also print the observed values.
"""

import sys

import numpy as np
import pytest

import workloads
from oracle import integral, levy, output, scheme

pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-6


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


def _std(m):
    return (m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


def _oracle_problem(w):
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(levy.nts_from_std(*_std(w["model"])), h, w["r"])
    return scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"])


def test_mixed_nig64_matches_oracle(lp):
    """64 x 64 NIG, 32 steps: mixed GPU grid, prices and deltas vs the oracle."""
    _note("mixed nig64")
    w = workloads.workload("nig64")
    plan = lp.plan_from_workload(w, precision="fp32conv")
    V = plan.solve()
    prob = _oracle_problem(w)
    Vo, _ = scheme.solve(prob, tol=1e-14)
    eg = _rel(V.cpu().numpy(), Vo)
    spots = workloads.spot_pairs(64, seed=1)
    pg, dg = plan.price(V, spots, with_delta=True)
    po, do = output.prices(Vo, prob.y_lo, prob.h, w["K"], spots, with_delta=True)
    ep = _rel(pg.cpu().numpy(), po)
    ed = float(np.max(np.abs(dg.cpu().numpy() - do)))
    _note("mixed nig64: grid %.2e prices %.2e deltas %.2e" % (eg, ep, ed))
    assert eg < TOL_MIXED and ep < TOL_MIXED and ed < TOL_MIXED
    assert plan.info()["max_step_iters"] <= 20


@pytest.mark.parametrize("n", [41, 50])
def test_mixed_ragged_sizes(lp, n):
    _note("mixed ragged n=%d" % n)
    w = workloads.workload("nig64", n=n, N_t=10, y_lo=-2.5, y_hi=2.5)
    Vg = lp.plan_from_workload(w, precision="fp32conv").solve().cpu().numpy()
    Vo, _ = scheme.solve(_oracle_problem(w), tol=1e-14)
    e = _rel(Vg, Vo)
    _note("mixed ragged n=%d: grid %.2e" % (n, e))
    assert e < TOL_MIXED


def test_mixed_steps_prefix(lp):
    """Inside and after the damped block, and marches that end between two
    FP64 anchors of B V^{n-1} (every 8 steps by default)."""
    w = workloads.workload("nig64", n=40, N_t=16, y_lo=-2.5, y_hi=2.5)
    plan = lp.plan_from_workload(w, precision="fp32conv")
    prob = _oracle_problem(w)
    for k in (0, 1, 4, 7, 9, 13):
        _note("mixed solve_steps k=%d" % k)
        Vg = plan.solve_steps(k).cpu().numpy()
        Vo, _ = scheme.solve(prob, tol=1e-14, n_steps=k)
        assert _rel(Vg, Vo) < TOL_MIXED, k


@pytest.mark.parametrize("anchor", [1, 3, 8, 40])
def test_mixed_anchor_spacing(lp, anchor):
    """B V^{n-1} carried between FP64 anchors every `anchor` steps (40: only the
    first step of the march is anchored): 64 x 64 NIG, 32 steps, vs the oracle."""
    _note("mixed anchor every %d" % anchor)
    w = workloads.workload("nig64")
    plan = lp.plan_from_workload(w, precision="fp32conv", mixed_anchor=anchor)
    Vg = plan.solve().cpu().numpy()
    Vo, _ = scheme.solve(_oracle_problem(w), tol=1e-14)
    e = _rel(Vg, Vo)
    _note("mixed anchor every %d: grid %.2e, iterations %d" % (anchor, e, plan.info()["total_iters"]))
    assert e < TOL_MIXED


def test_mixed_range_restart_between_anchors(lp):
    """A march resumed at a step that is not a multiple of the anchor spacing
    anchors its own first step: steps 0..5 then 5..16 equal 0..16 within the bar."""
    _note("mixed solve_range restart at step 5")
    w = workloads.workload("nig64", n=40, N_t=16, y_lo=-2.5, y_hi=2.5)
    plan = lp.plan_from_workload(w, precision="fp32conv")
    n_steps = plan.info()["n_steps"]
    mid = plan.solve_steps(5)
    Vr = plan.solve_range(5, n_steps, mid).cpu().numpy()
    Vo, _ = scheme.solve(_oracle_problem(w), tol=1e-14)
    assert _rel(Vr, Vo) < TOL_MIXED


def test_mixed_anchor_rejects_negative(lp):
    with pytest.raises(lp.LpideError):
        lp.plan_from_workload(workloads.workload("nig64", n=16, N_t=2), precision="fp32conv", mixed_anchor=-1)


def test_mixed_fv512_first_steps_matches_oracle(lp):
    """The 512 x 512 finite-variation workload: the mixed state after the damped
    block and four main steps against the oracle."""
    _note("mixed fv512 first 8 steps")
    w = workloads.workload("fv512")
    Vg = lp.plan_from_workload(w, precision="fp32conv").solve_steps(8).cpu().numpy()
    Vo, _ = scheme.solve(_oracle_problem(w), tol=1e-14, inner="bicgstab", n_steps=8)
    e = _rel(Vg, Vo)
    _note("mixed fv512 8 steps: grid %.2e" % e)
    assert e < TOL_MIXED


def test_mixed_vs_plain_fv512_full_march(lp):
    """The full 256-step fv512 march, mixed vs plain FP64 on the GPU, at 64
    seeded spot pairs uniform in [80, 120]^2: prices and both deltas."""
    _note("mixed vs plain fv512 full march")
    w = workloads.workload("fv512")
    spots = workloads.spot_pairs(64, seed=7)
    res = {}
    for prec in ("fp64", "fp32conv"):
        plan = lp.plan_from_workload(w, precision=prec)
        V = plan.solve()
        p, d = plan.price(V, spots, with_delta=True)
        res[prec] = (V.cpu().numpy(), p.cpu().numpy(), d.cpu().numpy(), plan.info())
    eg = _rel(res["fp32conv"][0], res["fp64"][0])
    ep = _rel(res["fp32conv"][1], res["fp64"][1])
    ed = float(np.max(np.abs(res["fp32conv"][2] - res["fp64"][2])))
    _note("mixed vs plain fv512: grid %.2e prices %.2e deltas %.2e; iterations %d vs %d" % (
        eg, ep, ed, res["fp32conv"][3]["total_iters"], res["fp64"][3]["total_iters"]))
    assert eg < TOL_MIXED and ep < TOL_MIXED and ed < TOL_MIXED


def test_mixed_has_no_effect_without_jumps(lp):
    """With a zero Levy measure the precision switch changes nothing (no B)."""
    _note("mixed without jumps")
    g = lp.make_grid(48, -2.0, 2.0)
    lv = lp.levy_black_scholes(0.03, (0.09, 0.024, 0.04))
    pay = lp.make_payoff("put_1", 100.0, 1.0)
    a = lp.Plan(g, lv, pay, M=16).solve().cpu().numpy()
    b = lp.Plan(g, lv, pay, M=16, precision="fp32conv").solve().cpu().numpy()
    assert np.array_equal(a, b)
