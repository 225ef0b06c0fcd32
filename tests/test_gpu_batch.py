"""GPU tests of the batched form: many plans with uneven grids, parameters,
pay-offs and step counts marched together (one launch per kernel and group,
optionally replayed from hipGraphs), against the same plans marched alone and
against the FP64 oracle.

Bars: batch vs solo within 1e-12 in |a - b| / max(1, |b|) for FP64 plans
(the group may chunk the axis-1 line solves differently, which changes
rounding only) and 1e-6 for mixed plans (there a different rounding of the
iterates changes the FP32 increments, so the two marches differ at the level
of the FP32 correlation error, about 1e-9); batch vs oracle within 1e-10
(plain) and 1e-6 (mixed).
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


def _bar(precision):
    return 1e-12 if precision == "fp64" else 1e-6


def _mixed_workloads():
    """Seven small plans: four grid sizes (two transform sizes), finite and
    infinite variation, both correlation signs, several pay-offs, maturities
    and step counts, two precisions."""
    ws = []
    rng = np.random.default_rng(11)
    for q, (n, payoff) in enumerate([(40, "put_avg"), (48, "call_avg"), (64, "put_1"), (40, "exchange"),
                                     (56, "put_avg"), (64, "call_1"), (48, "put_avg")]):
        w = workloads.workload("nig64", n=n, y_lo=-2.5, y_hi=2.5, payoff=payoff,
                               alpha=float(rng.uniform(0.2, 0.6)), corr=float(rng.uniform(-0.6, 0.6)),
                               sigma1=float(rng.uniform(0.15, 0.3)), sigma2=float(rng.uniform(0.15, 0.3)),
                               K=float(rng.uniform(90, 110)), T=float(rng.uniform(0.5, 1.5)),
                               N_t=int(rng.integers(6, 14)))
        ws.append((w, "fp32conv" if q in (2, 5) else "fp64"))
    return ws


def _oracle(w):
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    prob = scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"])
    return scheme.solve(prob, tol=1e-14)[0]


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_solo_and_oracle(lp, use_graph):
    ws = _mixed_workloads()
    _note("batch of %d plans, graph=%s" % (len(ws), use_graph))
    plans = [lp.plan_from_workload(w, precision=pr) for w, pr in ws]
    batch = lp.Batch(plans, use_graph=use_graph, slots=4)
    groups = batch.groups()
    assert len(groups) >= 2 and sum(g["n_plans"] for g in groups) == len(ws)
    outs = [o.cpu().numpy() for o in batch.solve()]
    infos = [p.info() for p in plans]
    for (w, pr), p, vb, ib in zip(ws, plans, outs, infos):
        vs = p.solve().cpu().numpy()
        assert _rel(vb, vs) < _bar(pr), (w["n"], pr)
        assert ib["n_steps"] == w["N_t"] + 3 and ib["total_iters"] > 0
    for q in (0, 2):
        w, pr = ws[q]
        _note("batch member %d vs oracle (%s)" % (q, pr))
        e = _rel(outs[q], _oracle(w))
        assert e < (1e-10 if pr == "fp64" else 1e-6), (q, e)


def test_batch_with_black_scholes_member(lp):
    """A plan without jumps forms its own group beside the jump plans."""
    _note("batch with a zero-Levy member")
    w = workloads.workload("nig64", n=48, y_lo=-2.0, y_hi=2.0, N_t=12)
    g = lp.make_grid(48, -2.0, 2.0)
    bs = lp.Plan(g, lp.levy_black_scholes(0.03, (0.09, 0.024, 0.04)), lp.make_payoff("put_1", 100.0, 1.0), M=12)
    jp = lp.plan_from_workload(w)
    batch = lp.Batch([bs, jp], use_graph=True)
    vb = [o.cpu().numpy() for o in batch.solve()]
    assert len(batch.groups()) == 2
    assert _rel(vb[0], bs.solve().cpu().numpy()) < 1e-12
    assert _rel(vb[1], jp.solve().cpu().numpy()) < 1e-12


def test_batch_tune_then_solve(lp):
    """The autotuner times its candidates and keeps one per group; the tuned
    batch still reproduces the solo results."""
    ws = _mixed_workloads()[:4]
    _note("batch tune")
    plans = [lp.plan_from_workload(w, precision=pr) for w, pr in ws]
    batch = lp.Batch(plans)
    groups = batch.tune(trial_steps=6)
    for g in groups:
        assert g["trial_ms"] > 0 and g["P_cols"] in (8, 16, 32, 64, 128, 256) and g["slots"] in (16, 32)
    outs = [o.cpu().numpy() for o in batch.solve()]
    for (w, pr), p, vb in zip(ws, plans, outs):
        e = _rel(vb, p.solve().cpu().numpy())
        _note("tuned batch member n=%d %s: %.2e" % (w["n"], pr, e))
        assert e < _bar(pr)


def test_batch_forced_recovery(lp):
    """A member whose steps need more iterations than predicted is completed
    while the other members are held; everything still matches solo runs."""
    _note("batch recovery")
    w1 = workloads.workload("nig64", n=40, N_t=8, y_lo=-2.5, y_hi=2.5)
    w2 = workloads.workload("nig64", n=40, N_t=10, y_lo=-2.5, y_hi=2.5, alpha=0.3)
    p1 = lp.plan_from_workload(w1, tol=1e-14)
    p2 = lp.plan_from_workload(w2)
    batch = lp.Batch([p1, p2], use_graph=True, slots=8)
    v1, v2 = [o.cpu().numpy() for o in batch.solve()]
    assert _rel(v1, p1.solve().cpu().numpy()) < 1e-12
    assert _rel(v2, p2.solve().cpu().numpy()) < 1e-12


def test_batched_draw_sample(lp):
    """Eight draws of the batched workload recipe (grids from {128, 256}^2
    here), marched in one batch: finite, and each equal to its solo march."""
    import torch
    draws = [d for d in workloads.batch_draw(64, seed=3) if d["n"] <= 256][:8]
    _note("batched draw sample of %d" % len(draws))
    plans = [lp.plan_from_workload(d) for d in draws]
    batch = lp.Batch(plans)
    outs = batch.solve()
    for p, o in zip(plans, outs):
        assert torch.isfinite(o).all()
        assert _rel(o.cpu().numpy(), p.solve().cpu().numpy()) < 1e-12


def test_batched_recipe_16_draws_vs_oracle(lp):
    """The first 16 draws of the batched workload recipe (n = 128 to 1024 with
    six at 512 and one at 1024, drawn model, strike and maturity) in one batch
    with 4-step slots (slots without the exiting kernels from the first main
    steps on), against the oracle's state after six step-list
    entries (tests/golden/oracle_batch.npz, written by
    tests/golden/make_oracle_batch.py, which calls only the oracle), on 64 x 64
    sampled nodes each: within 1e-10."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_batch.npz")
    g = np.load(path)
    count, entries = int(g["count"]), int(g["entries"])
    draws = workloads.batch_draw(256, seed=3)[:count]
    assert {512, 1024} <= {d["n"] for d in draws}
    _note("batched recipe: %d draws, n %s, first %d entries" % (count, sorted({d["n"] for d in draws}), entries))
    plans = [lp.plan_from_workload(d) for d in draws]
    batch = lp.Batch(plans, slots=4)
    outs = batch.solve_steps(entries)
    worst = 0.0
    for q, o in enumerate(outs):
        idx = g["idx_%d" % q]
        err = _rel(o.cpu().numpy()[np.ix_(idx, idx)], g["V_%d" % q])
        worst = max(worst, err)
        assert err < 1e-10, (q, draws[q]["n"], err)
    _note("batched recipe vs oracle: worst sampled grid %.2e" % worst)


def test_plan_batch_one_call(lp):
    """lpide_plan_batch builds the plans and their batch from arrays in one call
    (the batch owns the plans); lpide_solve_batch marches them.  The results
    equal plans made and solved one by one."""
    import ctypes as C
    import torch
    from paper_2511_02700_amd import _lib
    cfg = [(40, "put_avg", 8, 0.5), (48, "spread", 10, 0.3), (64, "call_1", 6, 0.4)]
    _note("lpide_plan_batch of %d plans" % len(cfg))
    grids = (_lib.Grid * 3)()
    levys = (_lib.Levy * 3)()
    pays = (_lib.Payoff * 3)()
    Ms = (C.c_int32 * 3)()
    ws = []
    for q, (n, pay, M, alpha) in enumerate(cfg):
        w = workloads.workload("nig64", n=n, y_lo=-2.5, y_hi=2.5, payoff=pay, N_t=M, alpha=alpha)
        ws.append(w)
        m = w["model"]
        grids[q] = lp.make_grid(n, w["y_lo"], w["y_hi"])
        levys[q] = lp.levy_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"],
                                    m["alpha"], w["r"])
        pays[q] = lp.make_payoff(pay, w["K"], w["T"])
        Ms[q] = M
    o = _lib.Opts()
    lp.lib().lpide_opts_default(C.byref(o))
    o.stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    b = C.c_void_p()
    _lib.check(lp.lib().lpide_plan_batch(3, grids, levys, pays, 0.5, Ms, C.byref(o), C.byref(b)))
    try:
        outs = [torch.empty((n, n), dtype=torch.float64, device="cuda") for n, _, _, _ in cfg]
        ptrs = (C.c_void_p * 3)(*[t.data_ptr() for t in outs])
        _lib.check(lp.lib().lpide_solve_batch(b, ptrs))
        torch.cuda.synchronize()
        for w, t in zip(ws, outs):
            assert _rel(t.cpu().numpy(), lp.plan_from_workload(w).solve().cpu().numpy()) < 1e-12
    finally:
        _lib.check(lp.lib().lpide_batch_destroy(b))
