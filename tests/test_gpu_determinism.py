"""Bitwise reproducibility on the GPU: the same inputs give the same bytes.

Every reduction of the march is order-independent (the stopping rule takes a
maximum, the adjoint accumulates per row and per spectral column in a fixed
order), so a solve, a batch, the correlation and the adjoint repeated on the
same plan return identical results, with graph replay and without.
"""

import sys

import numpy as np
import pytest

import workloads

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


@pytest.mark.parametrize("precision", ["fp64", "fp32conv"])
def test_solve_twice_is_bitwise_equal(lp, precision):
    import torch
    _note("determinism: fv512 %s solved twice" % precision)
    plan = lp.plan_from_workload(workloads.workload("fv512"), precision=precision)
    a = plan.solve()
    b = plan.solve()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    other = lp.plan_from_workload(workloads.workload("fv512"), precision=precision)
    assert torch.equal(other.solve(), a)          # a fresh plan of the same workload too


def test_batch_and_correlation_twice_are_bitwise_equal(lp):
    import torch
    draws = workloads.batch_draw(256, seed=3)[:6]
    _note("determinism: batch of %d draws twice, correlation twice" % len(draws))
    plans = [lp.plan_from_workload(d) for d in draws]
    batch = lp.Batch(plans)
    x = batch.solve()
    y = batch.solve()
    torch.cuda.synchronize()
    assert all(torch.equal(p, q) for p, q in zip(x, y))
    v = torch.from_numpy(workloads.random_grid(plans[0].n, seed=3)).cuda()
    assert torch.equal(plans[0].apply_B(v), plans[0].apply_B(v))


def test_adjoint_twice_is_bitwise_equal(lp):
    import torch
    w = workloads.workload("nig64", n=40, N_t=12, y_lo=-2.5, y_hi=2.5)
    _note("determinism: adjoint twice")
    plan = lp.plan_from_workload(w)
    vbar = torch.from_numpy(np.random.default_rng(2).standard_normal((w["n"], w["n"]))).cuda()
    _, n1, _ = plan.adjoint(vbar, checkpoint_every=4)
    _, n2, _ = plan.adjoint(vbar, checkpoint_every=4)
    assert np.array_equal(n1, n2)


def test_price_space_march_twice_is_bitwise_equal(lp):
    """The price-space plan, with the paper's iteration and with Anderson
    mixing, whose inner products are summed per block and then over the
    blocks in a fixed order: two marches, and a fresh plan, give the same
    bytes."""
    import csv
    import os
    import torch
    gold = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "table1_params.csv")
    with open(gold) as f:
        q = {r["name"]: r for r in csv.DictReader(line for line in f if not line.startswith("#"))}["NIG1"]
    lv = lp.levy_nts(float(q["alpha"]), float(q["delta"]), float(q["lambda"]), (float(q["eta1"]), float(q["eta2"])),
                     (float(q["rho11"]), float(q["rho12"]), float(q["rho22"])), float(q["r"]))
    pay = lp.make_payoff("put_avg", float(q["K"]), float(q["T"]))
    for accel in (0, 4):
        _note("determinism: price-space NIG1 N_x=48 accel=%d twice" % accel)
        mk = lambda: lp.PsPlan(lp.make_ps_grid(48, 700.0, c=45.0189), lv, pay, N_t=24, tol=1e-11, accel=accel)
        plan = mk()
        a = plan.solve()
        b = plan.solve()
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        assert torch.equal(mk().solve(), a)
