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
