"""The allocation-free correlation lpide_apply_B_noalloc (static device scratch,
no allocation in the call) through the C ABI, against lpide_apply_B on the
same plans and inputs: the same kernels on the same data, so the results must
agree bit for bit.  Two calls in a row, the second on a smaller grid (the
scratch keeps the first call's contents, which the second must not see); a
plan whose intermediate exceeds the scratch is refused before anything runs;
a plan without jumps gets zeros.
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


def test_noalloc_equals_apply_B_twice_shrinking(lp):
    import torch
    for n, half, seed in ((700, 3.0, 11), (130, 2.5, 12)):
        _note("apply_B_noalloc n=%d" % n)
        w = workloads.workload("nig64", n=n, y_lo=-half, y_hi=half)
        plan = lp.plan_from_workload(w)
        v = torch.from_numpy(workloads.random_grid(n, seed=seed)).cuda()
        out = torch.full_like(v, float("nan"))
        plan.apply_B_noalloc(v, out)
        ref = plan.apply_B(v)
        torch.cuda.synchronize()
        assert torch.isfinite(out).all()
        assert torch.equal(out, ref), float((out - ref).abs().max())
        _note("  L=%d: bit-identical to lpide_apply_B" % plan.info()["L"])


def test_noalloc_refuses_oversized_plans(lp):
    import torch
    w = workloads.workload("nig2048_m")
    plan = lp.plan_from_workload(w, fft_size=4096)      # 2048 x 2049 x 16 bytes > 64 MiB
    n = w["n"]
    v = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    out = torch.full_like(v, 7.0)
    _note("apply_B_noalloc oversized plan")
    with pytest.raises(lp.LpideError) as ei:
        plan.apply_B_noalloc(v, out)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert bool((out == 7.0).all())


def test_noalloc_without_jumps_is_zero(lp):
    import torch
    n = 48
    g = lp.make_grid(n, -2.0, 2.0)
    lv = lp.levy_black_scholes(0.03, (0.09, 0.012, 0.04))
    plan = lp.Plan(g, lv, lp.make_payoff("put_avg", 100.0, 1.0), theta=0.5, M=8)
    v = torch.from_numpy(np.ones((n, n))).cuda()
    out = torch.full_like(v, 3.0)
    plan.apply_B_noalloc(v, out)
    torch.cuda.synchronize()
    assert bool((out == 0.0).all())
