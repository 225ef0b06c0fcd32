"""GPU parity at the 2048 x 2048 size (transform side L = 3072): the four
workloads with alpha in {0.5, 0.3} and correlation -0.5 or +0.5, their state
after the damped block and one theta = 1/2 step (5 entries) and after 16
entries, against stored oracle values on the 256 x 256 sub-grid of every 8th
node (written by tests/golden/make_oracle_2048.py, which calls only the
oracle); the 16 entries also through a one-plan batch with 4-step slots, whose
slots after the first main steps run without the kernels that would exit; and
the full 1024-step march in the mixed form against the plain FP64 march.

Bars: plain FP64 within 1e-10 and mixed within 1e-6 in the metric
|a - b| / max(1, |b|); prices within 1e-6 relative, deltas 1e-6 absolute.
"""

import math
import os
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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


def _golden(name):
    path = os.path.join(GOLDEN, "oracle_2048_%s.npz" % name)
    if not os.path.exists(path):
        pytest.skip("oracle values for %s not generated (tests/golden/make_oracle_2048.py)" % name)
    return np.load(path)


NAMES = ["nig2048_m", "nig2048_p", "fv2048_m", "fv2048_p"]


@pytest.mark.parametrize("name", NAMES)
@pytest.mark.parametrize("precision,bar", [("fp64", 1e-10), ("fp32conv", 1e-6)])
def test_first_steps_2048_vs_oracle(lp, name, precision, bar):
    g = _golden(name)
    idx = g["idx"]
    plan = lp.plan_from_workload(workloads.workload(name), precision=precision)
    assert plan.info()["L"] == 3072
    for e in g["entries"]:
        e = int(e)
        _note("2048 %s %s first %d entries" % (name, precision, e))
        V = plan.solve_steps(e).cpu().numpy()
        err = _rel(V[np.ix_(idx, idx)], g["V_%d" % e])
        _note("2048 %s %s: sampled grid %.2e" % (name, precision, err))
        assert err < bar


@pytest.mark.parametrize("name", NAMES)
def test_first_steps_2048_batched_lean_slots(lp, name):
    g = _golden(name)
    idx, e = g["idx"], int(max(g["entries"]))
    plan = lp.plan_from_workload(workloads.workload(name))
    _note("2048 %s one-plan batch, 4-step slots, first %d entries" % (name, e))
    b = lp.Batch([plan], slots=4)
    V = b.solve_steps(e)[0].cpu().numpy()
    b.close()
    err = _rel(V[np.ix_(idx, idx)], g["V_%d" % e])
    _note("2048 %s batch: sampled grid %.2e" % (name, err))
    assert err < 1e-10


@pytest.mark.parametrize("name", ["nig2048_m", "fv2048_p"])
def test_full_march_2048_mixed_vs_plain(lp, name):
    """1024 steps at 2048^2: mixed vs plain FP64 at the 256 x 256 sampled nodes
    and at 64 seeded spot pairs; both finite and within no-arbitrage bounds."""
    import torch
    _note("2048 %s full march, fp64 and mixed" % name)
    w = workloads.workload(name)
    spots = workloads.spot_pairs(64, seed=2)
    idx = np.arange(0, w["n"], 8)
    res = {}
    for prec in ("fp64", "fp32conv"):
        plan = lp.plan_from_workload(w, precision=prec)
        V = plan.solve()
        assert torch.isfinite(V).all()
        p, d = plan.price(V, spots, with_delta=True)
        res[prec] = (V.cpu().numpy()[np.ix_(idx, idx)], p.cpu().numpy(), d.cpu().numpy())
        del V
    eg = _rel(res["fp32conv"][0], res["fp64"][0])
    ep = _rel(res["fp32conv"][1], res["fp64"][1])
    ed = float(np.max(np.abs(res["fp32conv"][2] - res["fp64"][2])))
    _note("2048 %s mixed vs plain: grid %.2e prices %.2e deltas %.2e" % (name, eg, ep, ed))
    assert eg < 1e-6 and ep < 1e-6 and ed < 1e-6
    K, r, T = w["K"], w["r"], w["T"]
    pr = res["fp64"][1]
    lower = np.maximum(K * math.exp(-r * T) - spots.mean(axis=1), 0.0)
    assert np.all(pr >= lower - 1e-6) and np.all(pr <= K * math.exp(-r * T))
