"""GPU parity of the benchmarked path over its whole length: the fv512 workload
(512 x 512 on [-4, 4]^2, alpha = 0.3, 256 time steps, 259 step-list entries)
marched by the library's default FP64 path -- the explicit part from the
previous step's equation, B Y^0 by linearity and the slots issued without the
kernels that would exit once every step in them is steady -- against the
oracle's full march (tests/golden/oracle_fv512.npz, written by
tests/golden/make_oracle_fv512.py, which calls only the oracle).

Bars: FP64 within 1e-10 in |a - b| / max(1, |b|) on the 64 x 64 sampled nodes
after 4, 8, 32, 96 and 259 entries, prices within 1e-10 relative and deltas
within 1e-10 absolute at 64 seeded spot pairs; the mixed form (FP32
correlation) within 1e-6 on the same quantities.  The Delta and Gamma surfaces
of the final grid (second-order differences, as in Sec. 4) on the sampled
nodes, each relative to its largest value: FP64 within 1e-10, mixed within
1e-6 (measured: about 1e-12 and 3e-8).
"""

import os
import sys

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_fv512.npz")


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


@pytest.fixture(scope="module")
def gold():
    return np.load(GOLDEN)


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.maximum(1.0, np.abs(b))))


GREEKS = ("delta1", "delta2", "gamma11", "gamma12", "gamma22")


def _check_final(plan, V, g, bar, tag, greek_bar=None):
    idx = g["idx"]
    e = _rel(V.cpu().numpy()[np.ix_(idx, idx)], g["V_259"])
    p, d = plan.price(V, g["spots"], with_delta=True)
    ep = _rel(p.cpu().numpy(), g["price"])
    ed = float(np.max(np.abs(d.cpu().numpy() - g["delta"])))
    _note("%s: grid %.2e prices %.2e deltas %.2e" % (tag, e, ep, ed))
    assert e < bar and ep < bar and ed < bar
    if greek_bar is not None:
        gs = plan.greeks(V).cpu().numpy()[:, idx][:, :, idx]
        eg = [float(np.max(np.abs(gs[q] - g["greeks"][q])) / np.max(np.abs(g["greeks"][q]))) for q in range(5)]
        _note("%s: Greeks %s" % (tag, ", ".join("%s %.2e" % kv for kv in zip(GREEKS, eg))))
        assert max(eg) < greek_bar


@pytest.mark.parametrize("fft_size", [0, 768])
def test_fv512_full_march_fp64_vs_oracle(lp, gold, fft_size):
    """Every stored prefix and the whole march, on the automatic transform side
    (1024) and on 768 = 3 * 256."""
    w = workloads.workload("fv512")
    plan = lp.plan_from_workload(w, fft_size=fft_size)
    idx = gold["idx"]
    for e in gold["entries"]:
        e = int(e)
        if e == 259:
            continue
        _note("fv512 fp64 L=%d first %d entries" % (plan.info()["L"], e))
        V = plan.solve_steps(e).cpu().numpy()
        err = _rel(V[np.ix_(idx, idx)], gold["V_%d" % e])
        _note("  sampled grid %.2e" % err)
        assert err < 1e-10, e
    _note("fv512 fp64 L=%d whole march" % plan.info()["L"])
    V = plan.solve()
    assert plan.info()["n_steps"] == 259
    _check_final(plan, V, gold, 1e-10, "fv512 fp64 L=%d" % plan.info()["L"], greek_bar=1e-10)


def test_fv512_full_march_mixed_vs_oracle(lp, gold):
    w = workloads.workload("fv512")
    _note("fv512 mixed whole march")
    plan = lp.plan_from_workload(w, precision="fp32conv")
    V = plan.solve()
    _check_final(plan, V, gold, 1e-6, "fv512 mixed", greek_bar=1e-6)


def test_fv512_full_march_batched_lean_slots(lp, gold):
    """The same march through a one-plan batch with 4-step slots, so that slots
    without the exiting kernels start right after the first main steps, and a
    two-plan batch (the plan next to a copy of itself)."""
    w = workloads.workload("fv512")
    plan = lp.plan_from_workload(w)
    _note("fv512 one-plan batch, 4-step slots")
    b = lp.Batch([plan], slots=4)
    V = b.solve()[0]
    _check_final(plan, V, gold, 1e-10, "fv512 batch slots=4")
    b.close()
    other = lp.plan_from_workload(w)
    _note("fv512 two-plan batch, 8-step slots")
    b2 = lp.Batch([plan, other], slots=8)
    Vs = b2.solve()
    for q, Vq in enumerate(Vs):
        _check_final(plan, Vq, gold, 1e-10, "fv512 batch of two, member %d" % q)
    b2.close()
