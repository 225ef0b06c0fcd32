"""GPU tests of the Greeks on the grid (lpide_greeks) and of the spread-call
pay-off, through the C ABI, against the oracle (oracle/output.py,
oracle/scheme.py) on the same seeded inputs.

Bars: the Greek surfaces elementwise within 1e-12 of each surface's largest
magnitude (both sides apply the same difference stencils in FP64; the
differences of O(h^-2) amplify rounding only); the spread march within 1e-10
in |a - b| / max(1, |b|), as for every other pay-off.
"""

import sys

import numpy as np
import pytest

import workloads
from oracle import integral, levy, output, scheme

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


def _oracle_problem(w):
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    return scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"])


def _check_greeks(lp, plan, V, w):
    import torch
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    got = plan.greeks(torch.from_numpy(np.ascontiguousarray(V)).cuda()).cpu().numpy()
    ref = output.greeks_on_grid(V, (w["y_lo"], w["y_lo"]), h, w["K"])
    for q, name in enumerate(("delta1", "delta2", "gamma11", "gamma12", "gamma22")):
        err = np.max(np.abs(got[q] - ref[q])) / np.max(np.abs(ref[q]))
        assert err < 1e-12, (name, err)


@pytest.mark.parametrize("n", [41, 64])
def test_greeks_random_grid(lp, n):
    """Seeded random grid, ragged and even sizes (edges and corners included)."""
    _note("greeks random grid n=%d" % n)
    w = workloads.workload("nig64", n=n, y_lo=-2.0, y_hi=2.0)
    plan = lp.plan_from_workload(w)
    _check_greeks(lp, plan, workloads.random_grid(n, seed=n), w)


def test_greeks_of_oracle_solution(lp):
    """The Greeks of the oracle's own march of the spread call (a smooth grid
    with a kink region)."""
    w = workloads.workload("nig64", n=40, N_t=8, y_lo=-2.5, y_hi=2.5, payoff="spread")
    _note("greeks of the oracle's spread solution")
    V, _ = scheme.solve(_oracle_problem(w), tol=1e-14)
    plan = lp.plan_from_workload(w)
    _check_greeks(lp, plan, V, w)


@pytest.mark.parametrize("n", [40, 57])
def test_spread_matches_oracle(lp, n):
    """The spread call under the NTS model: the whole march against the oracle."""
    w = workloads.workload("nig64", n=n, N_t=10, y_lo=-2.5, y_hi=2.5, payoff="spread")
    _note("spread march n=%d" % n)
    Vg = lp.plan_from_workload(w).solve().cpu().numpy()
    Vo, _ = scheme.solve(_oracle_problem(w), tol=1e-14)
    err = float(np.max(np.abs(Vg - Vo) / np.maximum(1.0, np.abs(Vo))))
    assert err < 1e-10, err
