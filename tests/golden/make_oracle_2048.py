"""Write the oracle's state of the 2048 x 2048 workloads after the first
step-list entries (the four damped quarter steps, then theta = 1/2 steps), on
the 256 x 256 sub-grid of every 8th node per axis (indices 0, 8, ..., 2040),
to oracle_2048_<name>.npz.

    python tests/golden/make_oracle_2048.py [nig2048_m nig2048_p fv2048_m fv2048_p]

Calls only the oracle (FP64, BiCGSTAB inner solves, tol 1e-14); about half an
hour per workload on eight cores.  The stored arrays: V_<e> (256 x 256, the
grid after the first e entries) for e in entries, idx (the sampled node
indices), iters (fixed-point iterations per entry) and the workload name.
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import integral, levy, scheme  # noqa: E402

ENTRIES = (5, 16)     # the damped block and one main step; then 11 more main steps
STRIDE = 8


def make(name):
    w = workloads.workload(name)
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    prob = scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"], N_t=w["N_t"],
                          theta=w["theta"])
    idx = np.arange(0, n, STRIDE)
    kept = {}
    t0 = time.time()

    def keep(s, V):
        print("  %s entry %d at %.0f s" % (name, s + 1, time.time() - t0), flush=True)
        if s + 1 in ENTRIES:
            kept["V_%d" % (s + 1)] = V[np.ix_(idx, idx)].copy()

    _, iters = scheme.solve(prob, tol=1e-14, inner="bicgstab", n_steps=max(ENTRIES), on_step=keep)
    out = os.path.join(HERE, "oracle_2048_%s.npz" % name)
    np.savez(out, idx=idx, entries=np.array(ENTRIES), name=name, iters=np.array(iters), **kept)
    print("%s: %d entries in %.0f s, iterations %s -> %s" % (name, len(iters), time.time() - t0, iters, out),
          flush=True)


if __name__ == "__main__":
    for nm in (sys.argv[1:] or ["nig2048_m", "nig2048_p", "fv2048_m", "fv2048_p"]):
        make(nm)
