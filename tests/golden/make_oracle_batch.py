"""Write the oracle's state of the first 16 draws of the batched workload recipe
(workloads.batch_draw(256, seed=3): n in {128, 256, 512, 1024}, drawn model,
strike and maturity per draw) after the first ENTRIES step-list entries (the
four damped quarter steps and two theta = 1/2 steps), on the 64 x 64 sub-grid
of every (n / 64)-th node, to oracle_batch.npz:

    python tests/golden/make_oracle_batch.py

Calls only the oracle (FP64, BiCGSTAB inner solves, tol 1e-14); about five
minutes on eight cores.  Stored arrays: V_<q> (64 x 64) and idx_<q> (the
sampled node indices) for draw q, entries, and count.
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

COUNT = 16
ENTRIES = 6


def main():
    out = {}
    t0 = time.time()
    for q, w in enumerate(workloads.batch_draw(256, seed=3)[:COUNT]):
        m = w["model"]
        p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
        n = w["n"]
        h = (w["y_hi"] - w["y_lo"]) / (n - 1)
        d = integral.discretize(p, h, w["r"])
        prob = scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, payoff=w["payoff"], K=w["K"], T=w["T"],
                              N_t=w["N_t"], theta=w["theta"])
        V, iters = scheme.solve(prob, tol=1e-14, inner="bicgstab", n_steps=ENTRIES)
        idx = np.arange(0, n, n // 64)
        out["V_%d" % q] = V[np.ix_(idx, idx)]
        out["idx_%d" % q] = idx
        print("draw %d: n %d, iterations %s, %.0f s" % (q, n, iters, time.time() - t0), flush=True)
    path = os.path.join(HERE, "oracle_batch.npz")
    np.savez(path, entries=ENTRIES, count=COUNT, **out)
    print("-> %s" % path, flush=True)


if __name__ == "__main__":
    main()
