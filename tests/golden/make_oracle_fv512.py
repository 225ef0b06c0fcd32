"""Write the oracle's full march of the fv512 workload (512 x 512 on [-4, 4]^2,
256 time steps, so 259 step-list entries with the damped block) to
oracle_fv512.npz:

    python tests/golden/make_oracle_fv512.py

Calls only the oracle (FP64, BiCGSTAB inner solves to 1e-15, fixed-point tol
1e-14); about three minutes on four cores.  Stored arrays:
  idx              the sampled node indices 0, 8, ..., 504 (per axis)
  entries          step-list entries (1-based counts) at which the grid is kept
  V_<e>            the grid after the first e entries on the sampled nodes
  spots            64 seeded spot pairs (workloads.spot_pairs(64, seed=1))
  price, delta     prices and spot deltas there after the whole march
  greeks           the Delta and Gamma surfaces of the final grid (delta1, delta2,
                   gamma11, gamma12, gamma22) on the sampled nodes
  iters            fixed-point iterations of every entry
"""

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads  # noqa: E402
from oracle import integral, levy, output, scheme  # noqa: E402

STRIDE = 8
# the damped block, the first 32-entry batch, two more batches, the whole march
ENTRIES = (4, 8, 32, 96, 259)


def make(name="fv512"):
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
        if s + 1 in ENTRIES:
            kept["V_%d" % (s + 1)] = V[np.ix_(idx, idx)].copy()
            print("  entry %d at %.0f s" % (s + 1, time.time() - t0), flush=True)

    V, iters = scheme.solve(prob, tol=1e-14, inner="bicgstab", on_step=keep)
    spots = workloads.spot_pairs(64, seed=1)
    price, delta = output.prices(V, prob.y_lo, h, w["K"], spots, with_delta=True)
    greeks = np.stack([g[np.ix_(idx, idx)] for g in output.greeks_on_grid(V, prob.y_lo, h, w["K"])])
    out = os.path.join(HERE, "oracle_%s.npz" % name)
    np.savez(out, idx=idx, entries=np.array(ENTRIES), spots=spots, price=price, delta=delta, greeks=greeks,
             iters=np.array(iters), name=name, **kept)
    print("%s: %d entries in %.0f s -> %s" % (name, len(iters), time.time() - t0, out), flush=True)


if __name__ == "__main__":
    make()
