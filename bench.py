#!/usr/bin/env python3
"""Benchmark of the MI355X time march (one GPU).

A bench "step" is one full solve of the workload: the whole hot path (explicit
part, semi-Lagrangian gather, extrapolated start, fixed-point iterations of
FFT correlation + stencil residual + line solves + update, for every entry of
the step list including the damped block) from V^0 to V^{N_t}, with the inputs
resident in device memory.  value = n^2 * N_t * steps / (timed wall time), in
grid-point time steps per second.

Default workload: nig2048_m, the 2048 x 2048 NIG case (alpha = 1/2,
correlation -0.5) on [-5, 5]^2 with 1024 time steps, theta = 1/2, fixed-point
tol 1e-12, FP64 (with the library's defaults: the explicit part from the
previous step's equation and B Y^0 of the first iteration from stored
products, both exact at the fixed point).  Its working set (grids, the
transposed intermediate and the spectrum: about 0.7 GB) exceeds the caches, so
the kernels are measured against HBM.

Printed (one JSON line): the metric, the roofline of the dominant kernel
(algorithmic bytes per launch / mean launch time from HIP events bound to the
kernel's own dispatches on the plan's stream, over the timed solves), the same
for the correlation's column pass and for the correlation as a whole, the
other precision timed beside it with the mixed-vs-plain differences (prices,
deltas, Delta/Gamma surfaces), the other candidate transform side, and a CPU
baseline: the FP64 oracle timed on this host on a bounded sample of the same
workload (in a child process, while the GPU extras run), and the plan time.
Unless --no-extras: the 512^2 finite-variation workload (fv512), the paper's
Table 3 prices against GPU marches on the log grid, the price-space plan (the
paper's own discretization) on each Table 1 set at the largest grid one
workgroup's transform holds and (unless --no-paper-grids) on the paper's own
grids, the adjoint form on its 1024^2 workload (ratio to the forward, with
checkpoints every 32 steps and with every state kept), a vectorised device copy
as the bandwidth reference, and the batched form on all 256 draws of the
batched recipe (autotuned, against solo solves).
"""

import argparse
import json
import math
import os
import resource
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "grid-pt-steps/s + FFT-conv %HBM roofline, mixed vs plain FP64 at ≤1e-6 rel"
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, 8 TB/s


def algorithmic_bytes(cls, n, L, mixed=False):
    """Bytes a kernel class must move per launch: 8 bytes per FP64 real, c = 8
    (FP64) or 4 (mixed form) per real of the correlation data; the intermediate
    X holds n x (L/2+1) complex values, the spectrum L x (L/2+1)."""
    hc = L // 2 + 1
    c = 4 if mixed else 8
    return {
        # read + write X, read the spectrum
        "cols": 2 * c * hc * (2 * n + L),
        # read X; read W and Y, write R; FP64: write the stored B Y (B Y^0 of later
        # steps by linearity); mixed: read and write the FP64 B Y
        "rows_inv": 2 * c * n * hc + (5 if mixed else 4) * 8 * n * n,
        # read + write R
        "line_cols": 2 * 8 * n * n,
        # read R, read + write Y, write X (row FFT of the new Y, or of delta)
        "line_rows": 3 * 8 * n * n + 2 * c * n * hc,
        # read E, write W, read four history grids, write Y0, write X
        "sl": 7 * 8 * n * n + 2 * c * n * hc,
        "step_end": 0,
        # FP64 column pass of B V^{n-1}
        "expl_cols": 2 * 8 * hc * (2 * n + L),
        # read X, read V, write E; mixed: write B V
        "expl_rows": 2 * 8 * n * hc + (3 if mixed else 2) * 8 * n * n,
        # read V, write X
        "rows_fwd": 8 * n * n + 2 * 8 * n * hc,
        # mixed form between anchors: read B Y, write B V, read V, write E
        "carry": 4 * 8 * n * n,
        # FP64 explicit part from the previous step's equation: read V and W, write E
        "expl_id": 3 * 8 * n * n,
        # FP64 iteration 1 by linearity: read 4 stored products (3 in the steps just
        # after the damping), W and Y; write R and the stored B Y^0
        "rows_lin": 8 * 8 * n * n,
        # SL without the row transform: read E, four history grids; write W and Y^0
        "sl_lin": 7 * 8 * n * n,
    }[cls]


def line_rows_capacity(n, L, el):
    """Chunk capacity the march launches the line-row kernel with: the smallest
    of E, 3E/2 and 2E that holds the longest chunk ceil(n / PR), PR = L / E / 2."""
    pr = L // el // 2
    m = -(-n // pr)
    return el if m <= el else (3 * el // 2 if m <= 3 * el // 2 else 2 * el)


def kernel_symbol(cls, L, mixed, sl_order, radix=(8, 8, 8, 8), n=None):
    """The kernel instantiation a timing class launches in the march (radix =
    elements per thread of the column pass, row c2r, line-row and SL kernels;
    n: grid side, for the line-row kernel's chunk capacity)."""
    tf = "true" if mixed else "false"
    c = "float" if mixed and cls == "cols" else "double"
    ec, er, el, es = radix
    return {
        "cols": "lpide::ks_cols<%d, %d, HIP_vector_type<%s, 2u>, false>" % (L, ec, c),
        "expl_cols": "lpide::ks_cols<%d, %d, HIP_vector_type<double, 2u>, false>" % (L, ec),
        "rows_inv": "lpide::ks_rows_inv<%d, %d, %d>" % (L, er, 2 if mixed else 1),
        "expl_rows": "lpide::ks_rows_inv<%d, %d, 0>" % (L, er),
        "line_cols": "lpide::ks_line_cols",
        "line_rows": "lpide::ks_line_rows<%d, %d, true, %s, %d>" % (L, el, tf,
                                                                   line_rows_capacity(n or L, L, el)),
        "sl": "lpide::ks_sl<%d, %d, %d, true, %s>" % (L, es, sl_order, tf),
        "step_end": "lpide::ks_step_end",
        "rows_fwd": "lpide::ks_rows_fwd<%d, %d>" % (L, er),
        "carry": "lpide::ks_carry",
        "expl_id": "lpide::ks_expl_identity",
        "rows_lin": "lpide::ks_rows_lin",
        "sl_lin": "lpide::ks_sl_lin<%d>" % sl_order,
    }[cls]


def measured_traffic(path, symbol):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, copy-calibrated), or None when there
    is none or the device sources changed since the counters were taken."""
    if not path or not os.path.exists(path):
        return None
    from paper_2511_02700_amd import profsum
    with open(path) as fh:
        s = json.load(fh)
    if s.get("source_sha256") != profsum.source_digest():
        return None
    for k, v in s["kernels"].items():
        bare = k[5:] if k.startswith("void ") else k
        if bare.startswith(symbol + "(") or bare == symbol:
            return v["hbm_bytes"]
    return None


def roofline(cls, n, L, mixed, launches, ms, traffic_json=None, sl_order=3, radix=(8, 8, 8, 8)):
    per_launch_ms = ms / max(1, launches)
    b = algorithmic_bytes(cls, n, L, mixed)
    achieved = b / (per_launch_ms * 1e-3) / 1e9 if per_launch_ms > 0 else 0.0
    sym = kernel_symbol(cls, L, mixed, sl_order, radix, n)
    return {"kernel": cls, "symbol": sym, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(traffic_json, sym), "bytes_per_launch": b,
            "mean_launch_ms": per_launch_ms, "launches": launches}


def conv_whole(n, L, mixed, stats):
    """The correlation as a whole, per iteration: its algorithmic bytes
    c [2 n^2 + 8 n (L/2+1) + 2 L (L/2+1)] (grid in and out, two round trips of
    the intermediate, one read of the spectrum; c = 8 in FP64, 4 in the mixed
    form) over the summed mean durations of the three kernels that carry it:
    the row r2c sits in the line-row kernel, the column pass is its own, the row
    c2r sits in the residual kernel.  Those two also solve lines and form the
    residual, so the fraction is a lower bound for the correlation itself."""
    hc = L // 2 + 1
    c = 4 if mixed else 8
    b = c * (2 * n * n + 8 * n * hc + 2 * L * hc)
    ks = ("line_rows", "cols", "rows_inv")
    ms = sum(stats[k][1] / max(1, stats[k][0]) for k in ks)
    ach = b / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"kernels": list(ks), "bound": "hbm", "bytes_per_iteration": b, "ms_per_iteration": ms,
            "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS}


def timed_solves(plan, out, steps, timed_classes):
    """steps full solves with HIP events around the named kernel classes (none:
    no events); wall seconds and the per-class (launches, ms)."""
    import torch
    plan.set_timing(timed_classes)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(out)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    stats = plan.kernel_stats()
    plan.set_timing([])
    return wall, stats


def cpu_baseline(w, entries=2):
    """The oracle (unchanged) on the first `entries` entries of the step list of
    the same workload; the sample is the last of them, timed from the previous
    entry's end with the oracle's own step observer (the set-up before it --
    cell averages of V^0, the ILU factors of the first step -- is left out).
    grid-pt-steps/s (one entry stands for N_t / n_entries time steps, as in
    the GPU figure) and the threads it kept busy in that entry."""
    from oracle import integral, levy, scheme
    m = w["model"]
    p = levy.nts_from_std(m["sigma1"], m["sigma2"], m["corr"], m["theta1"], m["theta2"], m["kappa"], m["alpha"])
    n = w["n"]
    h = (w["y_hi"] - w["y_lo"]) / (n - 1)
    d = integral.discretize(p, h, w["r"])
    prob = scheme.Problem(n, (w["y_lo"], w["y_lo"]), h, d, K=w["K"], T=w["T"], N_t=w["N_t"], theta=w["theta"])
    n_entries = len(scheme.step_list(w["theta"], w["T"], w["N_t"]))
    marks = []

    def mark(s, V):
        r = resource.getrusage(resource.RUSAGE_SELF)
        marks.append((time.perf_counter(), r.ru_utime + r.ru_stime))

    t0 = time.perf_counter()
    scheme.solve(prob, tol=w["tol"], inner="bicgstab", n_steps=entries, on_step=mark)
    total = time.perf_counter() - t0
    wall = marks[-1][0] - marks[-2][0]
    cpu = marks[-1][1] - marks[-2][1]
    return dict(value=n * n * (w["N_t"] / n_entries) / wall, unit="grid-pt-steps/s",
                cores=max(1, int(round(cpu / wall))), kind="oracle",
                sample="step-list entry %d of %d (a damped theta=1 quarter step) of the %dx%d workload, timed from the "
                       "end of entry %d (the oracle's set-up and first entry, %.0f s, left out): %.1f s wall, %.1f s "
                       "CPU; BiCGSTAB+ILU inner solves, tol %g; host threads available %d" % (
                           entries, n_entries, n, n, entries - 1, total - wall, wall, cpu, w["tol"],
                           len(os.sched_getaffinity(0))))


def cpu_baseline_start(name):
    """The oracle sample in a child process (CPU only), so it runs while the
    GPU extras do; returns the process (cpu_baseline_finish reads its line)."""
    import subprocess
    env = dict(os.environ, PYTHONPATH=ROOT)
    code = ("import json, bench, workloads; "
            "print(json.dumps(bench.cpu_baseline(workloads.workload(%r))))" % name)
    return subprocess.Popen([sys.executable, "-c", code], cwd=ROOT, env=env, stdout=subprocess.PIPE,
                            stderr=subprocess.PIPE, text=True)


def cpu_baseline_finish(proc, timeout=900):
    out, err = proc.communicate(timeout=timeout)
    if proc.returncode != 0:
        return {"error": "oracle sample failed: " + err.strip()[-400:]}
    return json.loads(out.strip().splitlines()[-1])


def central_nodes(w, lo=80.0, hi=120.0):
    """Grid indices whose spot S = K e^y lies in [lo, hi] (per axis)."""
    import numpy as np
    n = w["n"]
    y = w["y_lo"] + (w["y_hi"] - w["y_lo"]) / (n - 1) * np.arange(n)
    S = w["K"] * np.exp(y)
    return np.nonzero((S >= lo) & (S <= hi))[0]


def greek_diffs(pa, Va, pb, Vb, sel):
    """Max |a - b| / max |b| of the five Delta/Gamma surfaces on the nodes sel x sel."""
    import numpy as np
    ga = pa.greeks(Va).cpu().numpy()[:, sel][:, :, sel]
    gb = pb.greeks(Vb).cpu().numpy()[:, sel][:, :, sel]
    names = ("delta1", "delta2", "gamma11", "gamma12", "gamma22")
    return {k: float(np.max(np.abs(ga[q] - gb[q])) / max(1e-300, float(np.max(np.abs(gb[q])))))
            for q, k in enumerate(names)}


def measure_workload(lp, name, steps, warmup, precision="fp64", sl_order=3, fft_size=0, traffic_json=None,
                     other_side=True):
    """Throughput and rooflines of full solves of a workload (both forms), as in
    the headline: `steps` timed solves without events, then `steps` with HIP
    events bound to the dominant class and the three correlation kernels."""
    import numpy as np
    import torch
    import workloads
    w = workloads.workload(name)
    n, Nt = w["n"], w["N_t"]
    other = "fp32conv" if precision == "fp64" else "fp64"
    plan_ms, plans = {}, {}
    for pr in (precision, other):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plans[pr] = lp.plan_from_workload(w, sl_order=sl_order, precision=pr, fft_size=fft_size)
        torch.cuda.synchronize()
        plan_ms[pr] = 1e3 * (time.perf_counter() - t0)
    plan = plans[precision]
    mixed = precision == "fp32conv"
    info = plan.info()
    L = info["L"]
    outs = {pr: torch.empty((n, n), dtype=torch.float64, device="cuda") for pr in plans}
    for pr in plans:
        for _ in range(warmup):
            plans[pr].solve(outs[pr])
    torch.cuda.synchronize()
    # one untimed profiling solve with every kernel class timed: picks the dominant class
    plan.set_timing(lp._lib.KCLASSES)
    plan.solve(outs[precision])
    prof = plan.kernel_stats()
    dominant = max(prof, key=lambda c: prof[c][1])
    # timed region: K solves without events, giving value; then the same K
    # solves with start/stop events bound to every launch of the dominant
    # class and of the correlation's three kernels (the events take the
    # dispatch's own timestamps), giving their mean launch durations
    wall, _ = timed_solves(plan, outs[precision], steps, [])
    _, live = timed_solves(plan, outs[precision], steps, sorted({dominant, "cols", "rows_inv", "line_rows"}))
    info = plan.info()
    # the other precision on the same workload: throughput, conv roofline, and
    # the mixed-vs-plain differences at seeded spot pairs and on the Greeks
    wall_o, _ = timed_solves(plans[other], outs[other], steps, [])
    _, live_o = timed_solves(plans[other], outs[other], steps, ["cols", "rows_inv", "line_rows"])
    spots = workloads.spot_pairs(64, seed=7)
    pd = {pr: plans[pr].price(outs[pr], spots, with_delta=True) for pr in plans}
    p64, d64 = (t.cpu().numpy() for t in pd["fp64"])
    p32, d32 = (t.cpu().numpy() for t in pd["fp32conv"])
    rel_grid = float((outs["fp32conv"] - outs["fp64"]).abs().div(outs["fp64"].abs().clamp_min(1.0)).max())
    oinfo = plans[other].info()
    res = {
        "value": n * n * Nt * steps / wall,
        "ms_per_step": 1e3 * wall / steps,
        "dtype": "f64" if not mixed else "f32 correlation / f64 rest",
        "config": {"workload": "%s: put-on-average K=100 T=1 r=0.03, NTS alpha=%g sigma=(%g,%g) corr=%g "
                               "theta=(%g,%g) kappa=%g, %dx%d log grid on [%g,%g]^2, %d time steps, theta=%g, "
                               "tol %g, SL order %d, %s" % (
                                   name, w["model"]["alpha"], w["model"]["sigma1"], w["model"]["sigma2"],
                                   w["model"]["corr"], w["model"]["theta1"], w["model"]["theta2"],
                                   w["model"]["kappa"], n, n, w["y_lo"], w["y_hi"], Nt, w["theta"], w["tol"],
                                   sl_order, precision),
                   "n": n, "N_t": Nt, "L": L, "N_z": info["N_z"], "precision": precision,
                   "parallelism": "single GPU"},
        "roofline": roofline(dominant, n, L, mixed, *live[dominant], traffic_json=traffic_json, sl_order=sl_order,
                             radix=info["radix"]),
        "conv_roofline": roofline("cols", n, L, mixed, *live["cols"], traffic_json=traffic_json,
                                  sl_order=sl_order, radix=info["radix"]),
        "conv_whole": conv_whole(n, L, mixed, live),
        "plan_ms": plan_ms[precision],
        "radix_schedule": dict(zip(("cols", "row_c2r", "line_rows", "sl"), info["radix"])),
        "iters_per_step": info["total_iters"] / info["n_steps"],
        "kernel_ms_per_solve": {c: prof[c][1] for c in prof if prof[c][0]},
        other: {"value": n * n * Nt * steps / wall_o, "ms_per_step": 1e3 * wall_o / steps,
                "conv_roofline": roofline("cols", n, L, other == "fp32conv", *live_o["cols"],
                                          traffic_json=traffic_json, sl_order=sl_order, radix=oinfo["radix"]),
                "conv_whole": conv_whole(n, L, other == "fp32conv", live_o),
                "iters_per_step": oinfo["total_iters"] / oinfo["n_steps"], "plan_ms": plan_ms[other]},
        "mixed_vs_plain_rel": {"prices": float(np.max(np.abs(p32 - p64) / np.maximum(1.0, np.abs(p64)))),
                               "deltas_abs": float(np.max(np.abs(d32 - d64))), "grid": rel_grid,
                               "greeks_rel_S_80_120": greek_diffs(plans["fp32conv"], outs["fp32conv"],
                                                                  plans["fp64"], outs["fp64"], central_nodes(w)),
                               "spots": 64, "bound": 1e-6},
    }
    if other_side:
        # the same solve on the other candidate transform side: 3L/4 for a power
        # of two L (when it still covers the kernel's support), else the power of two above
        alt = 3 * L // 4 if L & (L - 1) == 0 else 1 << (L - 1).bit_length()
        try:
            p2 = lp.plan_from_workload(w, sl_order=sl_order, precision=precision, fft_size=alt)
        except lp.LpideError:
            p2 = None
        if p2 is not None:
            o2 = torch.empty((n, n), dtype=torch.float64, device="cuda")
            p2.solve(o2)
            wall2, _ = timed_solves(p2, o2, steps, [])
            res["other_side"] = {"L": alt, "radix": p2.info()["radix"], "value": n * n * Nt * steps / wall2,
                                 "ms_per_step": 1e3 * wall2 / steps,
                                 "max_rel_diff": float((o2 - outs[precision]).abs().div(
                                     outs[precision].abs().clamp_min(1.0)).max())}
            p2.close()
            del o2
    for pr in plans:
        plans[pr].close()
    del outs
    torch.cuda.empty_cache()
    return res


def table3_check(lp):
    """The paper's Table 3 (put-on-the-average prices at nine spot pairs for the
    four parameter sets of Table 1) against whole GPU marches on the log grid:
    max |price - printed price| per set, and the solve time."""
    import csv
    import numpy as np
    import torch

    def rows(name):
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return list(csv.DictReader(line for line in f if not line.startswith("#")))

    t1 = {r["name"]: r for r in rows("table1_params.csv")}
    gold = rows("table3_prices.csv")
    spots = [(float(g["x1"]), float(g["x2"])) for g in gold]
    out = {}
    for name, n, half in (("VG0", 1024, 4.0), ("VG1", 1024, 2.0), ("NIG0", 2048, 1.5), ("NIG1", 2048, 2.0)):
        r = t1[name]
        lv = lp.levy_nts(float(r["alpha"]), float(r["delta"]), float(r["lambda"]),
                         (float(r["eta1"]), float(r["eta2"])), (float(r["rho11"]), float(r["rho12"]), float(r["rho22"])),
                         float(r["r"]))
        plan = lp.Plan(lp.make_grid(n, -half, half), lv, lp.make_payoff("put_avg", float(r["K"]), float(r["T"])),
                       theta=0.5, M=n // 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V = plan.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        got = plan.price(V, spots).cpu().numpy()
        want = np.array([float(g[name]) for g in gold])
        out[name] = {"n": n, "domain": [-half, half], "L": plan.info()["L"], "ms": 1e3 * dt,
                     "max_abs_err": float(np.max(np.abs(got - want)))}
        del plan, V
        torch.cuda.empty_cache()
    return out


def price_space_paper_grids(lp):
    """All four Table 1 sets on the paper's own price-space grids (N_x = 800,
    NIG0 400; N_z = 2 N_x, N_t = N_x / 2, x_max and c of Sec. 4), tol 1e-9
    (the paper stops at 1e-7; on these NIG grids the stopping value's rounding
    floor lies near 1e-10): max |price - Table 3| over the nine spots, march
    time, iterations, the Anderson depth in use."""
    import csv
    import numpy as np
    import torch

    def rows(name):
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return list(csv.DictReader(line for line in f if not line.startswith("#")))

    t1 = {r["name"]: r for r in rows("table1_params.csv")}
    gold = rows("table3_prices.csv")
    spots = [(float(g["x1"]), float(g["x2"])) for g in gold]
    printed_c = {"VG0": 21.6164, "VG1": 67.1487, "NIG0": 55.0673, "NIG1": 45.0189}     # Sec. 4
    x_max = {"VG0": 5700.0, "VG1": 500.0, "NIG0": 600.0, "NIG1": 700.0}               # Sec. 4
    out = {}
    for name, N_x in (("VG0", 800), ("VG1", 800), ("NIG0", 400), ("NIG1", 800)):
        r = t1[name]
        lv = lp.levy_nts(float(r["alpha"]), float(r["delta"]), float(r["lambda"]),
                         (float(r["eta1"]), float(r["eta2"])), (float(r["rho11"]), float(r["rho12"]), float(r["rho22"])),
                         float(r["r"]))
        t0 = time.perf_counter()
        plan = lp.PsPlan(lp.make_ps_grid(N_x, x_max[name], c=printed_c[name]), lv,
                         lp.make_payoff("put_avg", float(r["K"]), float(r["T"])), N_t=N_x // 2, tol=1e-9,
                         max_iter=128)
        plan_s = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        V = plan.solve()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        info = plan.info()
        got = plan.price(V, spots).cpu().numpy()
        want = np.array([float(g[name]) for g in gold])
        out[name] = {"N_x": N_x, "n_in": info["n_in"], "L": info["L"], "n_steps": info["n_steps"],
                     "iterations": info["total_iters"], "accel_depth": info["accel_depth"], "plan_s": plan_s,
                     "march_s": dt,
                     "prices": [round(float(v), 6) for v in got],
                     "max_abs_err_vs_table3": float(np.max(np.abs(got - want)))}
        print("[price-space paper grid] %s: %s" % (name, json.dumps(out[name])), file=sys.stderr, flush=True)
        plan.close()
        del V
        torch.cuda.empty_cache()
    return out


def price_space_check(lp):
    """The paper's own price-space discretization (Sec. 3.2, 3.3, Sec. 4
    settings) on each Table 1 set at the largest N_x whose #in fits a
    transform side of 4096, N_t = N_x / 2, fixed-point tol 1e-10: march time
    (second of two marches), throughput in grid-pt-steps/s ((N_x+1)^2 x
    step-list entries / time), iterations, and max |price - Table 3| over the
    nine spots (the paper's N_x = 800, 400 for NIG0).  The plans choose the
    fixed-point iteration automatically (Anderson mixing of depth 4 on the
    slowly contracting NIG sets); where mixing is on, the paper's iteration is
    timed beside it."""
    import csv
    import numpy as np
    import torch

    def rows(name):
        with open(os.path.join(ROOT, "tests", "golden", name)) as f:
            return list(csv.DictReader(line for line in f if not line.startswith("#")))

    t1 = {r["name"]: r for r in rows("table1_params.csv")}
    gold = rows("table3_prices.csv")
    spots = [(float(g["x1"]), float(g["x2"])) for g in gold]
    printed_c = {"VG0": 21.6164, "VG1": 67.1487, "NIG0": 55.0673, "NIG1": 45.0189}     # Sec. 4
    x_max = {"VG0": 5700.0, "VG1": 500.0, "NIG0": 600.0, "NIG1": 700.0}               # Sec. 4
    out = {}
    for name, N_x in (("VG0", 700), ("VG1", 400), ("NIG0", 128), ("NIG1", 224)):
        r = t1[name]
        lv = lp.levy_nts(float(r["alpha"]), float(r["delta"]), float(r["lambda"]),
                         (float(r["eta1"]), float(r["eta2"])), (float(r["rho11"]), float(r["rho12"]), float(r["rho22"])),
                         float(r["r"]))
        def timed(accel):
            plan = lp.PsPlan(lp.make_ps_grid(N_x, x_max[name], c=printed_c[name]), lv,
                             lp.make_payoff("put_avg", float(r["K"]), float(r["T"])), N_t=N_x // 2, tol=1e-10,
                             max_iter=128, accel=accel)
            V = plan.solve()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            V = plan.solve(V)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            got = plan.price(V, spots).cpu().numpy()
            info = plan.info()
            plan.close()
            return info, dt, got

        info, dt, got = timed(-1)
        want = np.array([float(g[name]) for g in gold])
        out[name] = {"N_x": N_x, "n_in": info["n_in"], "L": info["L"], "n_steps": info["n_steps"],
                     "iterations": info["total_iters"], "accel_depth": info["accel_depth"], "ms": 1e3 * dt,
                     "grid_pt_steps_per_s": (N_x + 1) ** 2 * info["n_steps"] / dt,
                     "max_abs_err_vs_table3": float(np.max(np.abs(got - want)))}
        if info["accel_depth"] > 0:           # the paper's iteration beside the mixing
            i0, dt0, got0 = timed(0)
            out[name]["paper_iteration"] = {"iterations": i0["total_iters"], "ms": 1e3 * dt0,
                                            "max_price_diff": float(np.max(np.abs(got0 - got)))}
        torch.cuda.empty_cache()
    return out


def adjoint_measure(lp, name="nts1024", C=32):
    """The adjoint form on its workload: forward solve time, and the adjoint's
    march part (segment recompute + reverse steps + gather, with the solve's
    checkpoints reused) and host Jacobian, for J = a seeded combination of 64
    spot-pair prices."""
    import numpy as np
    import torch
    import workloads
    w = workloads.workload(name)
    spots = workloads.spot_pairs(64, seed=4)
    wts = np.random.default_rng(4).standard_normal(64)
    plan = lp.plan_from_workload(w)
    plan.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.solve()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    plan.set_checkpoints(C)
    V = plan.solve()
    vbar = plan.price_adjoint(spots, wts)
    # one untimed call first, as for the forward solves (graph captures, Jacobian cache)
    plan.adjoint(vbar, checkpoint_every=C, std_params=lp.std_params_of(w))
    t0 = time.perf_counter()
    grad, _, info = plan.adjoint(vbar, checkpoint_every=C, std_params=lp.std_params_of(w))
    t_adj = time.perf_counter() - t0
    march = info["recompute_ms"] + info["reverse_ms"] + info["gather_ms"]
    # the forward with every product of B by the correlation (the reverse march
    # has no counterpart of the forward's two shortcuts)
    pa = lp.plan_from_workload(w, all_correlations=True)
    pa.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pa.solve()
    torch.cuda.synchronize()
    t_fwd_all = time.perf_counter() - t0
    pa.close()
    # every state and explicit part kept by the forward march (no recompute):
    # (2 n_steps + 1) n^2 FP64 of HBM
    n_steps = plan.info()["n_steps"]
    plan.close()
    pk = lp.plan_from_workload(w)
    pk.set_checkpoints(1 << 30)
    pk.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pk.solve()
    torch.cuda.synchronize()
    t_fwd_keep = time.perf_counter() - t0
    vbar_k = pk.price_adjoint(spots, wts)
    pk.adjoint(vbar_k, checkpoint_every=1 << 30)
    _, _, info_k = pk.adjoint(vbar_k, checkpoint_every=1 << 30)
    march_k = info_k["recompute_ms"] + info_k["reverse_ms"] + info_k["gather_ms"]
    keep_all = {"forward_recording_ms": 1e3 * t_fwd_keep, "adjoint_march_ms": march_k,
                "ratio_to_forward": march_k / (1e3 * t_fwd),
                "hbm_bytes": (2 * pk.info()["n_steps"] + 1) * 8 * w["n"] ** 2}
    pk.close()
    return {"workload": "%s: %dx%d, %d steps, checkpoints every %d, J = 64 seeded spot prices" % (
                name, w["n"], w["n"], w["N_t"], C),
            "forward_ms": 1e3 * t_fwd, "adjoint_march_ms": march, "ratio_to_forward": march / (1e3 * t_fwd),
            "recompute_ms": info["recompute_ms"], "reverse_ms": info["reverse_ms"], "gather_ms": info["gather_ms"],
            "forward_all_correlations_ms": 1e3 * t_fwd_all,
            "ratio_to_forward_all_correlations": march / (1e3 * t_fwd_all),
            "keep_all_states": keep_all,
            "host_jacobian_ms": info["jacobian_ms"], "adjoint_wall_ms": 1e3 * t_adj,
            "adjoint_iters_per_step": info["adj_iters"] / n_steps,
            "grad": [float(g) for g in grad]}


def batch_measure(lp, count=256, seed=3, trial_steps=32):
    """The batched form on `count` draws of the batched workload recipe: grid-
    pt-steps/s of one batched solve (autotuned on steady windows, hipGraph
    replay, one launch per kernel and group) against the same plans solved one
    after the other."""
    import torch
    import workloads
    draws = workloads.batch_draw(256, seed=seed)[:count]
    t0 = time.perf_counter()
    plans = [lp.plan_from_workload(d) for d in draws]
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    work = sum(d["n"] ** 2 * d["N_t"] for d in draws)
    batch = lp.Batch(plans)
    t0 = time.perf_counter()
    groups = batch.tune(trial_steps=trial_steps)
    tune_s = time.perf_counter() - t0
    outs = batch.solve()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    batch.solve(outs)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    solo = [p._grid_tensor() for p in plans]
    for p, o in zip(plans, solo):
        p.solve(o)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p, o in zip(plans, solo):
        p.solve(o)
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    diff = max(float((a - b).abs().max()) for a, b in zip(outs, solo))
    ns = {}
    for d in draws:
        ns[d["n"]] = ns.get(d["n"], 0) + 1
    batch.close()
    for p in plans:
        p.close()
    del outs, solo
    torch.cuda.empty_cache()
    return {"workload": "%d draws of the batched recipe (seed %d): plans per n %s, alpha ~ U[0.2, 0.6], sigma ~ "
                        "U[0.1, 0.4], corr ~ U[-0.7, 0.7], K ~ U[80, 120], T ~ U[0.25, 2], N_t = n/2" % (
                            count, seed, dict(sorted(ns.items()))),
            "value": work / t_b, "unit": "grid-pt-steps/s", "ms": 1e3 * t_b, "solo_ms": 1e3 * t_s,
            "speedup_vs_solo": t_s / t_b, "max_abs_diff_vs_solo": diff, "plans_s": plan_s, "tune_s": tune_s,
            "trial_steps": trial_steps, "groups": groups}


def fv512_vs_oracle(lp):
    """The whole fv512 march in both forms against the oracle's (the committed
    golden written by tests/golden/make_oracle_fv512.py): prices and deltas at
    its 64 spot pairs, the grid on its sampled nodes, and the Delta/Gamma
    surfaces there when the golden holds them."""
    import numpy as np
    import workloads
    g = np.load(os.path.join(ROOT, "tests", "golden", "oracle_fv512.npz"))
    idx = g["idx"]
    out = {}
    for pr in ("fp64", "fp32conv"):
        plan = lp.plan_from_workload(workloads.workload("fv512"), precision=pr)
        V = plan.solve()
        p, d = plan.price(V, g["spots"], with_delta=True)
        r = {"prices_rel": float(np.max(np.abs(p.cpu().numpy() - g["price"]) / np.maximum(1.0, np.abs(g["price"])))),
             "deltas_abs": float(np.max(np.abs(d.cpu().numpy() - g["delta"]))),
             "grid_rel": float(np.max(np.abs(V.cpu().numpy()[np.ix_(idx, idx)] - g["V_259"]) /
                                      np.maximum(1.0, np.abs(g["V_259"]))))}
        if "greeks" in g:
            gs = plan.greeks(V).cpu().numpy()[:, idx][:, :, idx]
            for q, k in enumerate(("delta1", "delta2", "gamma11", "gamma12", "gamma22")):
                r[k + "_rel"] = float(np.max(np.abs(gs[q] - g["greeks"][q])) / np.max(np.abs(g["greeks"][q])))
        out[pr] = r
        plan.close()
    return out


def copy_reference(torch, mib=512, reps=20):
    """Achievable device-to-device bandwidth on this GPU: torch's vectorised copy
    of a resident 512 MiB FP64 tensor (read + write bytes / time).  A reference
    for the kernels' rooflines beside the HBM peak, not part of the solver."""
    n = mib * (1 << 20) // 8
    a = torch.rand(n, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    gbs = 2.0 * n * 8 / (ms * 1e-3) / 1e9
    del a, b
    return {"kernel": "torch copy_ (%d MiB, FP64)" % mib, "GB/s": gbs, "ms": ms}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed full solves")
    ap.add_argument("--warmup", type=int, default=2, help="untimed full solves")
    ap.add_argument("--workload", default="nig2048_m")
    ap.add_argument("--sl-order", type=int, default=3)
    ap.add_argument("--precision", choices=["fp64", "fp32conv"], default="fp64",
                    help="form timed for the headline value; the other form is timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip fv512, Table 3, the price-space plan, the adjoint and the batched measurements")
    ap.add_argument("--batch-count", type=int, default=256, help="draws of the batched recipe in the batched leg")
    ap.add_argument("--no-paper-grids", action="store_true",
                    help="skip the four Table 3 sets on the paper's own price-space grids (N_x = 800, NIG0 400; "
                         "about 35 s)")
    ap.add_argument("--fft-size", type=int, default=0,
                    help="transform side of the correlation (0: the smallest supported one, 2^m or 3*2^m)")
    ap.add_argument("--traffic-json", default=None,
                    help="rocprofv3 counter summary (profsum pmc --json) giving measured HBM bytes per launch; "
                         "default profiles/pmc_<workload>.json")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (this solver has no multi-GPU path); got --gpus %d" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch  # noqa: F401

    import paper_2511_02700_amd as lp

    rank = int(os.environ.get("RANK", "0"))
    tj = args.traffic_json or os.path.join(ROOT, "profiles", "pmc_%s.json" % args.workload)
    head = measure_workload(lp, args.workload, args.steps, args.warmup, args.precision, args.sl_order,
                            args.fft_size, tj)
    result = {
        "metric": METRIC,
        "value": head.pop("value"),
        "unit": "grid-pt-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": head.pop("dtype"),
        "data": "synthetic",
        "config": head.pop("config"),
        "roofline": head.pop("roofline"),
    }
    result.update(head)
    ref = copy_reference(torch)
    ref["roofline_kernel_frac_of_copy"] = result["roofline"]["achieved"] / ref["GB/s"]
    result["copy_reference"] = ref
    # the small, launch-bound fv512 leg runs with the host cores idle; the oracle
    # sample then runs on the host while the other GPU extras run
    if not args.no_extras:
        fv = measure_workload(lp, "fv512", args.steps, args.warmup,
                              traffic_json=os.path.join(ROOT, "profiles", "pmc_fv512.json"), other_side=True)
        fv["vs_oracle"] = fv512_vs_oracle(lp)
        result["fv512"] = fv
    child = cpu_baseline_start(args.workload) if rank == 0 and not args.no_cpu_baseline else None
    if not args.no_extras:
        result["paper_table3"] = table3_check(lp)
        result["price_space"] = price_space_check(lp)
        if not args.no_paper_grids:
            result["price_space_paper_grids"] = price_space_paper_grids(lp)
        result["adjoint"] = adjoint_measure(lp)
        result["batched"] = batch_measure(lp, count=args.batch_count)
    if child is not None:
        result["cpu_baseline"] = cpu_baseline_finish(child)
    if rank == 0:
        print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
