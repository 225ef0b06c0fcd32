"""Summaries of rocprofv3 output for the solver's kernels (text for the
profile records, JSON for bench.py's measured-traffic field).

    python -m paper_2511_02700_amd.profsum stats DIR
        kernel table (calls, mean/min/max duration, total, share) from the
        *_kernel_stats.csv that `rocprofv3 --kernel-trace --stats
        --output-format csv -d DIR -o run` writes.

    python -m paper_2511_02700_amd.profsum table DIR [DIR ...] [--ref COUNTER]
        per kernel: the mean of every counter of the --pmc runs in the DIRs
        over the working dispatches (those whose reference counter, by default
        SQ_WAVE_CYCLES, reaches a quarter of the median of the kernel's upper
        half: iterations after convergence exit at once), with the VGPR
        count, the LDS bytes per
        workgroup and the workgroup size the runtime reports.

    python -m paper_2511_02700_amd.profsum pmc FETCH_DIR WRITE_DIR [--json OUT]
        per-kernel FETCH_SIZE and WRITE_SIZE (KiB per dispatch) from two
        `rocprofv3 --pmc FETCH_SIZE` / `--pmc WRITE_SIZE` runs, calibrated by
        the plain copy kernel k_copy of the same runs (one FP64 value per
        thread: known bytes = 8 x grid size).  Dispatches of a kernel that read
        or wrote less than 5% of that kernel's largest dispatch are early-exit
        launches (iterations after convergence) and are left out of the mean.
"""

import argparse
import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

# kernel-name prefixes of the march kernels -> the timing classes of the C ABI
# (the template arguments tell the FP64 and mixed instantiations apart)
CLASS_OF = [
    ("lpide::ks_cols<", "cols"),
    ("lpide::ks_rows_inv<", "rows_inv"),
    ("lpide::ks_line_cols", "line_cols"),
    ("lpide::ks_line_rows<", "line_rows"),
    ("lpide::ks_sl<", "sl"),
    ("lpide::ks_step_end", "step_end"),
    ("lpide::ks_rows_fwd<", "rows_fwd"),
]


# The sources that define the march kernels and their launch sequences (grid,
# block, radix): a kernel's measured traffic holds while these are unchanged.
# Host-only code (plans, the C ABI, pricing) is not part of it.
KERNEL_SOURCES = ("fft.hpp", "kernels.hpp", "linesolve.hpp", "step_kernels.hpp", "conv_kernels.hpp",
                  "march_L.hip", "plan.hpp")


def source_digest():
    """SHA-256 over the kernel sources: the measured traffic of a kernel is
    valid only for the sources it was measured on."""
    h = hashlib.sha256()
    for name in sorted(KERNEL_SOURCES):
        with open(os.path.join(HERE, "csrc", name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()


def _one(pattern):
    hits = sorted(glob.glob(pattern, recursive=True))
    if not hits:
        raise SystemExit("no file matches " + pattern)
    return hits[0]


def kernel_stats(d):
    path = _one(os.path.join(d, "**", "*kernel_stats.csv"))
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((r["Name"], int(r["Calls"]), float(r["TotalDurationNs"]), float(r["AverageNs"]),
                         float(r["MinNs"]), float(r["MaxNs"]), float(r["Percentage"])))
    rows.sort(key=lambda x: -x[2])
    return rows


def active_durations(d):
    """Per kernel: (calls, active calls, mean active duration in us) from the
    kernel trace.  Active = at least a quarter of the median of the kernel's
    upper half of durations, which separates the early-exit launches (about
    1 us) of iterations after convergence from the launches that work."""
    path = _one(os.path.join(d, "**", "*kernel_trace.csv"))
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            per.setdefault(r["Kernel_Name"], []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = {}
    for k, ds in per.items():
        s = sorted(ds)
        up = s[len(s) // 2:]
        thr = 0.25 * up[len(up) // 2]
        act = [x for x in ds if x >= thr]
        out[k] = (len(ds), len(act), sum(act) / len(act) / 1e3)
    return out


def print_stats(d, out=sys.stdout):
    rows = kernel_stats(d)
    act = active_durations(d)
    tot = sum(r[2] for r in rows)
    out.write("%-64s %7s %9s %9s %9s %10s %6s %7s %13s\n" % ("kernel", "calls", "avg_us", "min_us", "max_us",
                                                             "total_ms", "pct", "active", "active_avg_us"))
    for name, calls, t, avg, mn, mx, pct in rows:
        a = act.get(name, (calls, calls, avg / 1e3))
        out.write("%-64s %7d %9.2f %9.2f %9.2f %10.2f %6.2f %7d %13.2f\n" % (name[:64], calls, avg / 1e3, mn / 1e3,
                                                                             mx / 1e3, t / 1e6, pct, a[1], a[2]))
    out.write("total kernel time %.2f ms\n" % (tot / 1e6))


def counters(d, counter):
    path = _one(os.path.join(d, "**", "*counter_collection.csv"))
    per = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            per.setdefault(r["Kernel_Name"], []).append((float(r["Counter_Value"]), int(r["Grid_Size"])))
    return per


def _bare(name):
    """Kernel name without a leading 'void ' and without namespace qualifiers."""
    name = name[5:] if name.startswith("void ") else name
    head = name.split("(", 1)[0].split("<", 1)[0]
    return name[head.rfind("::") + 2:] if "::" in head else name


def _active_mean(vals):
    top = max(v for v, _ in vals)
    act = [v for v, _ in vals if v >= 0.05 * top]
    return (sum(act) / len(act) if act else 0.0), len(act), len(vals)


def pmc_summary(fetch_dir, write_dir):
    fetch, write = counters(fetch_dir, "FETCH_SIZE"), counters(write_dir, "WRITE_SIZE")
    cal = {}
    for nm, per, key in (("FETCH_SIZE", fetch, "read"), ("WRITE_SIZE", write, "write")):
        copies = [(v, g) for k, vals in per.items() if _bare(k).startswith("k_copy(") for v, g in vals]
        big = max(copies, key=lambda x: x[1]) if copies else None
        if big is None or big[0] <= 0:
            raise SystemExit("no k_copy dispatch to calibrate " + nm)
        # bytes the copy must move per counter KiB
        cal[key] = {"copy_bytes": 8 * big[1], "counter_kib": big[0], "scale": 8 * big[1] / (1024.0 * big[0])}
    kernels = {}
    for k in sorted(set(fetch) | set(write)):
        bare = k[5:] if k.startswith("void ") else k
        cls = next((c for p, c in CLASS_OF if bare.startswith(p)), None)
        f = _active_mean(fetch[k]) if k in fetch else (0.0, 0, 0)
        w = _active_mean(write[k]) if k in write else (0.0, 0, 0)
        kernels[k] = {"class": cls, "fetch_kib": f[0], "write_kib": w[0], "dispatches": f[2],
                      "active_dispatches": f[1],
                      "hbm_bytes": 1024.0 * (f[0] * cal["read"]["scale"] + w[0] * cal["write"]["scale"])}
    return {"calibration": cal, "kernels": kernels, "source_sha256": source_digest()}


def counter_table(dirs, ref="SQ_WAVE_CYCLES"):
    """{kernel: {"meta": (vgpr, agpr, lds, wg), "n": (working, all), counter: mean}}."""
    rows = {}
    for d in dirs:
        path = _one(os.path.join(d, "**", "*counter_collection.csv"))
        with open(path) as fh:
            for r in csv.DictReader(fh):
                key = (d, r.get("Dispatch_Id") or r.get("Correlation_Id"))
                e = rows.setdefault(key, {"kernel": r["Kernel_Name"], "meta": (
                    int(r.get("VGPR_Count", 0) or 0), int(r.get("Accum_VGPR_Count", 0) or 0),
                    int(r.get("LDS_Block_Size", 0) or 0), int(r.get("Workgroup_Size", 0) or 0)), "c": {}})
                e["c"][r["Counter_Name"]] = e["c"].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    per = {}
    for (d, _), e in rows.items():
        per.setdefault(e["kernel"], {}).setdefault(d, []).append(e)
    out = {}
    for k, by_dir in per.items():
        res = {"meta": None, "n": [0, 0]}
        for d, lst in by_dir.items():
            # the reference counter of this run: the one asked for, else the
            # first of a few that scale with the work a dispatch did
            have = lst[0]["c"]
            rname = next((c for c in (ref, "SQ_WAVE_CYCLES", "GRBM_GUI_ACTIVE", "SQ_INSTS_VALU", "TA_BUSY_avr",
                                      "SQ_BUSY_CYCLES") if c in have), next(iter(have), None))
            refs = sorted(x["c"].get(rname, 0.0) for x in lst)
            up = refs[len(refs) // 2:]
            thr = 0.25 * up[len(up) // 2] if up else 0.0
            act = [x for x in lst if x["c"].get(rname, 0.0) >= thr]
            res["meta"] = lst[0]["meta"]
            res["n"][0] += len(act)
            res["n"][1] += len(lst)
            for name in act[0]["c"] if act else []:
                res[name] = sum(x["c"].get(name, 0.0) for x in act) / len(act)
        out[k] = res
    return out


def print_table(t, out=sys.stdout):
    names = sorted({c for v in t.values() for c in v if c not in ("meta", "n")})
    out.write("%-56s %5s %5s %6s %5s %9s" % ("kernel", "vgpr", "agpr", "lds_B", "wg", "working"))
    for c in names:
        out.write(" %14s" % c[:14])
    out.write("\n")
    for k, v in sorted(t.items(), key=lambda kv: -kv[1].get("SQ_WAVE_CYCLES", kv[1].get(names[0], 0.0) if names else 0)):
        m = v["meta"] or (0, 0, 0, 0)
        out.write("%-56s %5d %5d %6d %5d %4d/%-4d" % (k[:56], m[0], m[1], m[2], m[3], v["n"][0], v["n"][1]))
        for c in names:
            out.write(" %14.4g" % v.get(c, float("nan")))
        out.write("\n")


def print_pmc(s, out=sys.stdout):
    c = s["calibration"]
    out.write("calibration (k_copy): read %d B -> FETCH_SIZE %.1f KiB (scale %.4f); write %d B -> WRITE_SIZE %.1f KiB "
              "(scale %.4f)\n" % (c["read"]["copy_bytes"], c["read"]["counter_kib"], c["read"]["scale"],
                                  c["write"]["copy_bytes"], c["write"]["counter_kib"], c["write"]["scale"]))
    out.write("%-64s %9s %12s %12s %14s\n" % ("kernel", "active", "FETCH_KiB", "WRITE_KiB", "HBM_MB/launch"))
    for k, v in sorted(s["kernels"].items(), key=lambda kv: -kv[1]["hbm_bytes"]):
        out.write("%-64s %4d/%-4d %12.1f %12.1f %14.3f\n" % (k[:64], v["active_dispatches"], v["dispatches"],
                                                             v["fetch_kib"], v["write_kib"], v["hbm_bytes"] / 1e6))
    out.write("device sources sha256 %s\n" % s["source_sha256"])


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    sub = ap.add_subparsers(dest="cmd", required=True)
    a = sub.add_parser("stats")
    a.add_argument("dir")
    t = sub.add_parser("table")
    t.add_argument("dirs", nargs="+")
    t.add_argument("--ref", default="SQ_WAVE_CYCLES")
    b = sub.add_parser("pmc")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--json")
    args = ap.parse_args(argv)
    if args.cmd == "stats":
        print_stats(args.dir)
    elif args.cmd == "table":
        print_table(counter_table(args.dirs, args.ref))
    else:
        s = pmc_summary(args.fetch_dir, args.write_dir)
        print_pmc(s)
        if args.json:
            with open(args.json, "w") as fh:
                json.dump(s, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main()
