"""Summaries of rocprofv3 output (CSV) for the kernels of this library.

    python -m paper_2103_04770_amd.profiling stats <kernel_stats.csv> --trace <kernel_trace.csv> --cmd "..."
    python -m paper_2103_04770_amd.profiling counters <fetch_dir> <write_dir> \
        --copy-mib 1024 --cmd "..." [--json out.json]

Counter calibration: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled
by the ratio of the true byte count of a plain device copy of known size to
what the same counter reports for that copy (the largest copyBuffer dispatch
of the run).  A kernel's traffic is the mean over its full launches (counter
>= half of its maximum; launches that returned early because the Krylov
solve had converged are left out).
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import gzip
import hashlib
import json
import os

PKG = os.path.dirname(os.path.abspath(__file__))

# kernel template name -> class (the y passes share k_strided with the
# transforms and cannot be told apart by name)
CLASSES = {
    "k_x_fused_gal": "galerkin_x_fused",
    "k_gal_dir_inv": "galerkin_outer_dir_inv",
    "k_gal_dot_fwd": "galerkin_outer_dot_fwd",
    "k_gal_resid": "galerkin_resid",
    "k_gal_fwd_resid": "galerkin_outer_fwd_resid",
    "k_x_fused_helm": "helmholtz_x_fused",
    "k_h_dir_inv": "helmholtz_outer_dir_inv",
    "k_h_div_fwd": "helmholtz_outer_div_fwd",
    "k_h_fwd_resid": "helmholtz_outer_div_fwd",
    "k_h_resid": "helmholtz_resid",
}


def classify(name):
    """'void fftg::k_gal_dir_inv<double, 128>' -> ('fp64', 'galerkin_outer_dir_inv')."""
    base = name.split("<")[0].split("::")[-1]
    if "<" not in name:
        return None
    args = [a.strip() for a in name.split("<", 1)[1].rsplit(">", 1)[0].split(",")]
    prec = {"double": "fp64", "float": "fp32"}.get(args[0])
    if base == "k_h_y_split" and len(args) > 1:
        return (prec, "helmholtz_y_fwd" if args[1] == "true" else "helmholtz_y_inv")
    if base not in CLASSES:
        return None
    return (prec, CLASSES[base])


def source_sha256():
    h = hashlib.sha256()
    for f in ("kernels.hip", "fft_device.hpp"):
        h.update(open(os.path.join(PKG, "csrc", f), "rb").read())
    return h.hexdigest()


def short(name):
    return name.split("(")[0]


def _trace_durations(path):
    """Per kernel, the durations (us) of its launches in launch order."""
    rows = []
    fh = gzip.open(path, "rt") if path.endswith(".gz") else open(path)
    for r in csv.DictReader(fh):
        rows.append((int(r["Start_Timestamp"]), short(r["Kernel_Name"]),
                     (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3))
    rows.sort()
    d = collections.defaultdict(list)
    for _, k, us in rows:
        d[k].append(us)
    return d


def stats_text(path, cmd, trace=None, top=20):
    """Top kernels by total time.  With the kernel trace, also the mean over
    full launches (duration >= 20% of the kernel's longest), which leaves out
    Krylov launches that returned at once past convergence."""
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    dur = _trace_durations(trace) if trace else {}
    out = ["rocprofv3 --kernel-trace --stats summary", "command: " + cmd, "",
           "%-52s %7s %12s %10s %7s %7s %12s" % ("kernel", "calls", "total_us", "avg_us", "pct",
                                                 "full", "full_avg_us")]
    for r in rows[:top]:
        k = short(r["Name"])
        full = ""
        if k in dur:
            v = dur[k]
            f = [x for x in v if x >= 0.2 * max(v)]
            full = "%7d %12.2f" % (len(f), sum(f) / len(f))
        out.append("%-52s %7d %12.1f %10.2f %7.2f %s" % (
            k[:52], int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
            float(r["AverageNs"]) / 1e3, float(r["Percentage"]), full))
    return "\n".join(out) + "\n"


def _counter(dirpath, name):
    """Per kernel, the counter value of each dispatch, in dispatch order."""
    path = glob.glob(os.path.join(dirpath, "*counter_collection.csv"))[0]
    rows = []
    for i, r in enumerate(csv.DictReader(open(path))):
        if r["Counter_Name"] == name:
            order = int(r["Dispatch_Id"]) if r.get("Dispatch_Id", "").isdigit() else i
            rows.append((order, short(r["Kernel_Name"]), float(r["Counter_Value"])))
    rows.sort()
    agg = collections.defaultdict(list)
    for _, k, v in rows:
        agg[k].append(v)
    return agg


def _full_mean(v):
    m = max(v)
    full = [x for x in v if x >= 0.5 * m]
    return sum(full) / len(full), len(full)


def counters(fetch_dir, write_dir, copy_mib, cmd):
    F = _counter(fetch_dir, "FETCH_SIZE")
    W = _counter(write_dir, "WRITE_SIZE")
    true_kib = copy_mib * 1024.0
    cf = true_kib / max(F["__amd_rocclr_copyBuffer"])
    cw = true_kib / max(W["__amd_rocclr_copyBuffer"])
    lines = ["rocprofv3 --pmc FETCH_SIZE / --pmc WRITE_SIZE (separate runs)",
             "command: " + cmd,
             "calibration: %d MiB device copy reads %.0f KiB (FETCH_SIZE) and writes %.0f KiB"
             " (WRITE_SIZE) -> scale fetch x%.3f, write x%.3f" % (
                 copy_mib, max(F["__amd_rocclr_copyBuffer"]), max(W["__amd_rocclr_copyBuffer"]),
                 cf, cw), "",
             "%-46s %6s %14s %14s %12s" % ("kernel", "full", "fetch_MB", "write_MB", "total_MB")]
    rec = {"source_sha256": source_sha256(), "fetch_scale": cf, "write_scale": cw,
           "kernels": {}}
    for k in sorted(F, key=lambda k: -sum(F[k])):
        if k.startswith("__amd") or k not in W:
            continue
        f, nf = _full_mean(F[k])
        w, _ = _full_mean(W[k])
        fb, wb = f * cf * 1024, w * cw * 1024
        lines.append("%-46s %6d %14.1f %14.1f %12.1f" % (k[:46], nf, fb / 1e6, wb / 1e6,
                                                          (fb + wb) / 1e6))
        fc = classify(k)
        key = "%s/%s" % fc if fc and fc[0] else None
        # several instantiations share a class (grid lengths, tile budgets of
        # the autotuner's trial launches): keep the one that moved the most
        # bytes over the run, i.e. the benchmark's own (first in this order)
        if key and key not in rec["kernels"]:
            rec["kernels"][key] = dict(kernel=k, bytes_per_launch=round(fb + wb),
                                       fetch_bytes=round(fb), write_bytes=round(wb))
    return "\n".join(lines) + "\n", rec


def rates(trace, fetch_dir, write_dir, copy_mib, cmd_trace, cmd_counters, peak_gbs=8000.0,
          top=24):
    """Achieved HBM rate of every pass: counter bytes of a full launch (the
    counter runs, calibrated on a device copy) over the mean duration of the
    full launches of the same kernel (the kernel-trace run), against the
    nominal peak.  Kernels are joined by their full template name."""
    dur = _trace_durations(trace)
    F = _counter(fetch_dir, "FETCH_SIZE")
    W = _counter(write_dir, "WRITE_SIZE")
    cf = copy_mib * 1024.0 / max(F["__amd_rocclr_copyBuffer"])
    cw = copy_mib * 1024.0 / max(W["__amd_rocclr_copyBuffer"])
    rows = []
    paired = 0
    for k, v in dur.items():
        if k not in F or k not in W or k.startswith("__amd"):
            continue
        if len(v) == len(F[k]) == len(W[k]):
            # the same launches in both runs (deterministic workload): pair
            # them one by one, so that a launch's bytes go with its own
            # duration (lockstep Krylov launches cover a varying number of
            # live systems)
            b = [(f * cf + w * cw) * 1024.0 for f, w in zip(F[k], W[k])]
            bmax = max(b)
            sel = [i for i in range(len(v)) if b[i] >= 0.5 * bmax]
            tb, tu = sum(b[i] for i in sel), sum(v[i] for i in sel)
            us, mb = tu / len(sel), tb / len(sel) / 1e6
            rows.append((tu, k + " *", len(sel), us, mb, tb / tu / 1e3))
            paired += 1
            continue
        full = [x for x in v if x >= 0.2 * max(v)]
        us = sum(full) / len(full)
        mb = (_full_mean(F[k])[0] * cf + _full_mean(W[k])[0] * cw) * 1024.0 / 1e6
        rows.append((sum(full), k, len(full), us, mb, mb / us * 1e3))
    rows.sort(reverse=True)
    out = ["HBM rate per pass: rocprofv3 counter bytes / rocprofv3 kernel duration",
           "durations: " + cmd_trace, "bytes: " + cmd_counters,
           "full launches only (duration >= 20%% of the kernel's longest; bytes: counters >= 50%%"
           " of the kernel's largest); peak %.0f GB/s" % peak_gbs,
           "* = the runs launched this kernel the same number of times: launches paired one by one"
           " (bytes >= 50%% of the largest, their own durations); %d kernels paired" % paired, "",
           "%-52s %6s %10s %10s %10s %7s" % ("kernel", "full", "avg_us", "MB", "GB/s", "of_peak")]
    for _, k, n, us, mb, gbs in rows[:top]:
        out.append("%-52s %6d %10.2f %10.1f %10.0f %7.3f" % (k[:52], n, us, mb, gbs,
                                                            gbs / peak_gbs))
    return "\n".join(out) + "\n"


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_", required=True)
    a = sub.add_parser("stats")
    a.add_argument("csv")
    a.add_argument("--cmd", required=True)
    a.add_argument("--trace", help="kernel_trace.csv of the same run")
    b = sub.add_parser("counters")
    b.add_argument("fetch_dir")
    b.add_argument("write_dir")
    b.add_argument("--copy-mib", type=int, required=True)
    b.add_argument("--cmd", required=True)
    b.add_argument("--json")
    c = sub.add_parser("rates")
    c.add_argument("trace")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("--copy-mib", type=int, required=True)
    c.add_argument("--cmd-trace", required=True)
    c.add_argument("--cmd-counters", required=True)
    args = ap.parse_args()
    if args.cmd_ == "rates":
        print(rates(args.trace, args.fetch_dir, args.write_dir, args.copy_mib, args.cmd_trace,
                    args.cmd_counters), end="")
        return
    if args.cmd_ == "stats":
        print(stats_text(args.csv, args.cmd, args.trace), end="")
    else:
        text, rec = counters(args.fetch_dir, args.write_dir, args.copy_mib, args.cmd)
        print(text, end="")
        if args.json:
            json.dump(rec, open(args.json, "w"), indent=1)


if __name__ == "__main__":
    main()
