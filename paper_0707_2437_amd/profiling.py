"""Summaries of rocprofv3 output for the step kernels.

    # per-kernel time summary from `rocprofv3 --kernel-trace --stats -f csv`
    python -m paper_0707_2437_amd.profiling stats <..._kernel_stats.csv>

    # the same from the dispatch trace, split by launch grid (one kernel
    # stepping lattices of different sizes shows one line per grid)
    python -m paper_0707_2437_amd.profiling trace <..._kernel_trace.csv> [--kernel REGEX]

    # HBM traffic of one kernel from two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
    # runs, scaled by the same counters on a device copy of known size
    # (--grid: only the dispatches of one launch shape)
    python -m paper_0707_2437_amd.profiling traffic --kernel REGEX \\
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --copy-bytes 1073741824 --algorithmic-bytes B [--grid N] --out traffic.json

The traffic record carries the SHA-256 of the kernel source it was measured
on; a consumer reports it only while the source is unchanged.
"""
import argparse
import csv
import hashlib
import json
import os
import re
import statistics
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(PKG, "csrc", n) for n in ("kernels.hip", "step.h", "internal.h", "batch.hip")]


def kernel_source_sha():
    """SHA-256 over the device sources of the step kernels."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def stats_summary(path, top=12):
    rows = list(csv.DictReader(open(path)))
    lines = [f"{'kernel':<90} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'share%':>7}"]
    for r in rows[:top]:
        lines.append(f"{r['Name'][:90]:<90} {int(r['Calls']):>6} {float(r['AverageNs']) / 1e3:>10.2f} "
                     f"{float(r['MinNs']) / 1e3:>10.2f} {float(r['MaxNs']) / 1e3:>10.2f} {float(r['Percentage']):>7.2f}")
    return "\n".join(lines)


def trace_summary(path, kernel_regex=None, top=20):
    """Dispatches grouped by (kernel, grid size): count and duration stats."""
    rx = re.compile(kernel_regex) if kernel_regex else None
    groups = {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        if rx and not rx.search(name):
            continue
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        wg = int(r["Workgroup_Size_X"]) * int(r["Workgroup_Size_Y"]) * int(r["Workgroup_Size_Z"])
        dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
        groups.setdefault((name, grid // max(wg, 1)), []).append(dur)
    tot = sum(sum(v) for v in groups.values()) or 1.0
    lines = [f"{'kernel':<80} {'workgroups':>10} {'calls':>6} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'share%':>7}"]
    for (name, nwg), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"{name[:80]:<80} {nwg:>10} {len(v):>6} {statistics.fmean(v):>10.2f} {min(v):>10.2f} "
                     f"{max(v):>10.2f} {100 * sum(v) / tot:>7.2f}")
    return "\n".join(lines)


def pmc_mean(path, kernel_regex, counter, grid=None):
    """Mean counter value per dispatch of the kernels whose name matches (and,
    with `grid`, whose launch grid is that many work-items: one kernel
    launched in several shapes shows one grid per shape)."""
    rx = re.compile(kernel_regex)
    vals = [float(r["Counter_Value"]) for r in csv.DictReader(open(path))
            if r["Counter_Name"] == counter and rx.search(r["Kernel_Name"])
            and (grid is None or int(r["Grid_Size"]) == grid)]
    if not vals:
        raise ValueError(f"no {counter} rows for /{kernel_regex}/ in {path}")
    return statistics.fmean(vals), len(vals)


def traffic_record(kernel_regex, fetch, write, copy_fetch, copy_write, copy_bytes, algorithmic_bytes, grid=None):
    f_kib, nf = pmc_mean(fetch, kernel_regex, "FETCH_SIZE", grid)
    w_kib, nw = pmc_mean(write, kernel_regex, "WRITE_SIZE", grid)
    cf_kib, _ = pmc_mean(copy_fetch, "copyBuffer|elementwise", "FETCH_SIZE")
    cw_kib, _ = pmc_mean(copy_write, "copyBuffer|elementwise", "WRITE_SIZE")
    # the copy reads and writes copy_bytes each: scale = true bytes / counter bytes
    sf = copy_bytes / (cf_kib * 1024.0)
    sw = copy_bytes / (cw_kib * 1024.0)
    read_b = f_kib * 1024.0 * sf
    write_b = w_kib * 1024.0 * sw
    return {
        "kernel_regex": kernel_regex,
        "grid": grid,
        "kernel_source_sha256": kernel_source_sha(),
        "dispatches": {"fetch": nf, "write": nw},
        "counter_kib_per_dispatch": {"FETCH_SIZE": f_kib, "WRITE_SIZE": w_kib},
        "copy_reference": {"bytes_each_way": copy_bytes, "FETCH_SIZE_kib": cf_kib, "WRITE_SIZE_kib": cw_kib,
                           "fetch_scale": sf, "write_scale": sw},
        "read_bytes_per_launch": read_b,
        "write_bytes_per_launch": write_b,
        "traffic_bytes_per_launch": read_b + write_b,
        "algorithmic_bytes_per_launch": algorithmic_bytes,
        "traffic_over_algorithmic": (read_b + write_b) / algorithmic_bytes,
    }


def main(argv=None):
    p = argparse.ArgumentParser()
    sub = p.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    tr = sub.add_parser("trace")
    tr.add_argument("csv")
    tr.add_argument("--kernel", default=None)
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True, help="regex selecting the kernel's dispatches")
    t.add_argument("--name", required=True, help="kernel name as the benchmark reports it")
    for k in ("fetch", "write", "copy-fetch", "copy-write", "out"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--grid", type=int, default=None, help="only dispatches with this many work-items")
    a = p.parse_args(argv)
    if a.cmd == "stats":
        print(stats_summary(a.csv))
    elif a.cmd == "trace":
        print(trace_summary(a.csv, a.kernel))
    else:
        rec = traffic_record(a.kernel, a.fetch, a.write, a.copy_fetch, a.copy_write, a.copy_bytes,
                             a.algorithmic_bytes, a.grid)
        rec["kernel"] = a.name
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
        json.dump(rec, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
