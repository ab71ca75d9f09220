"""Summaries of rocprofv3 output for the step kernels.

    # per-kernel time summary from `rocprofv3 --kernel-trace --stats -f csv`
    python -m paper_0707_2437_amd.profiling stats <..._kernel_stats.csv>

    # the same from the dispatch trace, split by launch grid (one kernel
    # stepping lattices of different sizes shows one line per grid)
    python -m paper_0707_2437_amd.profiling trace <..._kernel_trace.csv> [--kernel REGEX]

    # HBM traffic of one kernel from two rocprofv3 --pmc runs of counters
    # whose units are fixed (read requests of 32, 64 and 128 bytes, and DRAM
    # reads in 32-byte units; write requests and those of 64 bytes), with
    # the same counters on a device copy of known size as a check of the
    # units (--grid: only the dispatches of one launch shape)
    python -m paper_0707_2437_amd.profiling traffic --kernel REGEX --name NAME \\
        --reads R.csv --writes W.csv --copy-reads CR.csv --copy-writes CW.csv \\
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
# Device sources of the single-lattice step kernels and of the batched kernels.
KERNEL_SOURCES = {
    "step": [os.path.join(PKG, "csrc", n) for n in ("kernels.hip", "step.h", "internal.h")],
    "batch": [os.path.join(PKG, "csrc", n) for n in ("batch.hip", "step.h", "internal.h")],
    "step2": [os.path.join(PKG, "csrc", n) for n in ("step2.hip", "step2.h", "step.h", "internal.h")],
}


def kernel_source_sha(which="step"):
    """SHA-256 over the device sources of the single-step ("step"), two-step
    ("step2") or batched ("batch") kernels."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES[which]:
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


def most_common_grid(path, kernel_regex):
    """The launch grid (work-items) of most dispatches of the matching kernels."""
    rx = re.compile(kernel_regex)
    grids = [int(r["Grid_Size"]) for r in csv.DictReader(open(path)) if rx.search(r["Kernel_Name"])]
    if not grids:
        raise ValueError(f"no dispatches of /{kernel_regex}/ in {path}")
    return max(set(grids), key=grids.count)


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


# Counters of the two passes (at most 4 TCC counters fit one pass).
READ_COUNTERS = ["TCC_EA0_RDREQ_32B_sum", "TCC_EA0_RDREQ_64B_sum", "TCC_EA0_RDREQ_128B_sum",
                 "TCC_EA0_RDREQ_DRAM_32B_sum"]
WRITE_COUNTERS = ["TCC_EA0_WRREQ_sum", "TCC_EA0_WRREQ_64B_sum"]


def read_bytes(path, kernel_regex, grid=None):
    """L2-to-memory read bytes per dispatch: 32, 64 and 128 bytes per request
    of each size; and the DRAM reads, counted in 32-byte units."""
    n32, nd = pmc_mean(path, kernel_regex, "TCC_EA0_RDREQ_32B_sum", grid)
    n64, _ = pmc_mean(path, kernel_regex, "TCC_EA0_RDREQ_64B_sum", grid)
    n128, _ = pmc_mean(path, kernel_regex, "TCC_EA0_RDREQ_128B_sum", grid)
    d32, _ = pmc_mean(path, kernel_regex, "TCC_EA0_RDREQ_DRAM_32B_sum", grid)
    return {"requests_32B": n32, "requests_64B": n64, "requests_128B": n128, "dram_32B_units": d32,
            "bytes": 32.0 * n32 + 64.0 * n64 + 128.0 * n128, "dram_bytes": 32.0 * d32, "dispatches": nd}


def write_bytes(path, kernel_regex, grid=None):
    """L2-to-memory write bytes per dispatch: 64 bytes per 64-byte request, 32
    per other request."""
    n, nd = pmc_mean(path, kernel_regex, "TCC_EA0_WRREQ_sum", grid)
    n64, _ = pmc_mean(path, kernel_regex, "TCC_EA0_WRREQ_64B_sum", grid)
    return {"requests": n, "requests_64B": n64, "bytes": 64.0 * n64 + 32.0 * (n - n64), "dispatches": nd}


COPY_REGEX = "copyBuffer"


def traffic_record(kernel_regex, reads, writes, copy_reads, copy_writes, copy_bytes, algorithmic_bytes, grid=None,
                   sources="step"):
    r = read_bytes(reads, kernel_regex, grid)
    w = write_bytes(writes, kernel_regex, grid)
    cr = read_bytes(copy_reads, COPY_REGEX)
    cw = write_bytes(copy_writes, COPY_REGEX)
    return {
        "kernel_regex": kernel_regex,
        "grid": grid,
        "kernel_sources": sources,
        "kernel_source_sha256": kernel_source_sha(sources),
        "counters": {"reads": READ_COUNTERS, "writes": WRITE_COUNTERS},
        "reads_per_dispatch": r,
        "writes_per_dispatch": w,
        # the same counters on a copy that reads and writes copy_bytes: a
        # check of the units (each ratio should be 1)
        "copy_check": {"bytes_each_way": copy_bytes, "read_ratio": cr["bytes"] / copy_bytes,
                       "dram_read_ratio": cr["dram_bytes"] / copy_bytes, "write_ratio": cw["bytes"] / copy_bytes},
        "read_bytes_per_launch": r["bytes"],
        "write_bytes_per_launch": w["bytes"],
        "traffic_bytes_per_launch": r["bytes"] + w["bytes"],
        "algorithmic_bytes_per_launch": algorithmic_bytes,
        "read_over_algorithmic": r["bytes"] / (algorithmic_bytes / 2),
        "write_over_algorithmic": w["bytes"] / (algorithmic_bytes / 2),
        "traffic_over_algorithmic": (r["bytes"] + w["bytes"]) / algorithmic_bytes,
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
    for k in ("reads", "writes", "copy-reads", "copy-writes", "out"):
        t.add_argument("--" + k, required=True)
    t.add_argument("--copy-bytes", type=float, default=float(1 << 30))
    t.add_argument("--algorithmic-bytes", type=float, required=True)
    t.add_argument("--grid", default=None,
                   help="only dispatches with this many work-items ('auto': the most common grid)")
    t.add_argument("--sources", default="step", choices=sorted(KERNEL_SOURCES),
                   help="which kernels' sources the record is tied to")
    a = p.parse_args(argv)
    if a.cmd == "stats":
        print(stats_summary(a.csv))
    elif a.cmd == "trace":
        print(trace_summary(a.csv, a.kernel))
    else:
        grid = a.grid
        if grid == "auto":
            grid = most_common_grid(a.reads, a.kernel)
        elif grid is not None:
            grid = int(grid)
        rec = traffic_record(a.kernel, a.reads, a.writes, a.copy_reads, a.copy_writes, a.copy_bytes,
                             a.algorithmic_bytes, grid, a.sources)
        rec["kernel"] = a.name
        with open(a.out, "w") as f:
            json.dump(rec, f, indent=1)
        json.dump(rec, sys.stdout, indent=1)
        print()


if __name__ == "__main__":
    main()
