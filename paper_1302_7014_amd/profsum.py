"""Summarise rocprofv3 output for the records under ``profiles/``.

    python -m paper_1302_7014_amd.profsum kernels <rocprof_dir> [--match REGEX]
        per-kernel calls / average / total time from a --kernel-trace --stats run
        (the rocpd database or the *_kernel_stats.csv file it wrote).
    python -m paper_1302_7014_amd.profsum pmc <rocprof_dir> <COUNTER> [--match REGEX]
        per-kernel average of a --pmc counter (counter_collection CSV or rocpd database).
    python -m paper_1302_7014_amd.profsum traffic <fetch> <write> <copy_fetch> <copy_write>
        HBM bytes per launch from FETCH_SIZE / WRITE_SIZE runs, calibrated on a plain copy.

Only reads files; prints a Markdown table.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import re
import sqlite3
from collections import defaultdict


def _short(name: str) -> str:
    m = re.search(r"\b(k_\w+)(<[^>]*>)?", name)
    return (m.group(1) + (m.group(2) or "")) if m else name[:60]


def kernel_stats(path: str) -> list[tuple[str, int, float, float]]:
    """[(kernel, calls, avg_us, total_us)] sorted by total time."""
    rows = []
    dbs = glob.glob(os.path.join(path, "**", "*.db"), recursive=True)
    csvs = glob.glob(os.path.join(path, "**", "*kernel_stats.csv"), recursive=True)
    if csvs:
        with open(csvs[0]) as f:
            for r in csv.DictReader(f):
                rows.append((r["Name"], int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                             float(r["TotalDurationNs"]) / 1e3))
    elif dbs:
        db = sqlite3.connect(dbs[0])
        for name, start, end in db.execute("select name, start, end from kernels"):
            rows.append((name, 1, (end - start) / 1e3, (end - start) / 1e3))
        agg = defaultdict(lambda: [0, 0.0])
        for name, _, _, tot in rows:
            agg[name][0] += 1
            agg[name][1] += tot
        rows = [(k, c, t / c, t) for k, (c, t) in agg.items()]
    rows.sort(key=lambda r: -r[3])
    return rows


def pmc_means(path: str, counter: str) -> dict[str, tuple[int, float]]:
    """{kernel: (dispatches, mean counter value per dispatch)} from the counter_collection
    CSVs or the rocpd database of a --pmc run."""
    acc = defaultdict(lambda: defaultdict(float))
    csvs = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    for fn in csvs:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                acc[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    if not csvs:
        for fn in glob.glob(os.path.join(path, "**", "*.db"), recursive=True):
            db = sqlite3.connect(fn)
            q = "select kernel_name, dispatch_id, value from counters_collection where counter_name = ?"
            for name, disp, val in db.execute(q, (counter,)):
                acc[name][disp] += float(val)
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in acc.items() if v}


def traffic(fetch_dir: str, write_dir: str, copy_fetch_dir: str, copy_write_dir: str,
            copy_bytes: int, pattern: str) -> dict:
    """HBM bytes per launch of the kernels matching ``pattern``: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by bytes / counter for a plain copy of ``copy_bytes``."""
    pat = re.compile(pattern)

    def copy_factor(d, counter):
        vals = [mean for name, (_, mean) in pmc_means(d, counter).items() if "copyBuffer" in name]
        return copy_bytes / (vals[0] * 1024.0)

    ff = copy_factor(copy_fetch_dir, "FETCH_SIZE")
    wf = copy_factor(copy_write_dir, "WRITE_SIZE")
    out = {"fetch_factor": ff, "write_factor": wf, "kernels": {}}
    fetch = pmc_means(fetch_dir, "FETCH_SIZE")
    write = pmc_means(write_dir, "WRITE_SIZE")
    for name in sorted(set(fetch) & set(write)):
        if not pat.search(name):
            continue
        fb = fetch[name][1] * 1024.0 * ff
        wb = write[name][1] * 1024.0 * wf
        out["kernels"][_short(name)] = {"fetch_bytes": fb, "write_bytes": wb,
                                        "bytes_per_launch": fb + wb}
    return out


def main() -> None:
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    k = sub.add_parser("kernels")
    k.add_argument("path")
    k.add_argument("--match", default="")
    p = sub.add_parser("pmc")
    p.add_argument("path")
    p.add_argument("counter")
    p.add_argument("--match", default="")
    t = sub.add_parser("traffic")
    for arg in ("fetch_dir", "write_dir", "copy_fetch_dir", "copy_write_dir"):
        t.add_argument(arg)
    t.add_argument("--copy-bytes", type=int, default=1 << 30)
    t.add_argument("--match", default="")
    a = ap.parse_args()
    if a.cmd == "traffic":
        import json
        print(json.dumps(traffic(a.fetch_dir, a.write_dir, a.copy_fetch_dir, a.copy_write_dir,
                                 a.copy_bytes, a.match), indent=1))
        return
    pat = re.compile(a.match) if a.match else None
    if a.cmd == "kernels":
        print("| kernel | calls | average (us) | total (us) |")
        print("|---|---:|---:|---:|")
        for name, calls, avg, tot in kernel_stats(a.path):
            if pat and not pat.search(name):
                continue
            print(f"| {_short(name)} | {calls} | {avg:.1f} | {tot:.1f} |")
    else:
        print(f"| kernel | dispatches | mean {a.counter} per dispatch |")
        print("|---|---:|---:|")
        for name, (n, mean) in sorted(pmc_means(a.path, a.counter).items()):
            if pat and not pat.search(name):
                continue
            print(f"| {_short(name)} | {n} | {mean:.1f} |")


if __name__ == "__main__":
    main()
