"""Summarise rocprofv3 output for the records under ``profiles/``.

    python -m paper_1302_7014_amd.profsum kernels <rocprof_dir> [--match REGEX]
        per-kernel calls / average / total time from a --kernel-trace --stats run
        (the rocpd database or the *_kernel_stats.csv file it wrote).
    python -m paper_1302_7014_amd.profsum pmc <rocprof_dir> <COUNTER> [--match REGEX]
        per-kernel average of a --pmc counter (*_counter_collection.csv).

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
    """{kernel: (dispatches, mean counter value per dispatch)} from counter_collection CSVs."""
    acc = defaultdict(lambda: defaultdict(float))
    for fn in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") != counter:
                    continue
                acc[r["Kernel_Name"]][r["Dispatch_Id"]] += float(r["Counter_Value"])
    return {k: (len(v), sum(v.values()) / len(v)) for k, v in acc.items() if v}


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
    a = ap.parse_args()
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
