"""Schedule autotuner for batched IBLT listing, per size class.

``iblt_list_batched`` takes a schedule: threads per workgroup (256, 512 or
1024), the size up to which a table is listed from LDS, and the size from
which a table is listed by a team of workgroups (and the team's size); any
other table is listed in place by one workgroup.  Which schedule wins depends
on the table sizes and on how many tables share the GPU, so the tuner times
the candidates on the caller's own tables, one size class at a time:

- small tables (at most ``IBLT_LDS_MAX_CELLS`` cells): LDS-resident (as far
  as the thread count's LDS holds them, ``IBLT_LDS_CELLS``) or in place, for
  each thread count;
- medium tables: in place, for each thread count;
- large tables (at least ``LARGE_MIN`` cells): one workgroup each, or teams
  of 2 to 32 workgroups, for each thread count.

Each class is timed as a batch of its own tables.  The launch takes one
thread count for every table, so the classes' choices are then combined and
the thread count is taken from a last round of trials on the whole batch.
Listing consumes the tables, so the tables being timed are snapshotted and
restored before every trial; every table ends restored to its input state.
"""
from __future__ import annotations

import torch

from . import binding as pk

THREADS = (256, 512, 1024)
LARGE_MIN = 1 << 17
TEAMS = (0, 2, 4, 8, 16, 32)
KEYS = ("block_threads", "lds_max_cells", "tile_min_cells", "tile_workgroups")


def size_class(ncells: int) -> str:
    if ncells <= pk.IBLT_LDS_MAX_CELLS:
        return "small"
    return "large" if ncells >= LARGE_MIN else "medium"


def class_candidates(cls: str) -> list[dict]:
    out = []
    for t in THREADS:
        if cls == "small":
            for lds in (0, pk.IBLT_LDS_MAX_CELLS):
                out.append({"block_threads": t, "lds_max_cells": lds, "tile_min_cells": 0,
                            "tile_workgroups": 0})
        elif cls == "medium":
            out.append({"block_threads": t, "lds_max_cells": 0, "tile_min_cells": 0,
                        "tile_workgroups": 0})
        else:
            for g in TEAMS:
                out.append({"block_threads": t, "lds_max_cells": 0,
                            "tile_min_cells": LARGE_MIN if g else 0, "tile_workgroups": g})
    return out


def _time(tables, entries, max_cells, max_rounds, ws, sched, reps, stream) -> float:
    snap = [t.cells.clone() for t in tables]
    best = float("inf")
    for _ in range(reps):
        for t, s in zip(tables, snap):
            t.cells.copy_(s)
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        pk.iblt_list_batched(entries, len(tables), max_cells, max_rounds, ws=ws, stream=stream,
                             **sched)
        b.record(stream)
        b.synchronize()
        best = min(best, a.elapsed_time(b))
    for t, s in zip(tables, snap):
        t.cells.copy_(s)
    torch.cuda.synchronize()
    return best


def tune_batched(tables: list[pk.BatchTable], entries: torch.Tensor, max_cells: int,
                 max_rounds: int, ws: torch.Tensor, reps: int = 2) -> tuple[dict, dict]:
    """Returns (schedule for the whole batch, report).  The report holds, per
    size class, its table count, every candidate's time on the class's own
    tables and the class's choice, then the whole-batch trials of the thread
    counts with the classes' choices combined."""
    stream = torch.cuda.current_stream()
    classes: dict[str, list[int]] = {}
    for i, t in enumerate(tables):
        classes.setdefault(size_class(t.desc.ncells), []).append(i)
    report: dict = {"classes": {}, "combined": []}
    choice = {"lds_max_cells": 0, "tile_min_cells": 0, "tile_workgroups": 0}
    for cls in ("small", "medium", "large"):
        idx = classes.get(cls)
        if not idx:
            continue
        sub = [tables[i] for i in idx]
        ent = pk.batch_entries(sub, entries.device)
        mc = max(t.desc.ncells for t in sub)
        trials = []
        for c in class_candidates(cls):
            trials.append({**c, "ms": _time(sub, ent, mc, max_rounds, ws, c, reps, stream)})
        win = min(trials, key=lambda x: x["ms"])
        report["classes"][cls] = {"tables": len(idx), "trials": trials,
                                  "choice": {k: win[k] for k in KEYS}}
        if cls == "small":
            choice["lds_max_cells"] = win["lds_max_cells"]
        elif cls == "large":
            choice["tile_min_cells"] = win["tile_min_cells"]
            choice["tile_workgroups"] = win["tile_workgroups"]
    for t in THREADS:
        sched = {"block_threads": t, **choice}
        report["combined"].append({**sched, "ms": _time(tables, entries, max_cells, max_rounds, ws,
                                                        sched, reps, stream)})
    win = min(report["combined"], key=lambda x: x["ms"])
    return {k: win[k] for k in KEYS}, report
