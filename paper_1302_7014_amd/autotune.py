"""Schedule autotuner for batched IBLT listing.

``iblt_list_batched`` takes a schedule: threads per workgroup (256, 512 or
1024) and the size below which a table is listed from LDS instead of in place.
Which is fastest depends on the mix of table sizes, so the tuner times every
candidate on the caller's own batch and keeps the fastest.  Listing consumes
the tables, so they are snapshotted once and restored before every trial; the
tables end restored to their input state.
"""
from __future__ import annotations

import itertools

import torch

from . import binding as pk

THREADS = (256, 512, 1024)
LDS_LIMITS = (0, pk.IBLT_LDS_MAX_CELLS)


def candidates() -> list[dict]:
    return [{"block_threads": t, "lds_max_cells": l} for t, l in itertools.product(THREADS, LDS_LIMITS)]


def tune_batched(tables: list[pk.BatchTable], entries: torch.Tensor, max_cells: int,
                 max_rounds: int, ws: torch.Tensor, reps: int = 2,
                 cands: list[dict] | None = None) -> tuple[dict, list[dict]]:
    """Returns (fastest schedule, [{schedule..., "ms": best time}] for every candidate)."""
    cands = candidates() if cands is None else cands
    snap = [t.cells.clone() for t in tables]
    stream = torch.cuda.current_stream()

    def restore():
        for t, s in zip(tables, snap):
            t.cells.copy_(s)
        torch.cuda.synchronize()

    trials = []
    for c in cands:
        best = float("inf")
        for _ in range(reps):
            restore()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            pk.iblt_list_batched(entries, len(tables), max_cells, max_rounds, ws=ws, stream=stream,
                                 **c)
            b.record(stream)
            b.synchronize()
            best = min(best, a.elapsed_time(b))
        trials.append({**c, "ms": best})
    restore()
    del snap
    win = min(trials, key=lambda x: x["ms"])
    return {k: win[k] for k in ("block_threads", "lds_max_cells")}, trials
