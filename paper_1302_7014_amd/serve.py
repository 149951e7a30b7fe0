"""Continuous-batching IBLT decode server on one GPU.

Requests are IBLT list jobs of mixed sizes.  The server keeps every admitted
table resident in a fixed HBM arena (the budget), admits arrivals first come
first served as arena space frees up, and runs the GPU as a pipeline:

* admission: the request's table and buffers are carved from the arena, its
  keys are produced on the device by the caller's ``fill_keys`` and inserted
  on the insert stream (this stands for receiving the table), overlapping
  whatever listing is running: with ``iblt_insert``, or for a table of 2^18
  cells and more (larger than an XCD's L2) with the binned ``iblt_update``;
* listing, routed by table size: a table of more than ``small_cells`` cells is
  listed alone by ``iblt_list`` on one of ``large_lanes`` streams (taken in
  turn), as soon as its insert is done.  Each lane's runs use an equal share
  of the CUs, so runs on all lanes are resident together; a run on a
  mid-sized table is bound by its per-round barriers, and runs on several
  lanes overlap well.  The small tables that are
  inserted and not yet listed are listed together in one
  ``iblt_list_batched`` launch (one workgroup per table) on a small-lane
  stream, up to ``max_inflight`` such launches at once.  One workgroup lists a
  small table about as fast as the whole chip does;
* retirement: when a launch's completion event fires, its requests complete,
  their arena space is freed and their results (the summary) are kept.

``FifoServer`` is the plain baseline: one request at a time, insert then
``iblt_list`` on one stream.

Latency of a request = (host clock when its completion is observed) - (its
arrival time on the same clock).  The loop polls events with short sleeps.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as pk

_ALIGN = 256


@dataclass
class Request:
    rid: int
    arrival: float     # seconds after the start of the run
    r: int
    ncells: int
    nkeys: int
    key_seed: int
    table_seed: int
    # filled by the server
    admitted: float = -1.0
    done: float = -1.0
    summary: np.ndarray | None = None
    keys_out: np.ndarray | None = None
    _alloc: list = field(default_factory=list, repr=False)
    _table: object = field(default=None, repr=False)
    _event: object = field(default=None, repr=False)

    def footprint(self, max_rounds: int) -> int:
        """Arena bytes: cells (32 B each), output keys (8 B per cell), the inserted
        keys (8 B each), round stats and summary."""
        pieces = [32 * self.ncells, 8 * self.ncells, 8 * max(self.nkeys, 1), 8 * max_rounds, 64]
        return sum(_round(p) for p in pieces)


def _round(n: int) -> int:
    return (n + _ALIGN - 1) // _ALIGN * _ALIGN


class Arena:
    """First-fit allocator over one device buffer of ``budget`` bytes (the HBM budget)."""

    def __init__(self, budget: int, device):
        self.budget = _round(budget)
        self.buf = torch.empty(self.budget, dtype=torch.uint8, device=device)
        self.free_list = [(0, self.budget)]  # (offset, size), sorted by offset
        self.used = 0
        self.peak = 0

    def alloc(self, nbytes: int):
        nbytes = _round(nbytes)
        for i, (off, size) in enumerate(self.free_list):
            if size >= nbytes:
                if size == nbytes:
                    self.free_list.pop(i)
                else:
                    self.free_list[i] = (off + nbytes, size - nbytes)
                self.used += nbytes
                self.peak = max(self.peak, self.used)
                return off, nbytes
        return None

    def free(self, off: int, nbytes: int) -> None:
        self.used -= nbytes
        fl = self.free_list
        lo, hi = 0, len(fl)
        while lo < hi:
            mid = (lo + hi) // 2
            if fl[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        fl.insert(lo, (off, nbytes))
        # merge with the neighbours
        if lo + 1 < len(fl) and fl[lo][0] + fl[lo][1] == fl[lo + 1][0]:
            fl[lo] = (fl[lo][0], fl[lo][1] + fl[lo + 1][1])
            fl.pop(lo + 1)
        if lo > 0 and fl[lo - 1][0] + fl[lo - 1][1] == fl[lo][0]:
            fl[lo - 1] = (fl[lo - 1][0], fl[lo - 1][1] + fl[lo][1])
            fl.pop(lo)

    def view(self, off: int, nbytes: int, dtype) -> torch.Tensor:
        return self.buf[off: off + nbytes].view(dtype)


class _Base:
    def __init__(self, budget: int, fill_keys, max_rounds: int = 256, keep_keys: bool = False,
                 device="cuda"):
        self.device = torch.device(device)
        self.arena = Arena(budget, self.device)
        self.fill_keys = fill_keys
        self.max_rounds = max_rounds
        self.keep_keys = keep_keys
        self.rejected = []
        # tables from this size on (larger than an XCD's L2) are filled with the
        # binned update; admissions run in order on one stream, so they share
        # one workspace, grown as needed (outside the arena, like the list
        # workspaces)
        self.binned_min_cells = 1 << 18
        self.upd_ws = None

    def _admit(self, q: Request, stream) -> bool:
        pieces = [32 * q.ncells, 8 * q.ncells, 8 * max(q.nkeys, 1), 8 * self.max_rounds, 64]
        got = []
        for p in pieces:
            a = self.arena.alloc(p)
            if a is None:
                for off, nb in got:
                    self.arena.free(off, nb)
                return False
            got.append(a)
        q._alloc = got
        (co, cn), (ko, kn), (io, inn), (so, sn), (mo, mn) = got
        cells = self.arena.view(co, cn, torch.int64)[: 4 * q.ncells].view(q.ncells, 4)
        keys_out = self.arena.view(ko, kn, torch.int64)[: q.ncells]
        ins = self.arena.view(io, inn, torch.int64)[: max(q.nkeys, 1)]
        stats = self.arena.view(so, sn, torch.int64)[: self.max_rounds]
        summ = self.arena.view(mo, mn, torch.int64)[:8]
        desc = pk.iblt_desc(q.ncells, q.r, q.table_seed)
        with torch.cuda.stream(stream):
            cells.zero_()
            if q.nkeys:
                self.fill_keys(q, ins[: q.nkeys])
                if q.ncells >= self.binned_min_cells:
                    need = pk.iblt_update_workspace(desc, q.nkeys)
                    if self.upd_ws is None or self.upd_ws.numel() < need:
                        torch.cuda.current_stream().wait_stream(stream)
                        grown = 2 * self.upd_ws.numel() if self.upd_ws is not None else 0
                        self.upd_ws = pk.workspace(max(need, grown), self.device)
                        self.upd_ws.record_stream(stream)
                        stream.wait_stream(torch.cuda.current_stream())
                    pk.iblt_update(desc, cells, ins[: q.nkeys], 1, ws=self.upd_ws, stream=stream)
                else:
                    pk.iblt_insert(desc, cells, ins[: q.nkeys], stream=stream)
        q._table = pk.BatchTable(desc, cells, keys_out, stats, summ)
        return True

    def _retire(self, q: Request, now: float, summary: np.ndarray | None = None) -> None:
        q.done = now
        q.summary = q._table.summary.cpu().numpy().copy() if summary is None else summary
        if self.keep_keys:
            listed = int(q.summary[0])
            q.keys_out = q._table.keys[:listed].cpu().numpy().view(np.uint64).copy()
            q.round_stats = q._table.round_stats[: int(q.summary[1])].cpu().numpy().view(np.uint64).copy()
        for off, nb in q._alloc:
            self.arena.free(off, nb)
        q._alloc = []
        q._table = None


class ContinuousServer(_Base):
    """Continuous batching with size routing (see the module docstring)."""

    def __init__(self, budget: int, fill_keys, max_cells: int, max_rounds: int = 256,
                 max_inflight: int = 2, block_threads: int = 512, small_cells: int = 1 << 12,
                 large_lanes: int = 4, admit_group: int = 8, keep_keys: bool = False,
                 device="cuda", max_r: int = 8):
        super().__init__(budget, fill_keys, max_rounds, keep_keys, device)
        self.max_cells = max_cells
        self.max_inflight = max_inflight
        self.block_threads = block_threads
        self.small_cells = small_cells
        self.insert_stream = torch.cuda.Stream(device=self.device)
        self.list_streams = [torch.cuda.Stream(device=self.device) for _ in range(max_inflight)]
        self.admit_group = admit_group
        # each large lane: a stream, an equal share of the CUs for its listing's
        # persistent workgroups (so that every lane's run gets its whole team at
        # once), and a listing workspace for the largest table
        cus = torch.cuda.get_device_properties(self.device).multi_processor_count
        self.lane_workgroups = max(1, cus // large_lanes)
        self.large_streams = [torch.cuda.Stream(device=self.device) for _ in range(large_lanes)]
        # (the listing's workspace grows with r: sized for the largest r served)
        self.large_ws = [pk.workspace(pk.iblt_list_workspace(
            pk.iblt_desc(max_cells, max_r, 0, self.lane_workgroups)), self.device)
            for _ in range(large_lanes)]
        # one batched-listing workspace per in-flight launch, sized for the largest small table
        self.ws = [pk.workspace(pk.iblt_list_batched_workspace(1 << 16, min(small_cells, max_cells)),
                                self.device) for _ in range(max_inflight)]
        self.batches = 0
        self.large = 0

    def _list_large(self, q: Request, lane: int) -> torch.cuda.Event:
        s = self.large_streams[lane]
        s.wait_event(q._event)
        t = q._table
        d = pk.iblt_desc(t.desc.ncells, t.desc.r, t.desc.seed, self.lane_workgroups)
        with torch.cuda.stream(s):
            pk.iblt_list(d, t.cells, max_rounds=self.max_rounds,
                         out=pk.ListOut(t.keys, t.round_stats, t.summary),
                         ws=self.large_ws[lane], stream=s)
        ev = torch.cuda.Event()
        ev.record(s)
        self.large += 1
        return ev

    def run(self, requests: list[Request], poll_s: float = 2e-5) -> list[Request]:
        pending = sorted(requests, key=lambda q: q.arrival)
        waiting: list[Request] = []      # arrived, not admitted
        ready: list[Request] = []        # small tables inserted, not listed
        inflight: list[tuple] = []       # (event, requests, slot, entries) of batched launches
        lanes = [[] for _ in self.large_streams]  # per large lane: (event, request) in order
        next_lane = 0
        free_slots = list(range(self.max_inflight))
        done: list[Request] = []
        t0 = time.perf_counter()
        i = 0
        while len(done) + len(self.rejected) < len(requests):
            now = time.perf_counter() - t0
            while i < len(pending) and pending[i].arrival <= now:
                waiting.append(pending[i])
                i += 1
            # admit in arrival order while the arena has room, a few at a time so
            # that listing starts while later arrivals are still being admitted
            admitted = []
            while waiting and len(admitted) < self.admit_group:
                q = waiting[0]
                if q.footprint(self.max_rounds) > self.arena.budget:
                    self.rejected.append(waiting.pop(0))
                    continue
                if not self._admit(q, self.insert_stream):
                    break
                q.admitted = now
                admitted.append(waiting.pop(0))
            if admitted:
                ev = torch.cuda.Event()
                ev.record(self.insert_stream)
                for q in admitted:
                    q._event = ev
                    if q.ncells > self.small_cells:
                        lanes[next_lane].append((self._list_large(q, next_lane), q))
                        next_lane = (next_lane + 1) % len(lanes)
                    else:
                        ready.append(q)
            # retire finished work: each large lane completes in launch order
            for lane in lanes:
                while lane and lane[0][0].query():
                    q = lane.pop(0)[1]
                    self._retire(q, time.perf_counter() - t0)
                    done.append(q)
            still = []
            for ev, qs, slot, ent in inflight:
                if ev.query():
                    tnow = time.perf_counter() - t0
                    # the batch's summaries in one copy rather than one per table
                    sums = torch.stack([q._table.summary for q in qs]).cpu().numpy()
                    for q, srow in zip(qs, sums):
                        self._retire(q, tnow, srow.copy())
                        done.append(q)
                    free_slots.append(slot)
                else:
                    still.append((ev, qs, slot, ent))
            inflight = still
            # launch the ready small tables as one batch
            if ready and free_slots:
                slot = free_slots.pop()
                s = self.list_streams[slot]
                qs = sorted(ready, key=lambda q: -q.ncells)
                ready = []
                for ev in {id(q._event): q._event for q in qs}.values():
                    s.wait_event(ev)
                with torch.cuda.stream(s):
                    ent = pk.batch_entries([q._table for q in qs], self.device)
                    pk.iblt_list_batched(ent, len(qs), max(q.ncells for q in qs), self.max_rounds,
                                         block_threads=self.block_threads, ws=self.ws[slot],
                                         stream=s)
                ev = torch.cuda.Event()
                ev.record(s)
                inflight.append((ev, qs, slot, ent))
                self.batches += 1
            if (i >= len(pending) and not waiting and not ready and not inflight
                    and not any(lanes)):
                break
            if not waiting:
                time.sleep(poll_s)
        return done


class FifoServer(_Base):
    """Plain baseline: one request at a time, insert then iblt_list, one stream."""

    def __init__(self, budget: int, fill_keys, max_rounds: int = 256, keep_keys: bool = False,
                 device="cuda", max_cells: int = 1 << 22, max_r: int = 8):
        super().__init__(budget, fill_keys, max_rounds, keep_keys, device)
        self.stream = torch.cuda.Stream(device=self.device)
        self.ws = pk.workspace(pk.iblt_list_workspace(pk.iblt_desc(max_cells, max_r, 0)),
                               self.device)

    def run(self, requests: list[Request], poll_s: float = 2e-5) -> list[Request]:
        pending = sorted(requests, key=lambda q: q.arrival)
        done = []
        t0 = time.perf_counter()
        for q in pending:
            while time.perf_counter() - t0 < q.arrival:
                time.sleep(poll_s)
            if q.footprint(self.max_rounds) > self.arena.budget or not self._admit(q, self.stream):
                self.rejected.append(q)
                continue
            q.admitted = time.perf_counter() - t0
            t = q._table
            out = pk.ListOut(t.keys, t.round_stats, t.summary)
            with torch.cuda.stream(self.stream):
                pk.iblt_list(t.desc, t.cells, max_rounds=self.max_rounds, out=out, ws=self.ws,
                             stream=self.stream)
            self.stream.synchronize()
            self._retire(q, time.perf_counter() - t0)
            done.append(q)
        return done


def latency_stats(done: list[Request]) -> dict:
    lat = np.array([q.done - q.arrival for q in done]) if done else np.zeros(1)
    span = (max(q.done for q in done) - min(q.arrival for q in done)) if done else 0.0
    return {
        "requests": len(done),
        "p50_ms": float(np.percentile(lat, 50) * 1e3),
        "p99_ms": float(np.percentile(lat, 99) * 1e3),
        "mean_ms": float(lat.mean() * 1e3),
        "req_per_s": len(done) / span if span > 0 else 0.0,
    }
