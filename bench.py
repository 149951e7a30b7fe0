"""Benchmark: round-synchronous k-core peeling at n = 2^24 on one MI355X.

One step = hg_build + peel_kcore over the resident edge list of the r=4, k=2,
n=2^24, c=0.70 hypergraph (11,744,051 edges, partitioned model, seed 1): the
whole path from edges in HBM to the k-core, its per-round counts and every
vertex's and edge's removal round.  `value` is edges peeled per second over
the step.  The line also carries the roofline of the dominant kernel (HIP
events on the stream the kernels run on), the CPU oracle timed on the host
on the same workload, and secondary measurements (peel alone, IBLT insert and
list at 2^24 cells).

    python bench.py [--steps K] [--warmup W] [--gpus 1] [--no-cpu] [--no-sweep] ...
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import paper_1302_7014_amd as pk  # noqa: E402
from workloads import configs, gen  # noqa: E402

METRIC = "edges peeled/sec and HBM GB/s fraction at n=2^24; batched vs plain; p99 decode latency"
HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def peel_bytes(n, r, edges, deg0, vr, er):
    """Algorithmic HBM bytes of one peel: each word read or written once, an atomic
    or CAS read-modify-write of a w-byte word counts 2w.

    8n (read deg, write vertex_round) + 8 per removed vertex (its offsets pair)
    + 4 per incidence of a removed vertex (its edge list) + per removed edge
    8 (claim CAS) + 4r (its row) + 8(r-1) (the other slots' decrements).
    """
    removed_v = vr != 0
    m_rem = int((er != 0).sum())
    n_rem = int(removed_v.sum())
    inc_rem = int(deg0[removed_v].astype(np.int64).sum())
    return 8 * n + 8 * n_rem + 4 * inc_rem + m_rem * (8 + 4 * r + 8 * (r - 1))


def build_bytes(n, m, r):
    """Algorithmic bytes of hg_build: read edges twice (8rm), degree and cursor
    atomics (16rm), write inc (4rm), scan deg into offsets (8n)."""
    return 28 * r * m + 8 * n


def iblt_insert_bytes(m, r):
    """Per key: read it (8) and update r cells' count, key and checksum fields (r x 2 x 20)."""
    return m * (8 + 40 * r)


def iblt_list_bytes(N, r, listed):
    """Round-1 count scan (4N) + per listed key: its pure cell (20), r cell updates
    (r x 2 x 20) and the output word (8)."""
    return 4 * N + listed * (20 + 40 * r + 8)


class Timer:
    """HIP-event durations of calls made on the current stream (the stream the
    library launches on).  Recording never synchronises; collect() does, once."""

    def __init__(self):
        self.ms = []
        self._pending = []

    def __enter__(self):
        a = torch.cuda.Event(enable_timing=True)
        a.record()
        self._pending.append([a, None])
        return self

    def __exit__(self, *exc):
        b = torch.cuda.Event(enable_timing=True)
        b.record()
        self._pending[-1][1] = b
        return False

    def collect(self):
        torch.cuda.synchronize()
        self.ms.extend(a.elapsed_time(b) for a, b in self._pending)
        self._pending = []


def bench_kcore(spec, steps, warmup, subtables=False):
    log(f"generating {spec.name}: n={spec.n} m={spec.m} r={spec.r}")
    e_host = spec.edges(1)
    dev = torch.device("cuda", 0)
    e = torch.from_numpy(e_host.view(np.int32)).to(dev)
    n, m, r = spec.n, spec.m, spec.r
    csr = pk.Csr(torch.empty(n + 1, dtype=torch.int32, device=dev),
                 torch.empty(m * r, dtype=torch.int32, device=dev),
                 torch.empty(n, dtype=torch.int32, device=dev),
                 torch.empty(2, dtype=torch.int32, device=dev))
    max_rounds = 4096
    out = pk.PeelOut(csr.deg, torch.empty(n, dtype=torch.int32, device=dev),
                     torch.empty(m, dtype=torch.int32, device=dev),
                     torch.empty(2 * max_rounds, dtype=torch.int64, device=dev),
                     torch.empty(8, dtype=torch.int32, device=dev))
    ws_b = pk.workspace(pk.hg_build_workspace(n, m, r), dev)
    ws_p = pk.workspace(pk.peel_kcore_workspace(n, m, r), dev)
    tb, tp = Timer(), Timer()

    def step(timed):
        if timed:
            with tb:
                pk.hg_build(e, n, out=csr, ws=ws_b)
            with tp:
                pk.peel_kcore(e, n, spec.k, csr, max_rounds=max_rounds, out=out, ws=ws_p,
                              subtables=subtables)
        else:
            pk.hg_build(e, n, out=csr, ws=ws_b)
            pk.peel_kcore(e, n, spec.k, csr, max_rounds=max_rounds, out=out, ws=ws_p,
                          subtables=subtables)

    for _ in range(warmup):
        step(False)
    torch.cuda.synchronize()
    # the degrees right after hg_build, for the byte model
    pk.hg_build(e, n, out=csr, ws=ws_b)
    torch.cuda.synchronize()
    deg0 = csr.deg.cpu().numpy().view(np.uint32).copy()

    # the timed region: K steps between two synchronisations, each call bracketed
    # by HIP events on the stream it runs on
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step(True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    tb.collect()
    tp.collect()

    summ = out.summary.cpu().numpy().view(np.uint32)
    vr = out.vertex_round.cpu().numpy().view(np.uint32)
    er = out.edge_round.cpu().numpy().view(np.uint32)
    if int(summ[2]) != 0:
        raise RuntimeError(f"peel flags {int(summ[2])}")
    m_rem = int((er != 0).sum())
    return {
        "vr": vr, "er": er,
        "wall_s": wall, "m_removed": m_rem, "rounds": int(summ[0]), "edge_rounds": int(summ[1]),
        "core_vertices": int(summ[3]),
        "build_ms": float(np.mean(tb.ms)), "peel_ms": float(np.mean(tp.ms)),
        "build_ms_p10_p90": [float(np.percentile(tb.ms, 10)), float(np.percentile(tb.ms, 90))],
        "peel_ms_p10_p90": [float(np.percentile(tp.ms, 10)), float(np.percentile(tp.ms, 90))],
        "peel_bytes": peel_bytes(n, r, e_host, deg0, vr, er),
        "build_bytes": build_bytes(n, m, r), "edges_host": e_host,
    }


def bench_k2_xor(spec, steps, warmup, ref):
    """peel_k2_xor (no CSR: degrees and edge-id XORs per vertex) on the same
    workload: the whole k = 2 step in one call, its outputs compared with the
    build + peel_kcore run's on the device."""
    dev = torch.device("cuda", 0)
    e = torch.from_numpy(ref["edges_host"].view(np.int32)).to(dev).view(spec.m, spec.r)
    n, m, r = spec.n, spec.m, spec.r
    max_rounds = 4096
    out = pk.PeelOut(torch.empty(n, dtype=torch.int32, device=dev),
                     torch.empty(n, dtype=torch.int32, device=dev),
                     torch.empty(m, dtype=torch.int32, device=dev),
                     torch.empty(2 * max_rounds, dtype=torch.int64, device=dev),
                     torch.empty(8, dtype=torch.int32, device=dev))
    ws = pk.workspace(pk.peel_k2_xor_workspace(n, m, r), dev)
    t = Timer()
    for _ in range(warmup):
        pk.peel_k2_xor(e, n, max_rounds=max_rounds, out=out, ws=ws)
    torch.cuda.synchronize()
    for _ in range(steps):
        with t:
            pk.peel_k2_xor(e, n, max_rounds=max_rounds, out=out, ws=ws)
    t.collect()
    summ = out.summary.cpu().numpy().view(np.uint32)
    same = (np.array_equal(out.vertex_round.cpu().numpy().view(np.uint32), ref["vr"])
            and np.array_equal(out.edge_round.cpu().numpy().view(np.uint32), ref["er"])
            and int(summ[0]) == ref["rounds"])
    ms = float(np.median(t.ms))
    return {"workload": spec.name, "step": "peel_k2_xor (degree/XOR build + peel)",
            "step_ms": ms, "step_ms_p10_p90": [float(np.percentile(t.ms, 10)),
                                                float(np.percentile(t.ms, 90))],
            "edges_per_s": ref["m_removed"] / (ms * 1e-3), "rounds": int(summ[0]),
            "flags": int(summ[2]), "equal_to_build_peel": bool(same),
            "vs_build_peel_ms": ref["build_ms"] + ref["peel_ms"]}


def bench_iblt(spec, reps):
    keys_h = spec.keys(1)
    dev = torch.device("cuda", 0)
    keys = torch.from_numpy(keys_h.view(np.int64)).to(dev)
    pinned = torch.from_numpy(keys_h.view(np.int64)).pin_memory()
    d = pk.iblt_desc(spec.ncells, spec.r, spec.table_seed(1))
    cells = pk.iblt_table(spec.ncells, dev)
    lo = pk.ListOut(torch.empty(spec.ncells, dtype=torch.int64, device=dev),
                    torch.empty(4096, dtype=torch.int64, device=dev),
                    torch.empty(8, dtype=torch.int64, device=dev))
    ws = pk.workspace(pk.iblt_list_workspace(d), dev)
    wsu = pk.workspace(pk.iblt_update_workspace(d, spec.nkeys), dev)
    ti, tl, th, tsub, tu = Timer(), Timer(), Timer(), Timer(), Timer()
    for i in range(reps + 2):
        # the same insert by binning the keys per block of cells
        cells.zero_()
        with tu:
            pk.iblt_update(d, cells, keys, 1, ws=wsu)
        tu.collect()
        # the paper's process (listing with subtables) on a fresh table
        cells.zero_()
        pk.iblt_insert(d, cells, keys)
        with tsub:
            pk.iblt_list(d, cells, max_rounds=4096, out=lo, ws=ws, subtables=True)
        tsub.collect()
        sub_s = lo.summary.cpu().numpy()
        cells.zero_()
        with th:
            keys.copy_(pinned, non_blocking=True)
            pk.iblt_insert(d, cells, keys)
        th.collect()
        cells.zero_()
        with ti:
            pk.iblt_insert(d, cells, keys)
        ti.collect()
        with tl:
            pk.iblt_list(d, cells, max_rounds=4096, out=lo, ws=ws)
        tl.collect()
    s = lo.summary.cpu().numpy()
    sub_ms = float(np.median(tsub.ms[2:]))
    listed = int(s[0])
    ins = float(np.median(ti.ms[2:]))
    lst = float(np.median(tl.ms[2:]))
    h2d = float(np.median(th.ms[2:]))
    upd = float(np.median(tu.ms[2:]))
    return {
        "workload": spec.name, "cells": spec.ncells, "keys": spec.nkeys, "r": spec.r,
        "listed": listed, "recovered_frac": listed / spec.nkeys, "rounds": int(s[1]),
        "left": int(s[2]), "flags": int(s[3]),
        "insert_ms": ins, "list_ms": lst, "insert_incl_h2d_ms": h2d,
        "insert_binned_ms": upd, "insert_binned_keys_per_s": spec.nkeys / (upd * 1e-3),
        "insert_keys_per_s": spec.nkeys / (ins * 1e-3),
        "list_keys_per_s": listed / (lst * 1e-3),
        "insert_gbs": iblt_insert_bytes(spec.nkeys, spec.r) / (ins * 1e-3) / 1e9,
        "insert_binned_gbs": iblt_insert_bytes(spec.nkeys, spec.r) / (upd * 1e-3) / 1e9,
        "list_gbs": iblt_list_bytes(spec.ncells, spec.r, listed) / (lst * 1e-3) / 1e9,
        "list_frac_of_peak": iblt_list_bytes(spec.ncells, spec.r, listed) / (lst * 1e-3) / 1e9
                             / HBM_PEAK_GBS,
        "subtables": {"list_ms": sub_ms, "listed": int(sub_s[0]), "subrounds": int(sub_s[1]),
                      "list_keys_per_s": int(sub_s[0]) / (sub_ms * 1e-3)},
    }


def bench_signed(reps):
    """Set difference (Section 5): insert A, delete B, list the signed table.
    2^24 cells, r = 3, |A| = |B| = 8.05 M keys, |A xor B| = 7.05 M (load 0.42)."""
    N, r = 1 << 24, 3
    na = nb = int(0.48 * N)
    no = int(0.27 * N)
    pool = torch.from_numpy(gen.distinct_keys(na + nb - no, 901).view(np.int64)).cuda()
    a, b = pool[:na], pool[na - no:]
    d = pk.iblt_desc(N, r, gen.table_seed(901))
    cells = pk.iblt_table(N, "cuda")
    out = pk.SignedListOut(torch.empty(N, dtype=torch.int64, device="cuda"),
                           torch.empty(N, dtype=torch.int8, device="cuda"),
                           torch.empty(4096, dtype=torch.int64, device="cuda"),
                           torch.empty(8, dtype=torch.int64, device="cuda"))
    ws = pk.workspace(pk.iblt_list_workspace(d), "cuda")
    wsu = pk.workspace(max(pk.iblt_update_workspace(d, na), pk.iblt_update_workspace(d, nb)), "cuda")
    tu, tl, tb = Timer(), Timer(), Timer()
    for _ in range(reps + 2):
        cells.zero_()
        with tb:
            pk.iblt_update(d, cells, a, 1, ws=wsu)
            pk.iblt_update(d, cells, b, -1, ws=wsu)
        tb.collect()
        cells.zero_()
        with tu:
            pk.iblt_insert(d, cells, a)
            pk.iblt_delete(d, cells, b)
        with tl:
            pk.iblt_list_signed(d, cells, max_rounds=4096, out=out, ws=ws)
        tl.collect()
        tu.collect()
    s = out.summary.cpu().numpy()
    lst = float(np.median(tl.ms[2:]))
    upd = float(np.median(tu.ms[2:]))
    upd_b = float(np.median(tb.ms[2:]))
    return {"workload": "iblt_signed_r3_N16M_diff7M", "cells": N, "inserted": na, "deleted": nb,
            "difference": na + nb - 2 * no, "listed": int(s[0]), "rounds": int(s[1]),
            "cells_left": int(s[2]), "update_ms": upd, "update_binned_ms": upd_b, "list_ms": lst,
            "list_keys_per_s": int(s[0]) / (lst * 1e-3)}


def _tuner_summary(rep):
    """Per size class: tables, the chosen schedule, the fastest and slowest
    candidate; and the whole-batch trials of the thread counts."""
    out = {}
    for cls, c in rep["classes"].items():
        ms = [t["ms"] for t in c["trials"]]
        out[cls] = {"tables": c["tables"], "choice": c["choice"], "best_ms": min(ms),
                    "worst_ms": max(ms), "trials": c["trials"]}
    out["combined"] = rep["combined"]
    return out


def bench_batched(spec, reps, sched=None):
    """One launch for every table (schedule tuned per size class, or `sched`) vs
    one iblt_list per table."""
    draw = spec.draw(1)
    order = sorted(range(len(draw)), key=lambda i: -draw[i][0])
    dev = torch.device("cuda", 0)
    tables, pristine, nkeys = [], [], 0
    for i in order:
        N, m, kseed, tseed = draw[i]
        keys = torch.from_numpy(gen.distinct_keys(m, kseed).view(np.int64)).to(dev)
        d = pk.iblt_desc(N, spec.r, tseed)
        cells = pk.iblt_table(N, dev)
        pk.iblt_insert(d, cells, keys)
        tables.append(pk.batch_table(d, cells, 256))
        pristine.append(cells.clone())
        nkeys += m
    ent = pk.batch_entries(tables, dev)
    maxc = max(x[0] for x in draw)
    ws = pk.workspace(pk.iblt_list_batched_workspace(len(tables), maxc), dev)
    torch.cuda.synchronize()

    def reset():
        for t, p in zip(tables, pristine):
            t.cells.copy_(p)
        torch.cuda.synchronize()

    # pick the schedule on this batch, then capture the batched call in a graph
    tuner = None
    if sched is None:
        from paper_1302_7014_amd.autotune import tune_batched
        sched, tuner = tune_batched(tables, ent, maxc, 256, ws)
    log(f"batched schedule {sched}")
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pk.iblt_list_batched(ent, len(tables), maxc, 256, ws=ws, **sched)
    torch.cuda.current_stream().wait_stream(side)
    reset()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        pk.iblt_list_batched(ent, len(tables), maxc, 256, ws=ws, **sched)
    tb = Timer()
    for _ in range(reps):
        reset()
        with tb:
            graph.replay()
        tb.collect()
    listed = sum(int(t.summary[0].item()) for t in tables)
    incomplete = sum(int(t.summary[2].item()) > 0 for t in tables)
    # one plain launch per table, same stream, each table listed alone
    wsl = pk.workspace(max(pk.iblt_list_workspace(t.desc) for t in tables), dev)
    outs = [pk.ListOut(t.keys, t.round_stats, t.summary) for t in tables]
    tp = Timer()
    reset()
    with tp:
        for t, o in zip(tables, outs):
            pk.iblt_list(t.desc, t.cells, max_rounds=256, out=o, ws=wsl)
    tp.collect()
    listed_plain = sum(int(t.summary[0].item()) for t in tables)
    bt = float(np.median(tb.ms))
    pt = tp.ms[0]
    return {
        "workload": spec.name, "tables": len(tables), "cells": int(sum(x[0] for x in draw)),
        "keys": nkeys, "listed": listed, "incomplete_tables": incomplete,
        "schedule": sched, "tuner": _tuner_summary(tuner) if tuner else None,
        "batched_graph_ms": bt, "plain_per_table_ms": pt, "speedup": pt / bt,
        "batched_keys_per_s": listed / (bt * 1e-3), "plain_keys_per_s": listed_plain / (pt * 1e-3),
        # the listing's algorithmic bytes summed over the tables (each table's
        # 4N + listed (28 + 40r) adds up to the same form over the whole batch)
        "batched_gbs": iblt_list_bytes(int(sum(x[0] for x in draw)), spec.r, listed) / (bt * 1e-3) / 1e9,
        "listed_equal": listed == listed_plain,
    }


def bench_serve(spec, n_cal, n_rate, warm):
    """Served decoding: saturated rate, then p50/p99 at 0.3/0.6/0.9 of it, continuous
    batching vs the one-at-a-time FIFO server, same requests."""
    from paper_1302_7014_amd.serve import ContinuousServer, FifoServer, Request, latency_stats

    def fill(q, out):
        out.copy_(gen.distinct_keys_torch(q.nkeys, q.key_seed, out.device))

    def reqs(count, rate, seed):
        return [Request(i, *x) for i, x in enumerate(spec.requests(count, rate, seed))]

    def measured(done):
        return latency_stats([q for q in done if q.rid >= warm])

    # Each server first runs `warm` requests unmeasured: the first closed loop
    # pays one-time costs (first touch of the arena, first launches) that made
    # the saturated rate swing by a factor of two with what ran before it.
    cont = ContinuousServer(spec.budget_bytes, fill, max_cells=1 << 22, max_r=max(spec.r_choices))
    cont.run(reqs(warm, 0.0, 4))
    cal = latency_stats(cont.run(reqs(n_cal, 0.0, 5)))
    lam = cal["req_per_s"]
    fifo = FifoServer(spec.budget_bytes, fill, max_r=max(spec.r_choices))
    fifo.run(reqs(warm, 0.0, 4))
    fifo_sat = latency_stats(fifo.run(reqs(n_cal, 0.0, 5)))["req_per_s"]
    out = {"workload": spec.name, "budget_gb": spec.budget_bytes / 2 ** 30,
           "small_cells": cont.small_cells, "large_lanes": len(cont.large_streams),
           "saturated_req_per_s": lam,
           "fifo_saturated_req_per_s": fifo_sat, "warmup_requests": warm, "rates": []}
    for i, frac in enumerate((0.3, 0.6, 0.9)):
        rate = frac * lam
        log(f"serving at {rate:.0f} req/s")
        c = measured(cont.run(reqs(n_rate + warm, rate, 100 + i)))
        f = measured(fifo.run(reqs(n_rate + warm, rate, 100 + i)))
        out["rates"].append({"fraction": frac, "rate_req_per_s": rate, "continuous": c, "fifo": f})
    out["peak_budget_used_gb"] = cont.arena.peak / 2 ** 30
    out["batches"] = cont.batches
    out["large_lane_lists"] = cont.large
    return out


def copy_probe():
    """A plain device copy of 1 GiB, for calibrating the HBM byte counters."""
    dev = torch.device("cuda", 0)
    a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": a.numel() * 4, "copies": 3}))


def stream_copy_gbs(reps=5):
    """Bandwidth of a plain 1 GiB device-to-device copy (read + write bytes per
    second, median of `reps`): the practical HBM ceiling beside the 8 TB/s peak."""
    dev = torch.device("cuda", 0)
    a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    t = Timer()
    for _ in range(reps):
        with t:
            b.copy_(a)
    t.collect()
    ms = float(np.median(t.ms))
    del a, b
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def host_cpu():
    """The host's CPU model and the cores this process may use."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count(), "usable": len(os.sched_getaffinity(0))}


def traffic_from_profile(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or
    None when the kernel's source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    ent = doc.get(kernel)
    if not ent:
        return None
    # the kernel's own source and the headers it includes (barriers, scans)
    files = {ent["source"]: ent["source_sha256"], **ent.get("deps", {})}
    for rel, want in files.items():
        src = os.path.join(ROOT, rel)
        if not os.path.exists(src):
            return None
        if hashlib.sha256(open(src, "rb").read()).hexdigest() != want:
            return None
    return ent["bytes_per_launch"]


def cpu_baseline(spec, e_host):
    """The oracle's round-synchronous peel on the same workload, single-threaded."""
    from oracle import native  # CPU-baseline leg only
    t0 = time.perf_counter()
    o = native.peel_rounds(spec.n, e_host, spec.k)
    dt = time.perf_counter() - t0
    m_rem = int((o.edge_round != 0).sum())
    # the oracle's sequential queue peel (the serial process of Section 1), beside it
    t0 = time.perf_counter()
    _, core_e = native.peel_queue(spec.n, e_host, spec.k)
    dq = time.perf_counter() - t0
    mq = int(spec.m - core_e.sum())
    return {"value": m_rem / dt, "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"one full run of oracle peel_rounds (its own CSR build included) on "
                      f"{spec.name} ({spec.m} edges), {dt:.2f} s", "host": host_cpu(),
            "serial_queue": {"value": mq / dq, "unit": "edges/s", "cores": 1,
                             "sample": f"one full run of oracle peel_queue on the same "
                                       f"workload, {dq:.2f} s"},
            "all_cores": cpu_all_cores(spec, e_host)}


def cpu_all_cores(spec, e_host, cap=16):
    """The same single-threaded oracle run on every usable host core at once: one
    independent peel_rounds of the workload per thread (the C oracle releases the
    interpreter lock), so the aggregate is the host's throughput for this
    workload with the oracle as it stands."""
    import concurrent.futures as cf
    from oracle import native  # CPU-baseline leg only
    p = max(1, min(cap, len(os.sched_getaffinity(0))))

    def one(_):
        o = native.peel_rounds(spec.n, e_host, spec.k)
        return int((o.edge_round != 0).sum())

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=p) as ex:
        done = sum(ex.map(one, range(p)))
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "edges/s", "cores": p, "kind": "oracle",
            "sample": f"{p} concurrent oracle peel_rounds runs of {spec.name}, one per thread, "
                      f"{dt:.2f} s wall"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-iblt", action="store_true")
    ap.add_argument("--no-sweep", action="store_true",
                    help="skip the other c of the n=2^24 sweep and the near-threshold points")
    ap.add_argument("--no-subtables", action="store_true",
                    help="skip the subtables peel and the k = 3 peels (profiles of the main "
                         "workload alone)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-xor", action="store_true", help="skip the CSR-free k = 2 peel")
    ap.add_argument("--batched-main-only", action="store_true",
                    help="of the batched workloads, only the 4096-table batch")
    ap.add_argument("--no-tune", action="store_true",
                    help="batched listing with the schedule the tuner picks for the 4096-table "
                         "batch (1024 threads, LDS tables up to 5120 cells), no tuning runs "
                         "(profiles of one schedule)")
    ap.add_argument("--iblt-main", action="store_true",
                    help="of the IBLT workloads, only the 2^24-cell main one (profiles of one shape)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--serve-requests", type=int, default=5000, help="measured requests per rate")
    ap.add_argument("--copy-probe", action="store_true", help="only run a 1 GiB device copy")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the peel and the IBLT listing run on a single MI355X "
              "(multi-GPU sharding is a design note, not built); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe()
        return
    pk.lib()

    spec = configs.kcore_sweep(0.70)
    kc = bench_kcore(spec, args.steps, args.warmup)
    ms_step = kc["wall_s"] / args.steps * 1e3
    value = kc["m_removed"] / (kc["wall_s"] / args.steps)
    # dominant kernel: the longer of the two calls
    if kc["peel_ms"] >= kc["build_ms"]:
        dom, dom_ms, dom_bytes = "k_peel_owner", kc["peel_ms"], kc["peel_bytes"]
    else:
        dom, dom_ms, dom_bytes = "hg_build", kc["build_ms"], kc["build_bytes"]
    achieved = dom_bytes / (dom_ms * 1e-3) / 1e9
    extra = {
        "peel_ms": kc["peel_ms"], "build_ms": kc["build_ms"],
        "peel_edges_per_s": kc["m_removed"] / (kc["peel_ms"] * 1e-3),
        "peel_algorithmic_bytes": kc["peel_bytes"], "build_algorithmic_bytes": kc["build_bytes"],
        "peel_gbs": kc["peel_bytes"] / (kc["peel_ms"] * 1e-3) / 1e9,
        "build_gbs": kc["build_bytes"] / (kc["build_ms"] * 1e-3) / 1e9,
        "rounds": kc["rounds"], "edge_rounds": kc["edge_rounds"],
        "core_vertices": kc["core_vertices"],
        "peel_ms_p10_p90": kc["peel_ms_p10_p90"], "build_ms_p10_p90": kc["build_ms_p10_p90"],
    }
    # the peel's algorithmic rate against what a plain device copy reaches
    copy_gbs = stream_copy_gbs()
    extra["stream_copy_gbs"] = copy_gbs
    extra["peel_frac_of_copy"] = extra["peel_gbs"] / copy_gbs
    extra["build_frac_of_copy"] = extra["build_gbs"] / copy_gbs
    if not args.no_xor:
        log("CSR-free k = 2 peel")
        extra["csr_free_k2"] = bench_k2_xor(spec, args.steps, args.warmup, kc)
    if not args.no_subtables:
        # the paper's own schedule (peeling with subtables) on the same workload
        sb = bench_kcore(spec, max(3, args.steps // 2), 1, subtables=True)
        extra["subtables"] = {
            "peel_ms": sb["peel_ms"], "subrounds": sb["rounds"], "edge_subrounds": sb["edge_rounds"],
            "peel_edges_per_s": sb["m_removed"] / (sb["peel_ms"] * 1e-3),
            "vs_rounds_peel_ms": kc["peel_ms"]}
    if not args.no_subtables:
        # k = 3 on r = 3, n = 2^22, below and above its threshold
        k3 = []
        for which in ("lo", "hi"):
            s3 = configs.kcore_k3(which)
            r3 = bench_kcore(s3, max(3, args.steps // 4), 1)
            k3.append({"workload": s3.name, "m": s3.m, "rounds": r3["rounds"],
                       "m_removed": r3["m_removed"], "core_vertices": r3["core_vertices"],
                       "peel_ms": r3["peel_ms"], "build_ms": r3["build_ms"],
                       "peel_edges_per_s": r3["m_removed"] / (r3["peel_ms"] * 1e-3),
                       "peel_gbs": r3["peel_bytes"] / (r3["peel_ms"] * 1e-3) / 1e9})
        extra["k3"] = k3
    if not args.no_batched:
        log("batched IBLT listing (4096 tables)")
        fixed = ({"block_threads": 1024, "lds_max_cells": pk.IBLT_LDS_MAX_CELLS,
                  "tile_min_cells": 0, "tile_workgroups": 0} if args.no_tune else None)
        extra["batched"] = bench_batched(configs.batched_main(), 3, fixed)
        if not args.batched_main_only:
            log("batched IBLT listing, 5% of the tables above threshold")
            extra["batched_partial"] = bench_batched(configs.batched_partial(), 3, fixed)
            log("batched IBLT listing, 16 tables of 2^20 cells")
            extra["batched_few_large"] = bench_batched(
                configs.batched_few_large(), 3,
                {**fixed, "lds_max_cells": 0, "tile_min_cells": 1 << 17, "tile_workgroups": 16}
                if fixed else None)
    if not args.no_iblt:
        log("IBLT 2^24 cells")
        extra["iblt"] = [bench_iblt(configs.iblt_main(), 5)]
        if not args.iblt_main:
            # the shapes of the paper's Tables 5 and 6: r = 3, 4 at loads 0.75, 0.83
            for r_, load in ((3, 0.75), (3, 0.83), (4, 0.75), (4, 0.83)):
                extra["iblt"].append(bench_iblt(configs.iblt_paper(r_, load), 5))
            extra["iblt_signed"] = bench_signed(5)
    torch.cuda.empty_cache()
    if not args.no_serve:
        log("served decoding")
        extra["serve"] = bench_serve(configs.served_main(), 1000, args.serve_requests, 500)
    if not args.no_sweep:
        log("peel sweep over c at n = 2^24")
        sw = []
        for c in configs.SWEEP_C + configs.NEAR_C:
            s2 = configs.kcore_sweep(c)
            r2 = bench_kcore(s2, max(3, args.steps // 4), 1)
            gbs = r2["peel_bytes"] / (r2["peel_ms"] * 1e-3) / 1e9
            sw.append({"workload": s2.name, "c": c, "m": s2.m, "rounds": r2["rounds"],
                       "m_removed": r2["m_removed"], "core_vertices": r2["core_vertices"],
                       "peel_ms": r2["peel_ms"], "build_ms": r2["build_ms"],
                       "peel_edges_per_s": r2["m_removed"] / (r2["peel_ms"] * 1e-3),
                       "peel_gbs": gbs, "peel_frac_of_peak": gbs / HBM_PEAK_GBS})
        extra["sweep"] = sw
    line = {
        "metric": METRIC, "value": value, "unit": "edges/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": spec.name, "n": spec.n, "m": spec.m, "r": spec.r, "k": spec.k,
                   "model": spec.model, "seed": 1, "step": "hg_build + peel_kcore"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic_from_profile(dom)},
        "extra": extra,
    }
    if not args.no_cpu:
        log("oracle CPU baseline")
        line["cpu_baseline"] = cpu_baseline(spec, kc["edges_host"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
