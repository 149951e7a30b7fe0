"""The persistent kernels' bounded barrier wait, made to give up from the host.

PEEL_BARRIER_TIMEOUT_MS=0 (read at every call) makes each device-wide barrier
give up at its first poll that finds it still closed.  Each workgroup then
leaves its kernel at its next barrier, so every kernel ends normally; the call
reports PEEL_FLAG_TIMEOUT in its summary.  The next call, with the default
limit, must again agree with the oracle bit for bit.
"""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native
from workloads import gen

from gpu_helpers import gpu_peel, need_gpu, say
from test_gpu_iblt import check_list, gpu_insert, gpu_list

pytestmark = pytest.mark.gpu

TIMEOUT = pk.FLAG_TIMEOUT


@pytest.mark.parametrize("engine,subtables", [("owner", False), ("owner", True),
                                              ("global", False)])
def test_peel_gives_up_then_next_call_exact(engine, subtables, monkeypatch):
    need_gpu()
    if engine == "global":
        monkeypatch.setenv("PEEL_ENGINE", "global")
    n = (1 << 18) + 77
    e = gen.partitioned_edges(n, int(0.7 * n), 4, 41)
    monkeypatch.setenv("PEEL_BARRIER_TIMEOUT_MS", "0")
    say("give up: peel", engine, subtables)
    res = gpu_peel(n, e, 2, subtables=subtables)
    assert res["flags"] & TIMEOUT
    monkeypatch.delenv("PEEL_BARRIER_TIMEOUT_MS")
    say("after give up: peel", engine, subtables)
    res = gpu_peel(n, e, 2, subtables=subtables)
    o = (native.peel_subrounds if subtables else native.peel_rounds)(n, e, 2)
    assert res["flags"] == 0 and res["rounds"] == o.rounds
    assert np.array_equal(res["vertex_round"], o.vertex_round)
    assert np.array_equal(res["edge_round"], o.edge_round)
    assert np.array_equal(res["deg"], o.deg)


@pytest.mark.parametrize("engine", ["owner", "atomic"])
@pytest.mark.parametrize("ncells", [1 << 14, (1 << 20) + 77])
def test_list_gives_up_then_next_call_exact(ncells, engine, monkeypatch):
    # with the atomic engine, 2^20 + 77 cells also takes the binned first round
    # before the persistent kernel
    need_gpu()
    if engine == "atomic":
        monkeypatch.setenv("PEEL_LIST_ENGINE", "atomic")
    r, seed = 3, 43
    keys = gen.distinct_keys(int(0.7 * ncells), seed)
    d, cells = gpu_insert(ncells, r, seed, keys)
    monkeypatch.setenv("PEEL_BARRIER_TIMEOUT_MS", "0")
    say("give up: list", ncells)
    g = gpu_list(d, cells)
    assert g["flags"] & TIMEOUT
    for fn in (lambda d_, c_: pk.iblt_list(d_, c_, subtables=True), pk.iblt_list_signed):
        d2, cells2 = gpu_insert(ncells, r, seed, keys)
        out = fn(d2, cells2)
        torch.cuda.synchronize()
        assert int(out.summary.cpu().numpy()[3]) & TIMEOUT
    monkeypatch.delenv("PEEL_BARRIER_TIMEOUT_MS")
    say("after give up: list", ncells)
    check_list(ncells, r, seed, keys)


def test_batched_team_gives_up_then_next_call_exact(monkeypatch):
    # a team's barrier gives up: its tables report PEEL_FLAG_TIMEOUT, every
    # workgroup leaves, and the next call lists the same tables exactly
    need_gpu()
    from test_gpu_batched import _check_against_oracle, _make_tables
    N = 1 << 16
    specs = [(N, 3, int(0.7 * 0.818 * N), 80 + i) for i in range(6)]
    tables, keys, pristine = _make_tables(specs, 64)
    ent = pk.batch_entries(tables, "cuda")
    monkeypatch.setenv("PEEL_BARRIER_TIMEOUT_MS", "0")
    say("give up: batched teams")
    pk.iblt_list_batched(ent, len(tables), N, 64, tile_min_cells=N, tile_workgroups=16)
    torch.cuda.synchronize()
    assert any(int(t.summary[3].item()) & TIMEOUT for t in tables)
    monkeypatch.delenv("PEEL_BARRIER_TIMEOUT_MS")
    for t, p in zip(tables, pristine):
        t.cells.copy_(p)
    torch.cuda.synchronize()
    say("after give up: batched teams")
    pk.iblt_list_batched(ent, len(tables), N, 64, tile_min_cells=N, tile_workgroups=16)
    torch.cuda.synchronize()
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 64)
        assert int(t.summary[3].item()) == 0
