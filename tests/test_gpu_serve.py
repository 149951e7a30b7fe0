"""GPU check of the continuous-batching server: every request's result in the
mix equals its result served alone and the oracle's, and the HBM budget holds."""
import numpy as np
import pytest
import torch

from oracle import native
from paper_1302_7014_amd.serve import ContinuousServer, FifoServer, Request, latency_stats
from workloads import configs, gen

from gpu_helpers import need_gpu, say

pytestmark = pytest.mark.gpu


def _fill(q, out):
    out.copy_(gen.distinct_keys_torch(q.nkeys, q.key_seed, out.device))


def _requests(count, rate, seed, lo=6, hi=14):
    spec = configs.ServeSpec("test", log2_lo=lo, log2_hi=hi, load_lo=0.3, load_hi=1.1)
    return [Request(i, *x) for i, x in enumerate(spec.requests(count, rate, seed))]


def _groups(q):
    out, off = [], 0
    for kk in q.round_stats.tolist():
        out.append(np.sort(q.keys_out[off: off + kk]))
        off += kk
    return out


@pytest.mark.parametrize("binned_min", [None, 1 << 10])
def test_mix_equals_alone_and_oracle(binned_min):
    # binned_min: tables from this size on are filled with the binned update
    # (None: the server's default, which no table of this mix reaches)
    need_gpu()
    budget = 6 << 20  # small: arrivals must wait for space
    mix = _requests(80, 4000.0, 11)
    say("serve mix", len(mix), binned_min)
    srv = ContinuousServer(budget, _fill, max_cells=1 << 14, keep_keys=True)
    fifo = FifoServer(budget, _fill, keep_keys=True, max_cells=1 << 14)
    if binned_min is not None:
        srv.binned_min_cells = fifo.binned_min_cells = binned_min
    done = srv.run(mix)
    assert len(done) == len(mix) and not srv.rejected
    assert srv.arena.peak <= budget and srv.batches >= 2 and srv.large >= 1
    if binned_min is not None:
        assert sum(q.ncells >= binned_min for q in mix) >= 20
    alone = fifo.run(_requests(80, 0.0, 11))
    by_id = {q.rid: q for q in alone}
    for q in done:
        a = by_id[q.rid]
        assert np.array_equal(q.summary[:4], a.summary[:4])
        ga, gm = _groups(a), _groups(q)
        assert len(ga) == len(gm) and all(np.array_equal(x, y) for x, y in zip(ga, gm))
        k = gen.distinct_keys(q.nkeys, q.key_seed)
        o = native.iblt_list_rounds(native.iblt_insert(q.ncells, q.r, q.table_seed, k), max_rounds=256)
        assert int(q.summary[0]) == o.keys.size and int(q.summary[1]) == o.rounds
        assert all(np.array_equal(x, y) for x, y in zip(gm, o.per_round()))
    st = latency_stats(done)
    assert st["p99_ms"] >= st["p50_ms"] > 0


def test_request_over_budget_is_rejected():
    need_gpu()
    reqs = _requests(5, 0.0, 3)
    big = Request(99, 0.0, 3, 1 << 20, 1000, 1, 2)
    srv = ContinuousServer(4 << 20, _fill, max_cells=1 << 20)
    done = srv.run(reqs + [big])
    assert [q.rid for q in srv.rejected] == [99] and len(done) == 5


@pytest.mark.timeout(600)
def test_mix_with_large_tables_equals_alone_and_oracle():
    # Tables of 2^12 .. 2^22 cells (a third of them 2^18 and more, the binned
    # fill and the large lanes): each result in the mix equals the request
    # served alone and the oracle's listing, round by round.
    need_gpu()
    mix = _requests(36, 2000.0, 29, lo=12, hi=22)
    big = sum(q.ncells >= 1 << 18 for q in mix)
    assert big >= 10
    budget = 768 << 20  # the three largest tables at once at most
    say("serve mix, large tables", len(mix), big)
    srv = ContinuousServer(budget, _fill, max_cells=1 << 22, keep_keys=True)
    done = srv.run(mix)
    assert len(done) == len(mix) and not srv.rejected
    assert srv.arena.peak <= budget and srv.large >= big
    fifo = FifoServer(budget, _fill, keep_keys=True, max_cells=1 << 22)
    alone = {q.rid: q for q in fifo.run(_requests(36, 0.0, 29, lo=12, hi=22))}
    for q in sorted(done, key=lambda q: q.rid):
        a = alone[q.rid]
        assert np.array_equal(q.summary[:4], a.summary[:4])
        ga, gm = _groups(a), _groups(q)
        assert len(ga) == len(gm) and all(np.array_equal(x, y) for x, y in zip(ga, gm))
        k = gen.distinct_keys(q.nkeys, q.key_seed)
        o = native.iblt_list_rounds(native.iblt_insert(q.ncells, q.r, q.table_seed, k),
                                    max_rounds=256)
        assert int(q.summary[0]) == o.keys.size and int(q.summary[1]) == o.rounds
        assert all(np.array_equal(x, y) for x, y in zip(gm, o.per_round()))
    say("serve mix, large tables: all equal")


@pytest.mark.parametrize("r", [3, 4, 8])
def test_largest_table_of_every_r_is_served(r):
    # a table of max_cells cells with the largest r the server is sized for
    # goes through a large lane (whose listing workspace grows with r)
    need_gpu()
    n = 1 << 20
    from oracle import theory
    m = int(0.6 * theory.cstar(2, r)[0] * n)
    q = Request(0, 0.0, r, n, m, 7000 + r, gen.table_seed(7000 + r))
    say("serve largest table, r", r)
    srv = ContinuousServer(256 << 20, _fill, max_cells=n, keep_keys=True, max_r=8)
    done = srv.run([q])
    assert len(done) == 1 and srv.large == 1
    k = gen.distinct_keys(m, q.key_seed)
    o = native.iblt_list_rounds(native.iblt_insert(n, r, q.table_seed, k), max_rounds=256)
    assert int(done[0].summary[0]) == o.keys.size and int(done[0].summary[1]) == o.rounds
    assert all(np.array_equal(x, y) for x, y in zip(_groups(done[0]), o.per_round()))
