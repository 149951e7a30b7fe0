"""GPU parity of iblt_delete and iblt_list_signed (tables holding deletions,
Section 5) against the oracle, bit for bit: the table after inserts and
deletes, the keys and signs of every round, the summary and the table left."""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native, theory
from workloads import gen

from gpu_helpers import dev_u64, host_u64, need_gpu, say, table_to_numpy

pytestmark = pytest.mark.gpu


def _sets(N, frac_a, frac_b, overlap, seed):
    na, nb, no = int(frac_a * N), int(frac_b * N), int(overlap * N)
    pool = gen.distinct_keys(na + nb - no, seed)
    return pool[:na], pool[na - no:]


def _run(N, r, a, b, seed, out_cap=None, max_rounds=4096, workgroups=0):
    d = pk.iblt_desc(N, r, seed, workgroups)
    cells = pk.iblt_table(N, "cuda")
    if a.size:
        pk.iblt_insert(d, cells, dev_u64(a))
    if b.size:
        pk.iblt_delete(d, cells, dev_u64(b))
    t = native.iblt_insert(N, r, seed, a)
    native.iblt_update(t, b, sign=-1)
    count, ks, hs, ok = table_to_numpy(cells)
    assert ok and np.array_equal(count, t.count)
    assert np.array_equal(ks, t.key_sum) and np.array_equal(hs, t.hash_sum)
    out = pk.iblt_list_signed(d, cells, out_cap=out_cap, max_rounds=max_rounds)
    torch.cuda.synchronize()
    s = out.summary.cpu().numpy()
    o = native.iblt_list_signed(t, max_rounds=max_rounds, out_cap=N if out_cap is None else out_cap)
    listed, rounds = int(s[0]), int(s[1])
    assert listed == o.keys.size and rounds == o.rounds
    K = host_u64(out.round_stats)[:rounds]
    assert np.array_equal(K, o.K)
    keys = host_u64(out.keys)[:listed]
    signs = out.signs.cpu().numpy()[:listed]
    off = 0
    for kk, (want_k, want_s) in zip(K.tolist(), o.per_round()):
        order = np.argsort(keys[off: off + kk])
        assert np.array_equal(keys[off: off + kk][order], want_k)
        assert np.array_equal(signs[off: off + kk][order], want_s)
        off += kk
    count, ks, hs, ok = table_to_numpy(cells)  # claims given back: reserved fields are 0
    assert ok and np.array_equal(count, t.count)
    assert np.array_equal(ks, t.key_sum) and np.array_equal(hs, t.hash_sum)
    assert int(s[2]) == o.nonempty
    flags = int(s[3])
    assert flags & 0x8 == 0
    assert bool(flags & 0x2) == (o.status == native.EROUNDS)
    assert bool(flags & 0x4) == (o.status == native.ENOSPC)
    return s, o


@pytest.mark.parametrize("r", [2, 3, 4, 5])
@pytest.mark.parametrize("load", [0.5, 0.95, 1.3])
def test_signed_listing_matches_oracle(r, load):
    # the difference A xor B at `load` x threshold; A and B overlap
    need_gpu()
    N = (1 << 16) + 33
    cs = theory.cstar(2, r)[0] if r > 2 else 0.5
    d = load * cs
    a, b = _sets(N, 0.6 * d + 0.2, 0.4 * d + 0.2, 0.4, 500 + r)
    say("signed", r, load, a.size, b.size)
    s, o = _run(N, r, a, b, gen.table_seed(500 + r))
    if load < 1:
        assert o.status == native.OK and int(s[2]) == 0
        ks = o.keys
        assert np.array_equal(np.sort(ks[o.signs == 1]), np.sort(np.setdiff1d(a, b)))
        assert np.array_equal(np.sort(ks[o.signs == -1]), np.sort(np.setdiff1d(b, a)))


def test_signed_listing_limits_shares_and_degenerate():
    need_gpu()
    N = 1 << 14
    a, b = _sets(N, 0.55, 0.45, 0.3, 77)
    for mr in (1, 3):
        say("signed max_rounds", mr)
        _run(N, 3, a, b, 9, max_rounds=mr)
    for cap in (0, 25):
        say("signed out_cap", cap)
        _run(N, 3, a, b, 9, out_cap=cap)
    say("signed shares")
    _run(N, 4, a, b, 11, workgroups=5)
    say("signed only deletions; nothing; identical sets")
    _run(N, 3, np.zeros(0, np.uint64), b[:3000], 13)
    _run(N, 3, np.zeros(0, np.uint64), np.zeros(0, np.uint64), 13)
    _run(N, 3, a, a.copy(), 13)


def test_signed_full_size_difference():
    # 2^24 cells, r = 3: two sets of 8 M keys that differ in 7 M keys
    need_gpu()
    N = 1 << 24
    a, b = _sets(N, 0.48, 0.48, 0.27, 901)
    say("signed full size", a.size, b.size)
    s, o = _run(N, 3, a, b, gen.table_seed(901))
    assert o.status == native.OK and int(s[2]) == 0


@pytest.mark.parametrize("load", [0.5, 1.3])
def test_signed_overflow_queues(monkeypatch, load):
    # staging slots of 64 per workgroup: the overflow queues carry nearly all
    # keys and candidates, and a cell queued twice in a round is listed once
    need_gpu()
    monkeypatch.setenv("PEEL_LIST_SLOT_CAP", "64")
    N, r = (1 << 16) + 33, 3
    d = load * theory.cstar(2, r)[0]
    a, b = _sets(N, 0.6 * d + 0.2, 0.4 * d + 0.2, 0.4, 930)
    say("signed overflow queues", load, a.size, b.size)
    s, o = _run(N, r, a, b, gen.table_seed(930))
    if load < 1:
        assert o.status == native.OK and int(s[2]) == 0
