"""GPU parity of iblt_list on tables of 2^20 cells and more, whose first round
removes its keys through the binned update before the persistent kernel runs
the later rounds: keys per round, round counts, summary and the table left,
bit for bit against the oracle, including the cases that keep the old path
(a round limit of 1, a small out_cap, a share of the CUs)."""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native, theory
from workloads import gen

from gpu_helpers import dev_u64, host_u64, need_gpu, say, table_to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def atomic_engine(monkeypatch):
    """The binned first round belongs to the device-atomic listing engine."""
    monkeypatch.setenv("PEEL_LIST_ENGINE", "atomic")

N = (1 << 20) + 77


def _check(ncells, r, seed, keys, out_cap=None, max_rounds=4096, workgroups=0, corrupt=False):
    d = pk.iblt_desc(ncells, r, seed, workgroups)
    cells = pk.iblt_table(ncells, "cuda")
    if keys.size:
        pk.iblt_insert(d, cells, dev_u64(keys))
    t = native.iblt_insert(ncells, r, seed, keys)
    if corrupt:
        c = int(np.flatnonzero(t.count == 1)[0])
        t.hash_sum[c] ^= np.uint64(1)
        cells[c, 2] ^= 1
    out = pk.iblt_list(d, cells, out_cap=out_cap, max_rounds=max_rounds)
    torch.cuda.synchronize()
    s = out.summary.cpu().numpy()
    o = native.iblt_list_rounds(t, max_rounds=max_rounds, out_cap=ncells if out_cap is None else out_cap)
    listed, rounds = int(s[0]), int(s[1])
    assert rounds == o.rounds and listed == o.keys.size
    K = host_u64(out.round_stats)[:rounds]
    assert np.array_equal(K, o.K)
    assert not host_u64(out.round_stats)[rounds:max_rounds].any()
    ks = host_u64(out.keys)[:listed]
    off = 0
    for kk, want in zip(K.tolist(), o.per_round()):
        assert np.array_equal(np.sort(ks[off: off + kk]), want)
        off += kk
    count, ksum, hsum, ok = table_to_numpy(cells)
    assert ok and np.array_equal(count, t.count)
    assert np.array_equal(ksum, t.key_sum) and np.array_equal(hsum, t.hash_sum)
    flags = int(s[3])
    assert bool(flags & 0x8) == o.corrupt
    assert bool(flags & 0x2) == (o.status == native.EROUNDS)
    assert bool(flags & 0x4) == (o.status == native.ENOSPC)
    if not corrupt:
        assert int(s[2]) == keys.size - listed
    return s, o


@pytest.mark.parametrize("r", [2, 3, 4, 8])
@pytest.mark.parametrize("frac", [0.5, 0.95, 1.2])
def test_large_tables_below_and_above_threshold(r, frac):
    need_gpu()
    cs = theory.cstar(2, r)[0] if r > 2 else 0.5
    keys = gen.distinct_keys(int(frac * cs * N), 4000 + r)
    say("first round binned", N, r, frac)
    _check(N, r, gen.table_seed(40 + r), keys)


def test_large_table_limits_corrupt_and_old_paths():
    need_gpu()
    keys = gen.distinct_keys(int(0.75 * N), 91)
    for mr in (1, 2, 3):  # 1 keeps the old path; 2 and 3 stop after the binned round 1
        say("first round binned, max_rounds", mr)
        _check(N, 3, 7, keys, max_rounds=mr)
    say("first round binned, small out_cap (old path)")
    _check(N, 3, 7, keys, out_cap=5000)
    say("first round binned, CU share (old path)")
    _check(N, 3, 7, keys, workgroups=64)
    say("first round binned, corrupt cell")
    _check(N, 3, 5, gen.distinct_keys(300000, 40), corrupt=True)
    say("first round binned, empty table")
    _check(N, 3, 5, np.zeros(0, np.uint64))


@pytest.mark.parametrize("ncells,r,frac,workgroups", [
    ((1 << 18) + 5, 3, 0.8, 0),    # round 1 in the persistent kernel
    ((1 << 18) + 5, 4, 1.2, 0),    # above threshold: a core is left
    ((1 << 16) + 3, 3, 0.8, 7),    # a share of the CUs
    (N, 3, 0.8, 0),                # binned first round, then the queues
])
def test_overflow_queues(monkeypatch, ncells, r, frac, workgroups):
    # staging slots of 64 per workgroup: nearly every key and candidate goes
    # through the shared overflow queues
    need_gpu()
    monkeypatch.setenv("PEEL_LIST_SLOT_CAP", "64")
    m = int(frac * theory.cstar(2, r)[0] * ncells)
    keys = gen.distinct_keys(m, 910 + r)
    say("overflow queues", ncells, r, m, workgroups)
    _check(ncells, r, gen.table_seed(910 + r), keys, workgroups=workgroups)
