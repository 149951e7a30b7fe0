"""GPU parity of iblt_list_subtables (listing with subtables, the paper's GPU
process) against the oracle, bit for bit: keys per subround, subround totals,
the summary and the table left behind."""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native, theory
from workloads import configs, gen

from gpu_helpers import dev_u64, host_u64, need_gpu, say, table_to_numpy

pytestmark = pytest.mark.gpu


def _run(ncells, r, seed, keys, out_cap=None, max_rounds=4096, workgroups=0, corrupt=False):
    d = pk.iblt_desc(ncells, r, seed, workgroups)
    cells = pk.iblt_table(ncells, "cuda")
    if keys.size:
        pk.iblt_insert(d, cells, dev_u64(keys))
    t = native.iblt_insert(ncells, r, seed, keys)
    if corrupt:
        c = int(np.flatnonzero(t.count == 1)[0])
        t.hash_sum[c] ^= np.uint64(1)
        cells[c, 2] ^= 1
    out = pk.iblt_list(d, cells, out_cap=out_cap, max_rounds=max_rounds, subtables=True)
    torch.cuda.synchronize()
    s = out.summary.cpu().numpy()
    o = native.iblt_list_subrounds(t, max_rounds=max_rounds,
                                   out_cap=ncells if out_cap is None else out_cap)
    listed, rounds = int(s[0]), int(s[1])
    assert rounds == o.rounds and listed == o.keys.size
    K = host_u64(out.round_stats)[:rounds]
    assert np.array_equal(K, o.K)
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
        assert int(s[2]) == keys.size - listed  # keys left in the table
    return s, o


@pytest.mark.parametrize("r", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("frac", [0.5, 0.95, 1.2])
def test_subtables_below_and_above_threshold(r, frac):
    need_gpu()
    ncells = (1 << 17) + 77
    cs = theory.cstar(2, r)[0] if r > 2 else 0.5
    keys = gen.distinct_keys(int(frac * cs * ncells), 3000 + r)
    say("list subtables", ncells, r, frac)
    _run(ncells, r, gen.table_seed(r), keys)


def test_subtables_small_ragged_and_shares():
    need_gpu()
    for ncells, r, nkeys, wg in [(3, 3, 1, 0), (10, 2, 4, 0), (1000, 3, 700, 3), (4097, 4, 3000, 1),
                                 (12345, 8, 5000, 0), ((1 << 16) + 5, 5, 40000, 7)]:
        say("list subtables small", ncells, r, nkeys, wg)
        _run(ncells, r, 11 + r, gen.distinct_keys(nkeys, ncells), workgroups=wg)
    say("list subtables empty")
    _run(4096, 3, 5, np.zeros(0, np.uint64))


def test_subtables_limits_and_corrupt_cell():
    need_gpu()
    keys = gen.distinct_keys(int(0.75 * (1 << 15)), 91)
    for mr in (1, 2, 4, 9):  # limits inside and after round 1
        say("list subtables max_rounds", mr)
        _run(1 << 15, 3, 7, keys, max_rounds=mr)
    for cap in (0, 10, 5000):
        say("list subtables out_cap", cap)
        _run(1 << 15, 3, 7, keys, out_cap=cap)
    say("list subtables corrupt")
    _run(1 << 12, 3, 5, gen.distinct_keys(1000, 40), corrupt=True)


@pytest.mark.parametrize("which", ["config", "paper"])
def test_subtables_full_size(which):
    need_gpu()
    spec = configs.iblt_main() if which == "config" else configs.iblt_paper(3, 0.75)
    keys = spec.keys()
    say(spec.name, "subtables")
    s, o = _run(spec.ncells, spec.r, spec.table_seed(), keys)
    assert o.status == native.OK and int(s[2]) == 0
