"""GPU parity of iblt_insert + iblt_list against the CPU oracle.

Insert: the whole cell table, bit for bit.  List: the set of keys of every
round (order inside a round is free, so each round is compared sorted), the
per-round counts, the round count, the summary and the final table, bit for bit.
"""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native, theory
from workloads import configs, gen

from gpu_helpers import dev_u64, host_u64, need_gpu, say, table_to_numpy

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True, params=["owner", "atomic"])
def list_engine(request, monkeypatch):
    """Every listing test runs on both engines: the owner engine (the default:
    each workgroup owns a range of cells and applies their updates with plain
    read-modify-writes) and the persistent kernel with device-atomic deletes."""
    if request.param == "atomic":
        monkeypatch.setenv("PEEL_LIST_ENGINE", "atomic")
    else:
        monkeypatch.delenv("PEEL_LIST_ENGINE", raising=False)
    return request.param


def gpu_insert(ncells, r, seed, keys):
    d = pk.iblt_desc(ncells, r, seed)
    cells = pk.iblt_table(ncells, "cuda")
    pk.iblt_insert(d, cells, dev_u64(keys))
    return d, cells


def gpu_list(d, cells, out_cap=None, max_rounds=4096):
    out = pk.iblt_list(d, cells, out_cap=out_cap, max_rounds=max_rounds)
    torch.cuda.synchronize()
    summ = out.summary.cpu().numpy()
    listed, rounds = int(summ[0]), int(summ[1])
    K = host_u64(out.round_stats)[:rounds]
    keys = host_u64(out.keys)[:listed]
    groups, off = [], 0
    for kk in K.tolist():
        groups.append(np.sort(keys[off: off + kk]))
        off += kk
    return {"listed": listed, "rounds": rounds, "left": int(summ[2]),
            "flags": int(summ[3]), "K": K, "groups": groups, "stats": host_u64(out.round_stats)}


def check_table(cells, t):
    count, ks, hs, ok = table_to_numpy(cells)
    assert ok
    assert np.array_equal(count, t.count)
    assert np.array_equal(ks, t.key_sum)
    assert np.array_equal(hs, t.hash_sum)


def check_list(ncells, r, seed, keys, out_cap=None, max_rounds=4096):
    d, cells = gpu_insert(ncells, r, seed, keys)
    t = native.iblt_insert(ncells, r, seed, keys)
    check_table(cells, t)
    g = gpu_list(d, cells, out_cap=out_cap, max_rounds=max_rounds)
    o = native.iblt_list_rounds(t, max_rounds=max_rounds,
                                out_cap=ncells if out_cap is None else out_cap)
    assert g["rounds"] == o.rounds
    assert np.array_equal(g["K"], o.K)
    for a, b in zip(g["groups"], o.per_round()):
        assert np.array_equal(a, b)
    assert g["listed"] == o.keys.size
    check_table(cells, t)  # the consumed tables agree too
    if o.status == native.OK and not o.corrupt:
        assert g["flags"] == 0
        assert g["left"] == keys.size - o.keys.size
    return g, o


def test_insert_small_and_ragged():
    need_gpu()
    for ncells, r, nkeys in [(3, 3, 1), (10, 2, 7), (1000, 3, 700), (4097, 4, 3000),
                             ((1 << 16) + 5, 5, 40000), (12345, 8, 5000)]:
        keys = gen.distinct_keys(nkeys, ncells)
        say("insert", ncells, r, nkeys)
        _, cells = gpu_insert(ncells, r, 99 + r, keys)
        check_table(cells, native.iblt_insert(ncells, r, 99 + r, keys))


@pytest.mark.parametrize("r", [2, 3, 4, 5, 8])
@pytest.mark.parametrize("frac", [0.5, 0.95, 1.1, 1.4])
def test_list_below_and_above_threshold(r, frac):
    need_gpu()
    ncells = (1 << 17) + 77
    cs = theory.cstar(2, r)[0] if r > 2 else 0.5
    m = int(frac * cs * ncells)
    keys = gen.distinct_keys(m, 1000 + r)
    say("list", ncells, r, frac, m)
    g, o = check_list(ncells, r, gen.table_seed(r), keys)
    if frac <= 0.5 and r >= 3:
        assert g["listed"] == m and g["left"] == 0


def test_list_tiny_and_empty():
    need_gpu()
    for ncells, r, m in [(3, 3, 0), (3, 3, 1), (6, 3, 2), (64, 2, 10), (5, 4, 3)]:
        keys = gen.distinct_keys(m, 5 + m)
        say("tiny list", ncells, r, m)
        check_list(ncells, r, 17, keys)


def test_list_limits():
    need_gpu()
    ncells = 1 << 14
    keys = gen.distinct_keys(int(0.7 * ncells), 3)
    for cap in (0, 1, 100, 5000):
        say("out_cap", cap)
        g, o = check_list(ncells, 3, 8, keys, out_cap=cap)
        assert o.status == native.ENOSPC and g["flags"] & 0x4
    for mr in (1, 2, 5):
        say("max_rounds", mr)
        g, o = check_list(ncells, 3, 8, keys, max_rounds=mr)
        assert o.status == native.EROUNDS and g["flags"] & 0x2


@pytest.mark.parametrize("wg", [1, 3, 64])
def test_list_with_fewer_workgroups(wg):
    # a listing given a share of the CUs: same rounds and keys as the oracle
    need_gpu()
    ncells = (1 << 17) + 77
    keys = gen.distinct_keys(int(0.75 * ncells), 77 + wg)
    d, cells = gpu_insert(ncells, 3, 9, keys)
    d = pk.iblt_desc(ncells, 3, 9, workgroups=wg)
    say("list workgroups", wg)
    out = pk.iblt_list(d, cells, max_rounds=4096)
    torch.cuda.synchronize()
    s = out.summary.cpu().numpy()
    o = native.iblt_list_rounds(native.iblt_insert(ncells, 3, 9, keys), max_rounds=4096)
    assert 1 <= int(s[4]) <= wg
    assert int(s[0]) == o.keys.size and int(s[1]) == o.rounds and int(s[3]) == 0
    K = host_u64(out.round_stats)[: int(s[1])]
    assert np.array_equal(K, o.K)
    ks = host_u64(out.keys)[: int(s[0])]
    off = 0
    for kk, want in zip(K.tolist(), o.per_round()):
        assert np.array_equal(np.sort(ks[off: off + kk]), want)
        off += kk


def test_corrupt_cell():
    need_gpu()
    ncells = 1 << 12
    keys = gen.distinct_keys(1000, 40)
    d, cells = gpu_insert(ncells, 3, 5, keys)
    t = native.iblt_insert(ncells, 3, 5, keys)
    c = int(np.flatnonzero(t.count == 1)[0])
    t.hash_sum[c] ^= np.uint64(1)
    cells[c, 2] ^= 1
    say("corrupt", c)
    g = gpu_list(d, cells)
    o = native.iblt_list_rounds(t)
    assert o.corrupt and g["flags"] & 0x8
    assert np.array_equal(g["K"], o.K)
    for a, b in zip(g["groups"], o.per_round()):
        assert np.array_equal(a, b)
    check_table(cells, t)


@pytest.mark.parametrize("r", [3, 4])
def test_list_past_the_owners_lds_bitmaps(r, list_engine):
    # 2^25 + 12345 cells: each of 256 owners holds ~131 K cells, more than its
    # LDS bitmaps cover (98304), so it reads every candidate back and clears
    # each listed key's cell at once instead of at the end
    need_gpu()
    ncells = (1 << 25) + 12345
    keys = gen.distinct_keys(int(0.6 * ncells), 31 + r)
    say("past the LDS bitmaps", list_engine, ncells, r, keys.size)
    g, o = check_list(ncells, r, gen.table_seed(31 + r), keys)
    assert g["listed"] == keys.size and g["left"] == 0


@pytest.mark.parametrize("seed", [1, 2, 3, 4, 5])
def test_config_iblt_full_size(seed):
    # 2^24 cells, r = 3, 10,296,982 keys: every key comes back, round by round as the oracle.
    need_gpu()
    spec = configs.iblt_main()
    keys = spec.keys(seed)
    say(spec.name, "seed", seed)
    g, o = check_list(spec.ncells, spec.r, spec.table_seed(seed), keys)
    assert g["listed"] == spec.nkeys and g["left"] == 0
    assert np.array_equal(np.sort(np.concatenate(g["groups"])), np.sort(keys))


@pytest.mark.parametrize("r,load", [(3, 0.75), (3, 0.83), (4, 0.75), (4, 0.83)])
def test_paper_table_shapes_full_size(r, load):
    # The IBLT shapes of the paper's Tables 5-6: 2^24 cells at loads 0.75 / 0.83.
    need_gpu()
    spec = configs.iblt_paper(r, load)
    keys = spec.keys(2)
    say(spec.name)
    g, o = check_list(spec.ncells, spec.r, spec.table_seed(2), keys)
