"""GPU parity of the batched IBLT listing (many tables, one launch).

Every table of a batch must come out exactly as the oracle lists it, round by
round, and exactly as iblt_list lists it alone.
"""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native, theory
from workloads import configs, gen

from gpu_helpers import dev_u64, host_u64, need_gpu, say, table_to_numpy

pytestmark = pytest.mark.gpu


def _make_tables(specs, max_rounds):
    """specs: [(ncells, r, nkeys, seed)] -> (BatchTables, keys, pristine copies)."""
    tables, keys, pristine = [], [], []
    for ncells, r, nkeys, seed in specs:
        k = gen.distinct_keys(nkeys, seed)
        d = pk.iblt_desc(ncells, r, gen.table_seed(seed))
        cells = pk.iblt_table(ncells, "cuda")
        if nkeys:
            pk.iblt_insert(d, cells, dev_u64(k))
        tables.append(pk.batch_table(d, cells, max_rounds))
        keys.append(k)
        pristine.append(cells.clone())
    torch.cuda.synchronize()
    return tables, keys, pristine


def _result(t: pk.BatchTable):
    s = t.summary.cpu().numpy()
    listed, rounds = int(s[0]), int(s[1])
    K = host_u64(t.round_stats)[:rounds]
    ks = host_u64(t.keys)[:listed]
    groups, off = [], 0
    for kk in K.tolist():
        groups.append(np.sort(ks[off: off + kk]))
        off += kk
    return s, K, groups


def _check_against_oracle(t, k, max_rounds):
    s, K, groups = _result(t)
    o_tab = native.iblt_insert(t.desc.ncells, t.desc.r, t.desc.seed, k)
    o = native.iblt_list_rounds(o_tab, max_rounds=max_rounds, out_cap=t.keys.numel())
    assert int(s[1]) == o.rounds
    assert np.array_equal(K, o.K)
    for a, b in zip(groups, o.per_round()):
        assert np.array_equal(a, b)
    count, ksum, hsum, ok = table_to_numpy(t.cells)
    assert ok
    assert np.array_equal(count, o_tab.count)
    assert np.array_equal(ksum, o_tab.key_sum) and np.array_equal(hsum, o_tab.hash_sum)
    if o.status == native.OK:
        assert int(s[3]) == 0 and int(s[2]) == k.size - o.keys.size


def _specs(n, seed, lo=6, hi=14, rs=(2, 3, 4, 5)):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        r = int(rng.choice(rs))
        N = max(r, int(2 ** rng.uniform(lo, hi)))
        cs = theory.cstar(2, r)[0] if r > 2 else 0.5
        load = rng.uniform(0.3, 1.2) * cs
        out.append((N, r, int(load * N), 1000 * seed + i))
    return out


@pytest.mark.parametrize("lds", [0, pk.IBLT_LDS_MAX_CELLS])
@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_batched_matches_oracle(threads, lds):
    # tables of 2^6 .. 2^14 cells: with lds on, those the workgroup size holds
    # (pk.IBLT_LDS_CELLS) are listed in LDS, the larger ones in place
    need_gpu()
    specs = _specs(48, 3)
    specs.sort(key=lambda x: -x[0])
    tables, keys, _ = _make_tables(specs, 256)
    ent = pk.batch_entries(tables, "cuda")
    say("batched", len(tables), "threads", threads, "lds", lds)
    pk.iblt_list_batched(ent, len(tables), max(x[0] for x in specs), 256, block_threads=threads,
                         lds_max_cells=lds)
    torch.cuda.synchronize()
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 256)


@pytest.mark.parametrize("threads", [256, 1024])
def test_in_place_filter_folds(threads):
    # The in-place schedule's ownership filter has one LDS bit per lower-subtable
    # cell up to 360,448 bits (256 threads) or 917,504 (1024 threads); these
    # tables have more lower cells than that, so cells share bits (a shared bit
    # only costs a read).  One is above threshold, so a core remains.
    need_gpu()
    c3, c4 = theory.cstar(2, 3)[0], theory.cstar(2, 4)[0]
    specs = [(1_500_000, 3, int(0.80 * c3 * 1_500_000), 41),
             (1_300_001, 4, int(0.90 * c4 * 1_300_001), 42),
             (1_400_000, 3, int(1.05 * c3 * 1_400_000), 43),
             (800_003, 2, int(0.45 * 800_003), 44),
             (600_000, 3, int(0.75 * c3 * 600_000), 45)]
    tables, keys, _ = _make_tables(specs, 256)
    ent = pk.batch_entries(tables, "cuda")
    say("batched filter folds", len(tables), "threads", threads)
    pk.iblt_list_batched(ent, len(tables), max(x[0] for x in specs), 256, block_threads=threads,
                         lds_max_cells=0)
    torch.cuda.synchronize()
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 256)


@pytest.mark.parametrize("threads", [256, 512, 1024])
def test_lds_schedule_edges(threads):
    # LDS-resident tables at the size limit of the workgroup size and around it,
    # above threshold (a core remains), a tiny round limit, a tiny output capacity
    # and a corrupt cell.
    need_gpu()
    L = pk.IBLT_LDS_CELLS[threads]
    specs = [(L, 3, int(0.80 * L), 11), (L, 4, int(0.90 * L), 12), (L + 1, 3, int(0.7 * L), 13),
             (L - 1, 5, int(0.6 * L), 14), (L, 2, int(0.45 * L), 15), (777, 3, 600, 16),
             (3, 3, 1, 17), (4, 4, 0, 18), (L, 3, int(0.75 * L), 19), (L, 3, int(0.7 * L), 20)]
    tables, keys, _ = _make_tables(specs, 64)
    tables[-1] = pk.batch_table(tables[-1].desc, tables[-1].cells, 64, out_cap=100)
    # corrupt one count-1 cell of table 5 (its checksum no longer matches)
    o5 = native.iblt_insert(specs[5][0], 3, gen.table_seed(specs[5][3]), keys[5])
    c = int(np.flatnonzero(o5.count == 1)[0])
    tables[5].cells[c, 2] ^= 1
    ent = pk.batch_entries(tables, "cuda")
    say("lds edges", threads)
    pk.iblt_list_batched(ent, len(tables), L + 1, 64, block_threads=threads, lds_max_cells=L)
    torch.cuda.synchronize()
    for i, (t, k) in enumerate(zip(tables, keys)):
        if i == 5:
            o5.hash_sum[c] ^= np.uint64(1)
            o = native.iblt_list_rounds(o5, max_rounds=64)
            s, K, groups = _result(t)
            assert o.corrupt and int(s[3]) & 0x8
            assert np.array_equal(K, o.K)
            for a, b in zip(groups, o.per_round()):
                assert np.array_equal(a, b)
            count, ksum, hsum, ok = table_to_numpy(t.cells)
            assert np.array_equal(count, o5.count) and np.array_equal(ksum, o5.key_sum)
            assert np.array_equal(hsum, o5.hash_sum)
            continue
        _check_against_oracle(t, k, 64)
    assert int(tables[-1].summary[3]) & 0x4   # ENOSPC
    # a round limit of 3 for a batch of LDS-resident and in-place tables
    specs = [(L, 3, int(0.78 * L), 21), (L + 64, 3, int(0.78 * L), 22), (1500, 4, 1000, 23)]
    tables, keys, _ = _make_tables(specs, 3)
    ent = pk.batch_entries(tables, "cuda")
    say("lds round limit", threads)
    pk.iblt_list_batched(ent, len(tables), L + 64, 3, block_threads=threads, lds_max_cells=L)
    torch.cuda.synchronize()
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 3)
        assert int(t.summary[3]) & 0x2   # EROUNDS


def test_batched_equals_each_table_alone():
    need_gpu()
    specs = _specs(24, 5, lo=8, hi=16)
    tables, keys, pristine = _make_tables(specs, 128)
    ent = pk.batch_entries(tables, "cuda")
    say("batched vs alone")
    pk.iblt_list_batched(ent, len(tables), max(x[0] for x in specs), 128)
    torch.cuda.synchronize()
    for t, p in zip(tables, pristine):
        alone = pk.iblt_list(t.desc, p, max_rounds=128)
        torch.cuda.synchronize()
        sb, Kb, gb = _result(t)
        sa = alone.summary.cpu().numpy()
        assert int(sa[0]) == int(sb[0]) and int(sa[1]) == int(sb[1]) and int(sa[3]) == int(sb[3])
        ka = host_u64(alone.keys)[: int(sa[0])]
        off = 0
        for g in gb:
            assert np.array_equal(np.sort(ka[off: off + g.size]), g)
            off += g.size
        assert torch.equal(p, t.cells)


def test_batched_limits_and_degenerate():
    need_gpu()
    specs = [(3, 3, 0, 1), (3, 3, 1, 2), (5, 4, 3, 3), (4096, 3, 2500, 4), (4096, 3, 3000, 5)]
    tables, keys, _ = _make_tables(specs, 64)
    # the last table gets a tiny output capacity and the fourth a tiny round limit
    tables[-1] = pk.batch_table(tables[-1].desc, tables[-1].cells, 64, out_cap=10)
    ent = pk.batch_entries(tables, "cuda")
    say("limits")
    pk.iblt_list_batched(ent, len(tables), 4096, 64)
    torch.cuda.synchronize()
    for t, k in zip(tables[:-1], keys[:-1]):
        _check_against_oracle(t, k, 64)
    s, _, _ = _result(tables[-1])
    assert int(s[3]) & 0x4  # ENOSPC
    _check_against_oracle(tables[-1], keys[-1], 64)


def test_batched_in_a_captured_graph_replays():
    need_gpu()
    specs = _specs(32, 7, lo=8, hi=13)
    tables, keys, pristine = _make_tables(specs, 128)
    ent = pk.batch_entries(tables, "cuda")
    maxc = max(x[0] for x in specs)
    ws = pk.workspace(pk.iblt_list_batched_workspace(len(tables), maxc), "cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm up on the capture stream
        pk.iblt_list_batched(ent, len(tables), maxc, 128, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    eager = [_result(t) for t in tables]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        pk.iblt_list_batched(ent, len(tables), maxc, 128, ws=ws)
    for rep in range(3):
        for t, p in zip(tables, pristine):
            t.cells.copy_(p)
        torch.cuda.synchronize()
        say("graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        for t, (se, Ke, ge) in zip(tables, eager):
            sr, Kr, gr = _result(t)
            assert np.array_equal(se[:4], sr[:4]) and np.array_equal(Ke, Kr)
            for a, b in zip(ge, gr):
                assert np.array_equal(a, b)


@pytest.mark.parametrize("which", ["main", "partial"])
def test_config_batched_sample(which):
    # The 4096-table workload (cells log-uniform in [2^10, 2^20], load 0.5-0.8 c*),
    # and the same batch with a seeded 5% of its tables at load 1.0-1.2 c*: all
    # listed in one launch. Sampled tables (hot ones among them) are checked
    # against the oracle round by round; tables below threshold come back whole
    # and most hot tables keep a core.
    need_gpu()
    spec = configs.batched_main() if which == "main" else configs.batched_partial()
    draw = spec.draw(1)
    base = configs.batched_main().draw(1)
    hot = {i for i in range(len(draw)) if draw[i] != base[i]}
    rng = np.random.default_rng(0)
    pick = set(rng.choice(len(draw), 24, replace=False).tolist())
    if hot:
        pick |= set(rng.choice(sorted(hot), 16, replace=False).tolist())
    order = sorted(range(len(draw)), key=lambda i: -draw[i][0])
    tables, keys = [], []
    for i in order:
        N, m, ks, ts = draw[i]
        k = gen.distinct_keys(m, ks)
        d = pk.iblt_desc(N, spec.r, ts)
        cells = pk.iblt_table(N, "cuda")
        pk.iblt_insert(d, cells, dev_u64(k))
        tables.append(pk.batch_table(d, cells, 256))
        keys.append(k if i in pick else None)
    ent = pk.batch_entries(tables, "cuda")
    torch.cuda.synchronize()
    say("config batched 4096", which, len(hot), "hot")
    pk.iblt_list_batched(ent, len(tables), max(x[0] for x in draw), 256)
    torch.cuda.synchronize()
    left_cold, left_hot = 0, 0
    for i, t, k in zip(order, tables, keys):
        s = t.summary.cpu().numpy()
        assert int(s[3]) == 0  # no round limit, no overflow, no corrupt cell
        if k is not None:
            _check_against_oracle(t, k, 256)
        if i in hot:
            left_hot += int(s[2]) > 0
        else:
            left_cold += int(s[2]) > 0
    assert left_cold <= 0.01 * (len(tables) - len(hot))
    if hot:
        assert left_hot >= 0.5 * len(hot)


def _oracle_groups(N, r, ts, k, max_rounds, cap):
    """The oracle's listing of one table: (summary-like tuple, K, groups, final table)."""
    o_tab = native.iblt_insert(N, r, ts, k)
    o = native.iblt_list_rounds(o_tab, max_rounds=max_rounds, out_cap=cap)
    return o, o_tab


@pytest.mark.timeout(900)
@pytest.mark.parametrize("which", ["main", "partial"])
def test_config_batched_every_table(which):
    # Every one of the 4096 tables of the batched workload (and of the partial
    # batch) against the oracle round by round -- per-round sorted key sets,
    # K_t, rounds, summary, final cells -- and against its own plain iblt_list.
    # The oracle runs on host threads (the C oracle releases the GIL).
    need_gpu()
    import concurrent.futures as cf
    spec = configs.batched_main() if which == "main" else configs.batched_partial()
    draw = spec.draw(1)
    order = sorted(range(len(draw)), key=lambda i: -draw[i][0])
    maxr = 256
    tables, pristine = [], []
    say("every table", which, "inserting")
    for i in order:
        N, m, ks, ts = draw[i]
        d = pk.iblt_desc(N, spec.r, ts)
        cells = pk.iblt_table(N, "cuda")
        pk.iblt_insert(d, cells, gen.distinct_keys_torch(m, ks, "cuda"))
        tables.append(pk.batch_table(d, cells, maxr))
        pristine.append(cells.clone())
    ent = pk.batch_entries(tables, "cuda")
    torch.cuda.synchronize()
    say("every table", which, "batched launch")
    pk.iblt_list_batched(ent, len(tables), max(x[0] for x in draw), maxr)
    torch.cuda.synchronize()
    # the plain per-table listing of a copy of each table
    plain = []
    for t, p in zip(tables, pristine):
        lo = pk.iblt_list(t.desc, p, max_rounds=maxr)
        plain.append(lo)
    torch.cuda.synchronize()
    say("every table", which, "plain launches done; oracle on host threads")

    def check(j):
        i = order[j]
        N, m, ks, ts = draw[i]
        t = tables[j]
        s, K, groups = _result(t)
        o, o_tab = _oracle_groups(N, spec.r, ts, gen.distinct_keys(m, ks), maxr, t.keys.numel())
        bad = []
        if int(s[1]) != o.rounds or not np.array_equal(K, o.K):
            bad.append("rounds")
        if any(not np.array_equal(a, b) for a, b in zip(groups, o.per_round())):
            bad.append("keys")
        count, ksum, hsum, ok = table_to_numpy(t.cells)
        if not (ok and np.array_equal(count, o_tab.count) and np.array_equal(ksum, o_tab.key_sum)
                and np.array_equal(hsum, o_tab.hash_sum)):
            bad.append("cells")
        if int(s[0]) != o.keys.size or int(s[2]) != m - o.keys.size or int(s[3]) != 0:
            bad.append("summary")
        # plain iblt_list on the same table: same summary, rounds and key sets
        ps = plain[j].summary.cpu().numpy()
        pK = host_u64(plain[j].round_stats)[: int(ps[1])]
        pk_ = host_u64(plain[j].keys)[: int(ps[0])]
        if not (np.array_equal(ps[:4], s[:4]) and np.array_equal(pK, K)):
            bad.append("plain summary")
        off = 0
        for kk, g in zip(K.tolist(), groups):
            if not np.array_equal(np.sort(pk_[off: off + kk]), g):
                bad.append("plain keys")
                break
            off += kk
        return j, bad, int(s[2]) > 0

    fails, left = [], 0
    with cf.ThreadPoolExecutor(max_workers=16) as ex:
        for n_done, (j, bad, kept) in enumerate(ex.map(check, range(len(tables))), 1):
            if bad:
                fails.append((j, bad))
            left += kept
            if n_done % 512 == 0:
                say("every table", which, n_done, "checked,", len(fails), "mismatches")
    assert fails == []
    say("every table", which, "tables that kept a core:", left)


def test_bad_entries_are_skipped_and_flagged():
    # An entry with r out of range, more cells than max_cells, or misaligned
    # cells is not listed; its summary says PEEL_FLAG_EINVAL and the other
    # tables of the launch are listed as usual.
    need_gpu()
    specs = _specs(6, 8, lo=8, hi=11, rs=(3,))
    tables, keys, pristine = _make_tables(specs, 64)
    ent = pk.batch_entries(tables, "cuda")
    raw = ent.cpu().numpy().view(np.dtype(pk.binding.BATCH_ENTRY)).copy()
    raw[1]["r"] = 9
    raw[3]["ncells"] = 1 << 20  # beyond max_cells below
    raw[4]["cells"] += 8        # not 32-byte aligned
    bad_ent = torch.from_numpy(raw.view(np.uint8).copy()).cuda()
    maxc = max(x[0] for x in specs)
    for i in (1, 3, 4):
        tables[i].summary.fill_(-1)
    say("bad batch entries")
    pk.iblt_list_batched(bad_ent, len(tables), maxc, 64)
    torch.cuda.synchronize()
    for i, (t, k, p) in enumerate(zip(tables, keys, pristine)):
        s = t.summary.cpu().numpy()
        if i in (1, 3, 4):
            assert s.tolist() == [0, 0, 0, pk.FLAG_EINVAL, 0, 0, 0, 0]
            assert torch.equal(t.cells, p)  # untouched
        else:
            _check_against_oracle(t, k, 64)


@pytest.mark.parametrize("threads,lds,tmin,G", [(256, 0, 1 << 12, 2), (512, pk.IBLT_LDS_MAX_CELLS, 1 << 13, 4),
                                                (1024, 0, 1 << 12, 16), (1024, pk.IBLT_LDS_MAX_CELLS, 1 << 14, 64)])
def test_team_schedule_matches_oracle(threads, lds, tmin, G):
    # tables of at least tmin cells are listed by teams of G workgroups; every
    # table, whatever its schedule, equals the oracle round by round
    need_gpu()
    specs = _specs(40, 5, lo=8, hi=16)
    specs.sort(key=lambda x: -x[0])
    tables, keys, _ = _make_tables(specs, 256)
    ent = pk.batch_entries(tables, "cuda")
    say("team schedule", threads, lds, tmin, G)
    pk.iblt_list_batched(ent, len(tables), max(x[0] for x in specs), 256, block_threads=threads,
                         lds_max_cells=lds, tile_min_cells=tmin, tile_workgroups=G)
    torch.cuda.synchronize()
    teams = 0
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 256)
        s = t.summary.cpu().numpy()
        want = G if t.desc.ncells >= tmin else 1
        assert int(s[4]) == want
        teams += want > 1
    assert teams >= 5


@pytest.mark.parametrize("ntables,G", [(1, 64), (3, 16), (2, 2)])
def test_team_schedule_few_tables(ntables, G):
    # fewer tables than a team has members: the launch still holds a whole team
    need_gpu()
    specs = [((1 << 18) + 17 * i, 3, int(0.7 * 0.818 * ((1 << 18) + 17 * i)), 60 + i)
             for i in range(ntables)]
    tables, keys, pristine = _make_tables(specs, 256)
    ent = pk.batch_entries(tables, "cuda")
    say("team few tables", ntables, G)
    pk.iblt_list_batched(ent, ntables, max(x[0] for x in specs), 256, tile_min_cells=1 << 16,
                         tile_workgroups=G)
    torch.cuda.synchronize()
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 256)
        assert int(t.summary[4].item()) == G


def test_team_schedule_limits():
    # a team table with a round limit, one with a tiny output capacity, one
    # with a corrupt cell, and one above the threshold (a core is left)
    need_gpu()
    N = 1 << 15
    specs = [(N, 3, int(0.70 * 0.818 * N), 71), (N, 3, int(0.70 * 0.818 * N), 72),
             (N, 3, int(0.70 * 0.818 * N), 73), (N, 4, int(0.85 * N), 74)]
    tables, keys, _ = _make_tables(specs, 3)
    tables[1] = pk.batch_table(tables[1].desc, tables[1].cells, 3, out_cap=1000)
    o2 = native.iblt_insert(N, 3, gen.table_seed(73), keys[2])
    c = int(np.flatnonzero(o2.count == 1)[0])
    tables[2].cells[c, 2] ^= 1 << 40
    ent = pk.batch_entries(tables, "cuda")
    say("team limits")
    pk.iblt_list_batched(ent, len(tables), N, 3, tile_min_cells=N, tile_workgroups=8)
    torch.cuda.synchronize()
    for i, (t, k) in enumerate(zip(tables, keys)):
        if i == 2:
            # the oracle lists the same corrupted table
            o2.hash_sum[c] ^= np.uint64(1 << 40)
            o = native.iblt_list_rounds(o2, max_rounds=3)
            s, K, groups = _result(t)
            assert o.corrupt and int(s[3]) & pk.FLAG_ECORRUPT
            assert np.array_equal(K, o.K)
            for a, b in zip(groups, o.per_round()):
                assert np.array_equal(a, b)
            count, ksum, hsum, ok = table_to_numpy(t.cells)
            assert np.array_equal(count, o2.count) and np.array_equal(ksum, o2.key_sum)
            assert np.array_equal(hsum, o2.hash_sum)
            continue
        _check_against_oracle(t, k, 3)
    assert int(tables[0].summary[3].item()) & pk.FLAG_EROUNDS
    assert int(tables[1].summary[3].item()) & pk.FLAG_ENOSPC


def test_team_schedule_graph_replays():
    # captured once, replayed three times on restored tables: every replay exact
    need_gpu()
    specs = _specs(24, 9, lo=10, hi=16, rs=(3,))
    specs.sort(key=lambda x: -x[0])
    tables, keys, pristine = _make_tables(specs, 128)
    ent = pk.batch_entries(tables, "cuda")
    maxc = max(x[0] for x in specs)
    ws = pk.workspace(pk.iblt_list_batched_workspace(len(tables), maxc), "cuda")
    kw = dict(block_threads=512, tile_min_cells=1 << 13, tile_workgroups=8, ws=ws)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        pk.iblt_list_batched(ent, len(tables), maxc, 128, **kw)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    for t, p in zip(tables, pristine):
        t.cells.copy_(p)
    with torch.cuda.graph(g):
        pk.iblt_list_batched(ent, len(tables), maxc, 128, **kw)
    for rep in range(3):
        for t, p in zip(tables, pristine):
            t.cells.copy_(p)
        torch.cuda.synchronize()
        say("team graph replay", rep)
        g.replay()
        torch.cuda.synchronize()
        for t, k in zip(tables, keys):
            _check_against_oracle(t, k, 128)


def test_autotuner_per_class_schedule_is_exact():
    # the tuner times each size class on its own tables, combines the choices
    # and leaves every table as it found it; its schedule lists exactly
    need_gpu()
    from paper_1302_7014_amd.autotune import LARGE_MIN, tune_batched
    specs = _specs(20, 13, lo=8, hi=12, rs=(3,)) + [
        (LARGE_MIN + 1000 * i, 3, int(0.7 * 0.818 * LARGE_MIN), 900 + i) for i in range(3)] + [
        (N, 3, int(0.7 * 0.818 * N), 950 + i) for i, N in enumerate((8000, 12000, 30000))]
    specs.sort(key=lambda x: -x[0])
    tables, keys, pristine = _make_tables(specs, 128)
    ent = pk.batch_entries(tables, "cuda")
    maxc = max(x[0] for x in specs)
    ws = pk.workspace(pk.iblt_list_batched_workspace(len(tables), maxc), "cuda")
    say("autotuner")
    sched, rep = tune_batched(tables, ent, maxc, 128, ws, reps=1)
    assert set(rep["classes"]) == {"small", "medium", "large"}
    assert len(rep["combined"]) == 3
    for t, p in zip(tables, pristine):
        assert torch.equal(t.cells, p)
    pk.iblt_list_batched(ent, len(tables), maxc, 128, ws=ws, **sched)
    torch.cuda.synchronize()
    for t, k in zip(tables, keys):
        _check_against_oracle(t, k, 128)
