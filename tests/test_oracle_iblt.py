"""Pins for the oracle's IBLT routines (paper, Section 5)."""
import numpy as np
import pytest

from oracle import native, theory
from workloads import gen


def _table(ncells, r, nkeys, seed):
    keys = gen.distinct_keys(nkeys, seed)
    t = native.iblt_insert(ncells, r, gen.table_seed(seed), keys)
    return keys, t


def test_insert_then_delete_is_identity():
    # Insert and delete XOR the same values (Section 5, "Motivation").
    keys, t = _table(1 << 12, 3, 2000, seed=1)
    native.iblt_update(t, keys, sign=-1)
    assert t.is_empty()


def test_insert_matches_cell_hashes():
    keys, t = _table(3000, 4, 500, seed=2)
    cells, chk = native.iblt_cells_of(3000, 4, t.seed, keys)
    # one cell per subtable: cell j lies in subtable j's id range
    sizes = gen.subtable_sizes(3000, 4)
    bases = gen.subtable_bases(3000, 4)
    for j in range(4):
        assert ((cells[:, j] >= bases[j]) & (cells[:, j] < bases[j] + sizes[j])).all()
    cnt = np.bincount(cells.ravel().astype(np.int64), minlength=3000)
    assert np.array_equal(cnt, t.count)
    ks = np.zeros(3000, np.uint64)
    hs = np.zeros(3000, np.uint64)
    for j in range(4):
        np.bitwise_xor.at(ks, cells[:, j].astype(np.int64), keys)
        np.bitwise_xor.at(hs, cells[:, j].astype(np.int64), chk)
    assert np.array_equal(ks, t.key_sum) and np.array_equal(hs, t.hash_sum)


@pytest.mark.parametrize("r", [3, 4])
def test_below_threshold_recovers_the_inserted_set(r):
    N = 1 << 15
    m = int(0.8 * theory.cstar(2, r)[0] * N)
    keys, t = _table(N, r, m, seed=10 + r)
    res = native.iblt_list_rounds(t)
    assert res.status == native.OK and not res.corrupt
    assert np.array_equal(np.sort(res.keys), np.sort(keys))
    assert t.is_empty()
    # keys within a round are distinct and ascending
    for grp in res.per_round():
        assert (np.diff(grp.astype(np.float64)) > 0).all() or grp.size <= 1


@pytest.mark.parametrize("r,load", [(3, 0.83), (4, 0.83), (3, 0.9)])
def test_listing_equals_peeling_the_key_hypergraph(r, load):
    # Section 5: keys are edges, cells are vertices, pure cells are vertices of
    # degree < 2; listing round t yields exactly the edges the parallel 2-core
    # peel removes in round t, and the keys left are the 2-core's edges.
    N = 1 << 14
    m = int(load * N)
    keys, t = _table(N, r, m, seed=20 + r)
    cells, _ = native.iblt_cells_of(N, r, t.seed, keys)
    peel = native.peel_rounds(N, cells.astype(np.uint32), 2)
    res = native.iblt_list_rounds(t.copy())
    assert res.rounds == peel.edge_rounds
    for rnd, grp in enumerate(res.per_round(), start=1):
        want = np.sort(keys[peel.edge_round == rnd])
        assert np.array_equal(grp, want), rnd
    left = keys[peel.edge_round == 0]
    # the sequential listing finds the same set (the 2-core is order independent)
    seq = native.iblt_list_seq(t.copy())
    assert np.array_equal(np.sort(seq), np.sort(res.keys))
    # XOR linearity: what is left equals a fresh insertion of the unlisted keys
    rest = t.copy()
    native.iblt_list_rounds(rest)
    fresh = native.iblt_insert(N, r, t.seed, left)
    assert np.array_equal(rest.count, fresh.count)
    assert np.array_equal(rest.key_sum, fresh.key_sum)
    assert np.array_equal(rest.hash_sum, fresh.hash_sum)


def test_recovered_fraction_near_paper_r4_load083(golden):
    # Table 6: r = 4, load 0.83 recovers 24.6% of the items (2^24 cells there; 2^20 here).
    N = 1 << 20
    keys, t = _table(N, 4, int(0.83 * N), seed=31)
    res = native.iblt_list_rounds(t)
    frac = 100.0 * res.keys.size / keys.size
    assert abs(frac - 24.6) < 1.0, frac


def test_corrupt_cell_is_flagged_not_listed():
    # A count-1 cell whose checksum field does not match its key field is not pure.
    keys, t = _table(1 << 12, 3, 1000, seed=40)
    c = int(np.flatnonzero(t.count == 1)[0])
    t.hash_sum[c] ^= np.uint64(1)
    res = native.iblt_list_rounds(t)
    assert res.corrupt
    assert np.isin(res.keys, keys).all()
    # the key is still listed through its other cells; only the planted bit is left
    assert res.keys.size == keys.size
    assert not t.count.any() and not t.key_sum.any()
    assert np.flatnonzero(t.hash_sum).tolist() == [c] and int(t.hash_sum[c]) == 1


def test_out_capacity_and_round_limit():
    keys, t = _table(1 << 12, 3, 2000, seed=41)
    res = native.iblt_list_rounds(t.copy(), out_cap=10)
    assert res.status == native.ENOSPC
    full = native.iblt_list_rounds(t.copy())
    part = native.iblt_list_rounds(t.copy(), max_rounds=2)
    assert part.status == native.EROUNDS
    assert np.array_equal(part.K, full.K[:2])


@pytest.mark.parametrize("r,load", [(3, 0.75), (4, 0.83), (3, 0.9), (2, 0.45)])
def test_subround_listing_equals_peeling_the_key_hypergraph_with_subtables(r, load):
    # The paper's GPU process (Section 5, Appendix B): subround (i, j) lists the
    # pure cells of subtable j.  On the key -> cell hypergraph (cells split into
    # the same subtables) that is peeling with subtables at k = 2: subround s
    # lists exactly the edges that subround removes.  The listed set is the
    # round-synchronous one (the 2-core does not depend on the order), and what
    # is left is the same table.
    N = (1 << 14) + 5
    m = int(load * N)
    keys, t = _table(N, r, m, seed=40 + r)
    cells, _ = native.iblt_cells_of(N, r, t.seed, keys)
    peel = native.peel_subrounds(N, cells.astype(np.uint32), 2)
    sub_t = t.copy()
    res = native.iblt_list_subrounds(sub_t)
    assert res.status == native.OK and not res.corrupt
    assert res.rounds == peel.edge_rounds
    for s, grp in enumerate(res.per_round(), start=1):
        assert np.array_equal(grp, np.sort(keys[peel.edge_round == s])), s
    rnd_t = t.copy()
    rnd = native.iblt_list_rounds(rnd_t)
    assert np.array_equal(np.sort(res.keys), np.sort(rnd.keys))
    assert np.array_equal(sub_t.count, rnd_t.count)
    assert np.array_equal(sub_t.key_sum, rnd_t.key_sum)
    assert np.array_equal(sub_t.hash_sum, rnd_t.hash_sum)


def test_subround_listing_limits_and_corrupt_cell():
    keys, t = _table(4096, 3, 2800, seed=61)
    full = native.iblt_list_subrounds(t.copy())
    # a round limit stops before the first subround past it that would list a key
    cut = native.iblt_list_subrounds(t.copy(), max_rounds=4)
    assert cut.status == native.EROUNDS and cut.rounds <= 4
    assert np.array_equal(cut.K, full.K[: cut.rounds])
    # an output capacity stops before the subround that would overflow it
    cap = int(full.K[:3].sum()) + 1
    small = native.iblt_list_subrounds(t.copy(), out_cap=cap)
    assert small.status == native.ENOSPC and small.keys.size <= cap
    assert np.array_equal(small.keys, full.keys[: small.keys.size])
    # a count-1 cell with a wrong checksum is not pure and is reported
    bad = t.copy()
    c = int(np.flatnonzero(bad.count == 1)[0])
    bad.hash_sum[c] ^= np.uint64(1)
    res = native.iblt_list_subrounds(bad)
    assert res.corrupt


@pytest.mark.parametrize("r", [3, 4])
def test_signed_listing_recovers_the_set_difference(r):
    # Section 5: insert A, delete B; below threshold the listing recovers
    # A \ B with sign +1 and B \ A with sign -1, exactly, and empties the table.
    N = (1 << 14) + 3
    pool = gen.distinct_keys(int(0.95 * N), 70 + r)
    a = pool[: int(0.65 * N)]
    b = pool[int(0.35 * N):]  # shares 0.3 N keys with a
    seed = gen.table_seed(70 + r)
    t = native.iblt_insert(N, r, seed, a)
    native.iblt_update(t, b, sign=-1)
    res = native.iblt_list_signed(t.copy())
    assert res.status == native.OK and res.nonempty == 0
    plus = np.sort(res.keys[res.signs == 1])
    minus = np.sort(res.keys[res.signs == -1])
    assert np.array_equal(plus, np.sort(np.setdiff1d(a, b)))
    assert np.array_equal(minus, np.sort(np.setdiff1d(b, a)))
    assert set(res.signs.tolist()) <= {1, -1}


def test_signed_listing_rounds_equal_plain_listing_of_the_difference():
    # Counts and XORs are linear: the table of (insert A, delete B) has the pure
    # cells of the table of A xor B inserted, up to checksum collisions, so the
    # round-by-round key sets are those of the plain listing of A xor B; above
    # the threshold both stop at the same core.
    for r, frac in [(3, 0.7), (3, 0.95), (4, 0.9)]:
        N = 1 << 14
        pool = gen.distinct_keys(int(1.6 * frac * N), 80 + r)
        half = pool.size // 2
        a, b = pool[: half + half // 2], pool[half // 2:]
        diff = np.setxor1d(a, b)
        seed = gen.table_seed(80 + r)
        t = native.iblt_insert(N, r, seed, a)
        native.iblt_update(t, b, sign=-1)
        res = native.iblt_list_signed(t)
        plain = native.iblt_list_rounds(native.iblt_insert(N, r, seed, diff))
        assert res.rounds == plain.rounds
        assert np.array_equal(res.K, plain.K)
        for (ks, sg), want in zip(res.per_round(), plain.per_round()):
            assert np.array_equal(ks, want)
            assert np.array_equal(sg, np.where(np.isin(ks, a), 1, -1).astype(np.int8))
        assert res.nonempty == int(((t.count != 0) | (t.key_sum != 0) | (t.hash_sum != 0)).sum())
