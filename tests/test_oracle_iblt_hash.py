"""Pins the IBLT hash convention of the oracle against an independent restatement.

The convention is the one the library's header documents for a table of
``ncells`` cells split into r near-equal subtables (Section 5, "Implementation
Details"; Appendix B): key x goes to cell ``base_j + floor(H_j(x) * size_j /
2^64)`` of subtable j, with ``H_j(x) = mix64(x ^ salt_j)``; its checksum is
``C(x) = mix64(x ^ salt_c)``; ``salt_j`` (j < r) and ``salt_c`` are draws j and
8 of the SplitMix64 stream whose state starts at the table seed.

The restatement below uses Python integers only (no numpy, no oracle code), so
a wrong salt index, subtable split, reduction or finaliser constant in the
oracle fails here.
"""
import numpy as np
import pytest

from oracle import native
from workloads import gen

M64 = (1 << 64) - 1


def _mix64(z: int) -> int:
    # SplitMix64 output finaliser (Steele, Lea and Flood, OOPSLA 2014)
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _draw(seed: int, i: int) -> int:
    # the (i+1)-th output of a SplitMix64 state that starts at `seed`
    return _mix64(seed + (i + 1) * 0x9E3779B97F4A7C15)


def _cells_of(ncells: int, r: int, seed: int, x: int):
    sizes = [ncells // r + (1 if j < ncells % r else 0) for j in range(r)]
    bases = [sum(sizes[:j]) for j in range(r)]
    cells = [bases[j] + ((_mix64(x ^ _draw(seed, j)) * sizes[j]) >> 64) for j in range(r)]
    return cells, _mix64(x ^ _draw(seed, 8))


def test_splitmix64_reference_values():
    # Sequence of a SplitMix64 state seeded with 1234567, as published with the
    # generator's reference code; pins the finaliser and the stream stepping.
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [_draw(1234567, i) for i in range(5)] == want


@pytest.mark.parametrize("ncells,r", [(3, 3), (7, 2), (1000, 3), (4099, 4), (65537, 5),
                                      (1 << 20, 8), ((1 << 24) + 11, 3)])
def test_oracle_cells_follow_the_documented_formula(ncells, r):
    seed = gen.table_seed(ncells * 31 + r)
    keys = gen.distinct_keys(257, seed=ncells + r)
    # edge cases: key 0, all ones, and keys equal to a salt (x ^ salt_j = 0)
    extra = [0, M64, _draw(seed, 0), _draw(seed, r - 1), _draw(seed, 8)]
    keys = np.concatenate([keys, np.array(extra, dtype=np.uint64)])
    cells, chk = native.iblt_cells_of(ncells, r, seed, keys)
    for i, x in enumerate(keys.tolist()):
        want_cells, want_chk = _cells_of(ncells, r, seed, int(x))
        assert cells[i].tolist() == want_cells, (ncells, r, i)
        assert int(chk[i]) == want_chk, (ncells, r, i)


def test_generator_helpers_agree_with_the_restatement():
    # The seeded input generator's own SplitMix64 and multiply-shift (shared by
    # the tests, the bench and the oracle's callers) against the same restatement.
    seed = 0x0123456789ABCDEF
    idx = np.arange(64, dtype=np.uint64)
    got = gen.splitmix64(seed, idx).tolist()
    assert got == [_draw(seed, int(i)) for i in idx]
    u = gen.splitmix64(seed, idx)
    for s in (1, 3, 5592405, (1 << 32) - 1):
        red = gen.mulhi_reduce(u, s).tolist()
        assert red == [(int(x) * s) >> 64 for x in u.tolist()]


def test_table_insert_uses_those_cells():
    # The table the oracle builds holds every key in exactly the restated cells.
    ncells, r = 5003, 3
    seed = gen.table_seed(9)
    keys = gen.distinct_keys(300, seed=9)
    t = native.iblt_insert(ncells, r, seed, keys)
    count = np.zeros(ncells, np.int64)
    ks = [0] * ncells
    hs = [0] * ncells
    for x in keys.tolist():
        cells, c = _cells_of(ncells, r, seed, int(x))
        for cell in cells:
            count[cell] += 1
            ks[cell] ^= int(x)
            hs[cell] ^= c
    assert np.array_equal(t.count.astype(np.int64), count)
    assert t.key_sum.tolist() == ks and t.hash_sum.tolist() == hs
