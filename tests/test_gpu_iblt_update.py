"""GPU parity of iblt_update (insert and delete by binning the keys per block
of cells) against the oracle and against iblt_insert / iblt_delete, cell for
cell: the counts and both sums as the oracle leaves them, and the whole 32-byte
cells, reserved words included, as the per-key atomic path leaves them."""
import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from oracle import native
from workloads import configs, gen

from gpu_helpers import dev_u64, need_gpu, say, table_to_numpy

pytestmark = pytest.mark.gpu


def _run(ncells, r, seed, keys, dels=None, reserved=False):
    d = pk.iblt_desc(ncells, r, seed)
    a = pk.iblt_table(ncells, "cuda")
    b = pk.iblt_table(ncells, "cuda")
    if reserved:
        # the update must leave the reserved words as they were
        pat = torch.arange(ncells, device="cuda", dtype=torch.int64) * 0x9E3779B97F4A7C15
        a[:, 3] = pat
        a[:, 0] = (pat >> 7) << 32
        b.copy_(a)
    pk.iblt_update(d, a, dev_u64(keys), 1)
    pk.iblt_insert(d, b, dev_u64(keys))
    if dels is not None:
        pk.iblt_update(d, a, dev_u64(dels), -1)
        pk.iblt_delete(d, b, dev_u64(dels))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    if not reserved:
        t = native.iblt_insert(ncells, r, seed, keys)
        if dels is not None:
            native.iblt_update(t, dels, sign=-1)
        count, ks, hs, ok = table_to_numpy(a)
        assert ok and np.array_equal(count, t.count)
        assert np.array_equal(ks, t.key_sum) and np.array_equal(hs, t.hash_sum)
    return a


@pytest.mark.parametrize("ncells,r,nkeys", [
    (3, 3, 1), (10, 2, 7), (1000, 3, 700), (4097, 4, 3000), ((1 << 16) + 5, 5, 40000),
    (12345, 8, 5000), (70000, 2, 60000), ((1 << 18) + 77, 3, 150000), ((1 << 20) + 4095, 4, 600000),
    ((1 << 20), 7, 100000)])
def test_update_matches_insert_and_oracle(ncells, r, nkeys):
    # one super-bucket holding several subtables up to many super-buckets with
    # a ragged last block; r from 2 to 8
    need_gpu()
    keys = gen.distinct_keys(nkeys, ncells + r)
    say("update", ncells, r, nkeys)
    _run(ncells, r, 31 + r, keys)


def test_update_deletes_and_reserved_words():
    need_gpu()
    ncells, r = (1 << 18) + 3, 3
    pool = gen.distinct_keys(180000, 5)
    a, b = pool[:120000], pool[60000:]
    say("update with deletions")
    _run(ncells, r, 77, a, dels=b)
    say("update keeps the reserved words")
    _run(ncells, r, 77, a, dels=b, reserved=True)
    say("update with no keys")
    _run(4096, 3, 5, np.zeros(0, np.uint64))
    # repeated keys (outside the insert precondition): the binned update still
    # leaves the cells exactly as the per-key atomics do
    say("update with repeated keys")
    dup = np.concatenate([pool[:50000], pool[:20000], pool[10000:15000]])
    d = pk.iblt_desc(ncells, r, 78)
    x = pk.iblt_table(ncells, "cuda")
    y = pk.iblt_table(ncells, "cuda")
    pk.iblt_update(d, x, dev_u64(dup), 1)
    pk.iblt_insert(d, y, dev_u64(dup))
    torch.cuda.synchronize()
    assert torch.equal(x, y)


def test_update_full_size():
    # 2^24 cells, r = 3, 10,296,982 keys, then the paper's r = 4 load 0.83 shape
    need_gpu()
    for spec in (configs.iblt_main(), configs.iblt_paper(4, 0.83)):
        keys = spec.keys(1)
        say(spec.name, "update")
        _run(spec.ncells, spec.r, spec.table_seed(1), keys)


def test_update_past_the_binned_limit():
    # 2^24 + 4097 cells: the per-key atomic path runs, with the same result
    need_gpu()
    ncells, r = (1 << 24) + 4097, 3
    keys = gen.distinct_keys(5000, 9)
    d = pk.iblt_desc(ncells, r, 3)
    assert pk.iblt_update_workspace(d, keys.size) == 256
    say("update past the binned limit")
    a = pk.iblt_table(ncells, "cuda")
    b = pk.iblt_table(ncells, "cuda")
    pk.iblt_update(d, a, dev_u64(keys), 1)
    pk.iblt_insert(d, b, dev_u64(keys))
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    del a, b
    torch.cuda.empty_cache()
