"""The batched listing's no-allocation entry point against iblt_list_batched.

iblt_list_batched_noalloc takes its scratch from the library's static device
array instead of a workspace.  Two calls in a row (the second on a smaller
batch, so the scratch holds the first call's leftovers) must each list every
table exactly as iblt_list_batched lists a copy of it: same summary, round
counts, per-round key sets and final cells.
"""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk
from paper_1302_7014_amd import binding
from oracle import theory
from workloads import gen

from gpu_helpers import dev_u64, host_u64, need_gpu, say

pytestmark = pytest.mark.gpu


def _batch(n, seed, hi, max_rounds):
    rng = np.random.default_rng(seed)
    specs = []
    for i in range(n):
        r = int(rng.choice((3, 4)))
        N = max(r, int(round(2 ** rng.uniform(8, hi))))
        load = rng.uniform(0.4, 1.1) * theory.cstar(2, r)[0]
        specs.append((N, r, int(load * N), 7000 * seed + i))
    specs.sort(key=lambda x: -x[0])
    a, b = [], []
    for N, r, m, s in specs:
        d = pk.iblt_desc(N, r, gen.table_seed(s))
        cells = pk.iblt_table(N, "cuda")
        if m:
            pk.iblt_insert(d, cells, dev_u64(gen.distinct_keys(m, s)))
        a.append(pk.batch_table(d, cells, max_rounds))
        b.append(pk.batch_table(d, cells.clone(), max_rounds))
    torch.cuda.synchronize()
    return a, b, max(x[0] for x in specs)


def _rounds(t):
    s = t.summary.cpu().numpy()
    K = host_u64(t.round_stats)[: int(s[1])]
    ks = host_u64(t.keys)[: int(s[0])]
    out, off = [], 0
    for kk in K.tolist():
        out.append(np.sort(ks[off: off + kk]))
        off += kk
    return s, K, out


def _same(ta, tb):
    sa, Ka, ga = _rounds(ta)
    sb, Kb, gb = _rounds(tb)
    assert np.array_equal(sa, sb)
    assert np.array_equal(Ka, Kb)
    assert all(np.array_equal(x, y) for x, y in zip(ga, gb))
    assert torch.equal(ta.cells, tb.cells)


@pytest.mark.parametrize("threads,lds", [(512, pk.IBLT_LDS_MAX_CELLS), (1024, 0)])
def test_noalloc_equals_batched_twice(threads, lds):
    need_gpu()
    maxr = 128
    for call, (n, hi) in enumerate([(600, 14), (90, 11)]):
        a, b, maxc = _batch(n, 31 + call, hi, maxr)
        assert maxc <= pk.IBLT_NOALLOC_MAX_CELLS
        say("noalloc call", call, "tables", n, "max_cells", maxc, "threads", threads, "lds", lds)
        ea = pk.batch_entries(a, "cuda")
        eb = pk.batch_entries(b, "cuda")
        torch.cuda.synchronize()
        pk.iblt_list_batched(ea, n, maxc, maxr, block_threads=threads, lds_max_cells=lds)
        sched = pk.BatchSchedule(threads, lds)
        # straight through the C ABI
        st = pk.lib().iblt_list_batched_noalloc(C.c_void_p(eb.data_ptr()), n, maxc, maxr,
                                                C.byref(sched),
                                                C.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == binding.PEEL_OK
        torch.cuda.synchronize()
        for ta, tb in zip(a, b):
            _same(ta, tb)


def test_noalloc_refuses_past_its_scratch():
    need_gpu()
    a, b, maxc = _batch(4, 41, 10, 16)
    e = pk.batch_entries(b, "cuda")
    before = [t.cells.clone() for t in b]
    torch.cuda.synchronize()
    with pytest.raises(pk.PeelError):
        pk.iblt_list_batched_noalloc(e, 4, pk.IBLT_NOALLOC_MAX_CELLS + 1, 16)
    torch.cuda.synchronize()
    assert all(torch.equal(x, t.cells) for x, t in zip(before, b))
    # and the same batch with a valid bound still lists as iblt_list_batched does
    pk.iblt_list_batched(pk.batch_entries(a, "cuda"), 4, maxc, 16)
    pk.iblt_list_batched_noalloc(e, 4, maxc, 16)
    torch.cuda.synchronize()
    for ta, tb in zip(a, b):
        _same(ta, tb)
