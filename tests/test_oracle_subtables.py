"""Pins of the oracle's peeling with subtables (Appendix B), no GPU.

- a from-scratch Python restatement gives identical subround outputs on tiny inputs;
- the process ends at the k-core (the core does not depend on the removal
  order, Section 1), bit for bit against the round-synchronous simulator;
- it takes at most r times as many subrounds as the plain process takes rounds
  (Appendix B, "Simulations with Subtables");
- the vertices left after each subround match the experiment column of the
  paper's Table 4, and the mean subround counts match Table 3.
"""
import os

import numpy as np

from oracle import naive, native
from workloads import gen

HERE = os.path.dirname(os.path.abspath(__file__))


def _tiny_cases(count, seed=5):
    rng = np.random.default_rng(seed)
    for _ in range(count):
        r = int(rng.integers(2, 5))
        n = int(rng.integers(r, 24))
        m = int(rng.integers(0, 2 * n))
        k = int(rng.integers(1, 4))
        yield n, r, k, rng.integers(0, n, size=(m, r)).astype(np.uint32)


def test_subrounds_match_naive_restatement():
    for n, r, k, e in _tiny_cases(200):
        res = native.peel_subrounds(n, e, k)
        vr, er, V, E = naive.peel_subrounds_naive(n, e, k, r)
        assert res.vertex_round.tolist() == vr, (n, r, k, e)
        assert res.edge_round.tolist() == er
        assert res.V.tolist() == V and res.E.tolist() == E
        assert res.rounds == len(V)


def test_subrounds_end_at_the_k_core():
    n = (1 << 14) + 333
    for r, k, c, model in [(4, 2, 0.7, "p"), (4, 2, 0.85, "p"), (3, 2, 0.9, "g"),
                           (3, 3, 1.7, "p"), (5, 2, 0.6, "g"), (2, 3, 1.2, "p")]:
        fn = gen.partitioned_edges if model == "p" else gen.gnm_edges
        e = fn(n, int(c * n), r, 3)
        sub = native.peel_subrounds(n, e, k)
        rnd = native.peel_rounds(n, e, k)
        assert np.array_equal(sub.vertex_round == 0, rnd.vertex_round == 0)
        assert np.array_equal(sub.edge_round == 0, rnd.edge_round == 0)
        assert np.array_equal(sub.deg, rnd.deg)
        # every vertex leaves in a subround of its own subtable
        lo = np.cumsum([0] + [n // r + (1 if j < n % r else 0) for j in range(r)])
        sub_of = np.searchsorted(lo, np.arange(n), side="right") - 1
        gone = sub.vertex_round != 0
        assert np.array_equal((sub.vertex_round[gone] - 1) % r, sub_of[gone])
        # an edge leaves with the first of its vertices to leave
        vr = sub.vertex_round[e.astype(np.int64)].astype(np.int64)
        vr[vr == 0] = 1 << 40
        first = vr.min(axis=1)
        first[first == 1 << 40] = 0
        assert np.array_equal(sub.edge_round, first)
        assert sub.rounds <= r * rnd.rounds


def _golden(name):
    rows = []
    with open(os.path.join(HERE, "golden", name)) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_table4_vertices_left_after_each_subround():
    # n = 10^6, r = 4, k = 2, c = 0.7, subtables: the paper's experiment column
    # (1000 trials) against the mean of 6 trials, within 5 standard errors
    n, r = 1_000_000, 4
    rows = _golden("table4.txt")
    left = []
    for seed in range(6):
        e = gen.partitioned_edges(n, int(0.7 * n), r, 100 + seed)
        res = native.peel_subrounds(n, e, 2)
        V = np.zeros(len(rows), np.int64)
        V[: min(len(rows), res.V.size)] = res.V[: len(rows)]
        left.append(n - np.cumsum(V))
    left = np.array(left, dtype=np.float64)
    mean = left.mean(axis=0)
    se = left.std(axis=0, ddof=1) / np.sqrt(left.shape[0])
    for s, (i, j, _pred, exp) in enumerate(rows):
        assert (int(i) - 1) * r + int(j) == s + 1
        assert abs(mean[s] - float(exp)) <= 5 * se[s] + 1.0, (i, j, mean[s], exp, se[s])


def test_table3_mean_subrounds():
    # r = 4, k = 2, subtables: mean subround count over 300 trials against the
    # paper's 1000-trial means at n = 10^4 and 4 * 10^4
    want = {}
    for row in _golden("table3.txt"):
        want[int(row[0])] = (float(row[2]), float(row[4]))
    for n in (10_000, 40_000):
        for col, c in enumerate((0.7, 0.75)):
            counts = []
            for seed in range(300):
                e = gen.partitioned_edges(n, int(round(c * n)), 4, 7000 + seed)
                res = native.peel_subrounds(n, e, 2)
                assert res.vertex_round.all()  # below threshold: empty core
                counts.append(res.rounds)
            counts = np.array(counts, dtype=np.float64)
            se = counts.std(ddof=1) / np.sqrt(counts.size)
            assert abs(counts.mean() - want[n][col]) <= 5 * se + 0.05, (n, c, counts.mean())
