"""Pins for the oracle's peeling routines (paper, Sections 1, 3 and 5).

The round-synchronous simulator is checked against things other than itself:
exhaustive search for the k-core on tiny hypergraphs, the sequential process in
random orders (the core does not depend on the order, Section 1), a from-scratch
pure-Python restatement, the uniqueness certificate, and the paper's printed
simulation results (Tables 1 and 2).
"""
import numpy as np
import pytest

from oracle import certify, naive, native
from workloads import gen


def _tiny_cases(count=300):
    rng = np.random.default_rng(20130228)
    for i in range(count):
        r = int(rng.integers(2, 5))
        k = int(rng.integers(1, 4))
        n = int(rng.integers(r, 12))
        m = int(rng.integers(0, 15))
        if i % 3 == 0:
            # allow repeated ids inside an edge (degree counts multiplicity)
            e = rng.integers(0, n, size=(m, r))
        else:
            e = np.array([rng.choice(n, size=r, replace=False) for _ in range(m)]).reshape(m, r)
        yield n, k, e.astype(np.uint32)
    # degenerate shapes
    yield 5, 2, np.zeros((0, 3), np.uint32)                              # no edges
    yield 4, 1, np.array([[0, 1, 2]], np.uint32)                         # k = 1
    yield 7, 2, np.array([[0, 1, 2], [0, 3, 4], [0, 5, 6]], np.uint32)   # star
    yield 3, 2, np.array([[0, 1, 2], [0, 1, 2]], np.uint32)              # duplicate edge: 2-core
    yield 3, 5, np.array([[0, 1, 2], [0, 1, 2]], np.uint32)              # k above every degree
    yield 4, 3, np.array([[0, 1], [0, 1], [0, 1], [2, 3]], np.uint32)    # r = 2, k = 3


def test_splitmix64_known_answers():
    # Published SplitMix64 outputs for state 1234567 (first five draws).
    want = [6457827717110365317, 3203168211198807973, 9817491932198370423,
            4593380528125082431, 16408922859458223821]
    assert [native.splitmix64(1234567, i) for i in range(5)] == want
    got = gen.splitmix64(1234567, np.arange(5, dtype=np.uint64))
    assert [int(x) for x in got] == want


def test_core_matches_brute_force_and_queue_orders():
    for n, k, e in _tiny_cases():
        bv, be = native.core_brute(n, e, k)
        res = native.peel_rounds(n, e, k)
        assert np.array_equal(res.vertex_round == 0, bv), (n, k, e)
        assert np.array_equal(res.edge_round == 0, be), (n, k, e)
        for seed in (0, 1, 2, 3):
            qv, qe = native.peel_queue(n, e, k, order_seed=seed)
            assert np.array_equal(qv, bv) and np.array_equal(qe, be)


def test_rounds_match_naive_restatement():
    for n, k, e in _tiny_cases(150):
        res = native.peel_rounds(n, e, k)
        vr, er, V, E = naive.peel_rounds_naive(n, e, k)
        assert res.vertex_round.tolist() == vr
        assert res.edge_round.tolist() == er
        assert res.V.tolist() == V and res.E.tolist() == E
        assert res.rounds == len(V)


def test_certificate_accepts_oracle_and_rejects_planted_mistakes():
    n = 1 << 14
    for r, k, c in [(3, 2, 0.7), (4, 2, 0.85), (3, 3, 1.7), (2, 3, 1.0)]:
        e = gen.partitioned_edges(n, int(c * n), r, seed=7)
        res = native.peel_rounds(n, e, k)
        assert certify.peel_certificate(n, e, k, res.vertex_round, res.edge_round, res.deg,
                                        res.V, res.E, res.rounds, res.edge_rounds) == []
        # plant mistakes in copies of the oracle's output
        vr = res.vertex_round.copy()
        v = int(np.flatnonzero(vr > 1)[0])
        vr[v] -= 1
        assert certify.peel_certificate(n, e, k, vr, res.edge_round) != []
        er = res.edge_round.copy()
        j = int(np.flatnonzero(er > 0)[0])
        er[j] += 1
        assert certify.peel_certificate(n, e, k, res.vertex_round, er) != []
        d = res.deg.copy()
        d[int(np.flatnonzero(res.vertex_round == 0)[0]) if (res.vertex_round == 0).any() else 0] += 1
        assert certify.peel_certificate(n, e, k, res.vertex_round, res.edge_round, d) != []


def test_first_round_removes_low_degree_vertices():
    n = 1 << 15
    e = gen.partitioned_edges(n, int(0.7 * n), 4, seed=3)
    deg0 = np.bincount(e.ravel(), minlength=n)
    res = native.peel_rounds(n, e, 2)
    assert res.V[0] == int((deg0 < 2).sum())
    assert np.array_equal(res.vertex_round == 1, deg0 < 2)
    # final degree: 0 for removed vertices; every removed vertex had < k at its round
    assert (res.deg[res.vertex_round > 0] == 0).all()


def test_max_rounds_stops_early_with_consistent_prefix():
    n = 1 << 14
    e = gen.partitioned_edges(n, int(0.7 * n), 4, seed=5)
    full = native.peel_rounds(n, e, 2)
    part = native.peel_rounds(n, e, 2, max_rounds=4)
    assert full.rounds > 4 and part.status == native.EROUNDS
    assert np.array_equal(part.V, full.V[:4])
    assert np.array_equal(np.minimum(full.vertex_round, 5) * (full.vertex_round <= 4),
                          part.vertex_round)


def _mean_rounds(n, c, trials, seed0):
    rounds, failed = [], 0
    for s in range(trials):
        e = gen.gnm_edges(n, int(round(c * n)), 4, seed=seed0 + s)
        res = native.peel_rounds(n, e, 2)
        rounds.append(res.rounds)
        failed += int((res.vertex_round == 0).any())
    return float(np.mean(rounds)), float(np.std(rounds)), failed


@pytest.mark.slow
@pytest.mark.parametrize("c,col", [(0.70, 2), (0.75, 4), (0.80, 6), (0.85, 8)])
def test_table1_mean_rounds_n10000(golden, c, col):
    # Table 1, n = 10^4: mean rounds over 1000 trials and the count of failures.
    row = golden("table1.txt")[0]
    trials = 200
    mean, std, failed = _mean_rounds(10000, c, trials, seed0=1000)
    se = max(std, 0.3) / np.sqrt(trials)
    assert abs(mean - row[col]) < 4 * se + 0.02, (c, mean, row[col])
    assert failed == (trials if row[col - 1] == 1000 else 0)


@pytest.mark.slow
def test_table1_growth_below_vs_above_threshold():
    # Below c*: rounds barely move with n (Theorem 1); above c*: they grow like log n (Theorem 3).
    lo_small, _, _ = _mean_rounds(10000, 0.70, 20, 50)
    lo_big, _, _ = _mean_rounds(640000, 0.70, 3, 60)
    hi_small, _, _ = _mean_rounds(10000, 0.85, 20, 70)
    hi_big, _, _ = _mean_rounds(640000, 0.85, 3, 80)
    assert lo_big - lo_small < 1.5
    # Table 1 at c = 0.85: 10.773 -> 17.334 over six doublings
    assert 4.5 < hi_big - hi_small < 8.5


@pytest.mark.slow
def test_table2_experiment_column_c070(golden):
    # Table 2, c = 0.7, n = 10^6: mean vertices left after each round (experiment column).
    # Trial-to-trial spread peaks mid-run (a few thousand vertices), so the band is
    # five standard errors of the sample mean.
    rows = golden("table2.txt")
    n, trials = 10 ** 6, 6
    left = np.zeros((trials, 20))
    for s in range(trials):
        e = gen.gnm_edges(n, int(0.7 * n), 4, seed=900 + s)
        res = native.peel_rounds(n, e, 2)
        rem = n - np.cumsum(res.V.astype(np.int64))
        left[s, : rem.size] = rem
        left[s, rem.size:] = rem[-1] if rem.size else n
    mean = left.mean(axis=0)
    sd = left.std(axis=0, ddof=1)
    for t, _, exp70, _, _ in rows:
        t = int(t)
        tol = 5 * max(sd[t - 1], 3.0) / np.sqrt(trials) + 2
        assert abs(mean[t - 1] - exp70) < tol, (t, mean[t - 1], exp70, tol)
    # the run ends after round 13 in every trial, as in Table 2
    assert (left[:, 12] == 0).all() and (left[:, 11] > 0).all()
