"""The seeded input generators: determinism, models and the multiply-shift map."""
import numpy as np

from oracle import theory
from workloads import configs, gen


def test_mulhi_reduce_exact():
    rng = np.random.default_rng(5)
    u = rng.integers(0, 2 ** 63, size=2000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    for s in [1, 3, 1000, 2 ** 22, 2 ** 32 - 1]:
        got = gen.mulhi_reduce(u, s)
        want = [(int(a) * s) >> 64 for a in u]
        assert got.tolist() == want


def test_partitioned_slots_stay_in_their_subtable():
    n, r = 1000, 3
    e = gen.partitioned_edges(n, 5000, r, seed=1)
    bases, sizes = gen.subtable_bases(n, r), gen.subtable_sizes(n, r)
    assert sizes == [334, 333, 333]
    for j in range(r):
        assert ((e[:, j] >= bases[j]) & (e[:, j] < bases[j] + sizes[j])).all()
    assert np.array_equal(e, gen.partitioned_edges(n, 5000, r, seed=1))
    assert not np.array_equal(e, gen.partitioned_edges(n, 5000, r, seed=2))


def test_gnm_rows_distinct_and_uniform():
    n, r, m = 50, 4, 20000
    e = gen.gnm_edges(n, m, r, seed=3)
    s = np.sort(e, axis=1)
    assert (np.diff(s, axis=1) > 0).all()
    cnt = np.bincount(e.ravel(), minlength=n)
    exp = m * r / n
    assert abs(cnt.mean() - exp) < 1e-9 and cnt.std() < 4 * np.sqrt(exp)


def test_degree_distribution_is_poisson_rc():
    # Section 3.1: a vertex's degree is close to Poisson(r c).
    n = 1 << 18
    e = gen.partitioned_edges(n, int(0.7 * n), 4, seed=9)
    deg = np.bincount(e.ravel(), minlength=n)
    for d in range(6):
        p = theory.p_at_least(d, 2.8) - theory.p_at_least(d + 1, 2.8)
        assert abs((deg == d).mean() - p) < 0.004


def test_keys_distinct():
    k = gen.distinct_keys(1 << 18, seed=4)
    assert np.unique(k).size == k.size


def test_config_sizes():
    assert configs.kcore_small().m == 45875
    assert [configs.kcore_sweep(c).m for c in configs.SWEEP_C] == [
        10066330, 11744051, 12582912, 13421773, 14260634]
    assert configs.iblt_main().nkeys == 10296982
    assert configs.kcore_k3("lo").m == 5861737 and configs.kcore_k3("hi").m == 7164345
    b = configs.batched_main().draw()
    assert len(b) == 4096
    assert all(2 ** 10 - 1 <= N <= 2 ** 20 + 1 for N, _, _, _ in b)


def test_partial_batch():
    # a seeded ~5% of the tables move above threshold (load 1.0-1.2 c*); the
    # rest are the plain batch's tables, unchanged
    main = configs.batched_main().draw()
    part = configs.batched_partial().draw()
    cs = configs.cstar(2, 3)
    hot = [i for i in range(len(main)) if main[i] != part[i]]
    assert 0.04 * len(main) <= len(hot) <= 0.06 * len(main)
    for i in hot:
        N, m, ks, ts = part[i]
        assert (N, ks, ts) == main[i][0:1] + main[i][2:]
        assert 1.0 * cs * N - 1 <= m <= 1.2 * cs * N + 1
