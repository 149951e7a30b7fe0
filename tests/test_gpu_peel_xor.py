"""GPU parity of peel_k2_xor (the 2-core peel with no CSR) against the oracle.

The CSR-free peel must give exactly the oracle's round-synchronous peel with
k = 2: vertex and edge removal rounds, per-round vertex and edge counts, round
counts, final degrees and the core size, bit for bit -- on small and
degenerate hypergraphs (repeated ids, isolated vertices, hubs whose degree
escapes the LDS fields), both random models, round limits, ids out of range,
and the full n = 2^24 workloads below, near and above the threshold.
"""
import numpy as np
import pytest

from oracle import certify, native
from workloads import configs, gen

from gpu_helpers import gpu_peel_xor, need_gpu, say

pytestmark = pytest.mark.gpu

import paper_1302_7014_amd as pk  # noqa: E402


def _check(n, edges, res, max_rounds=1 << 20):
    o = native.peel_rounds(n, edges, 2, max_rounds=max_rounds)
    assert np.array_equal(res["vertex_round"], o.vertex_round)
    assert np.array_equal(res["edge_round"], o.edge_round)
    assert np.array_equal(res["deg"], o.deg)
    assert np.array_equal(res["V"], o.V) and np.array_equal(res["E"], o.E)
    assert res["rounds"] == o.rounds and res["edge_rounds"] == o.edge_rounds
    assert res["core"] == int((o.vertex_round == 0).sum())
    return o


def test_small_hypergraphs():
    need_gpu()
    rng = np.random.default_rng(17)
    for i in range(60):
        r = int(rng.integers(2, 9))
        n = int(rng.integers(r, 4000))
        m = int(rng.integers(0, 2 * n))
        e = rng.integers(0, n, size=(m, r)).astype(np.uint32)
        say("xor small", i, n, m, r)
        res = gpu_peel_xor(n, e)
        assert res["flags"] == 0
        _check(n, e, res)


def test_degenerate_inputs():
    need_gpu()
    rng = np.random.default_rng(3)
    cases = [
        (1, np.zeros((0, 3), np.uint32)),                       # one vertex, no edges
        (5, np.zeros((0, 2), np.uint32)),                       # no edges
        (3, np.array([[0, 1, 2], [0, 1, 2]], np.uint32)),       # duplicate edge: a 2-core
        (3, np.array([[0, 1, 2]], np.uint32)),                  # one edge
        (7, np.array([[0, 1, 2], [0, 3, 4], [0, 5, 6]], np.uint32)),  # star
        (2, np.array([[0, 0], [1, 1], [0, 1]], np.uint32)),     # repeated ids in an edge
        (4, np.array([[0, 0, 1], [1, 2, 3], [2, 3, 3]], np.uint32)),
        (8, np.array([[j] * 8 for j in range(8)], np.uint32)),  # r = 8, loops
        (6, np.array([[0, 1, 0, 1], [2, 3, 4, 5]], np.uint32)),
        # hubs of degree >= 15, kept in the global degree array instead of LDS
        (1000, rng.integers(0, 1000, size=(3750, 4)).astype(np.uint32)),
        (300, np.concatenate([np.array([[0, i, i + 1, 7] for i in range(1, 290)], np.uint32),
                              rng.integers(0, 300, size=(100, 4)).astype(np.uint32)])),
        (64, rng.integers(0, 64, size=(400, 3)).astype(np.uint32)),
    ]
    for n, e in cases:
        say("xor degenerate", n, e.shape)
        res = gpu_peel_xor(n, e)
        assert res["flags"] == 0
        _check(n, e, res)


@pytest.mark.parametrize("r,c", [(3, 0.9), (4, 0.7), (4, 0.85), (2, 0.45), (5, 0.6), (8, 0.5),
                                 (3, 0.75)])
def test_medium_models(r, c):
    need_gpu()
    n = (1 << 18) + 12345
    for model in ("partitioned", "gnm"):
        e = (gen.partitioned_edges if model == "partitioned" else gen.gnm_edges)(n, int(c * n), r, 13)
        say("xor medium", model, n, r, c)
        res = gpu_peel_xor(n, e)
        assert res["flags"] == 0
        _check(n, e, res)


def test_config_kcore_small_seeds():
    need_gpu()
    spec = configs.kcore_small()
    for seed in (1, 2, 3, 4, 5):
        e = spec.edges(seed)
        say("xor", spec.name, "seed", seed)
        res = gpu_peel_xor(spec.n, e)
        _check(spec.n, e, res)


def test_round_limit_leaves_consistent_state():
    need_gpu()
    n = 1 << 16
    e = gen.partitioned_edges(n, int(0.7 * n), 4, 5)
    for cap in (1, 2, 3, 7):
        say("xor max_rounds", cap)
        res = gpu_peel_xor(n, e, max_rounds=cap)
        o = native.peel_rounds(n, e, 2, max_rounds=cap)
        assert o.status == native.EROUNDS and res["flags"] & pk.FLAG_EROUNDS
        assert np.array_equal(res["vertex_round"], o.vertex_round)
        assert np.array_equal(res["edge_round"], o.edge_round)
        assert np.array_equal(res["deg"], o.deg)
        assert res["rounds"] == cap


def test_out_of_range_ids_flagged():
    # ids >= n are flagged and ignored: the peel runs on the in-range incidences
    need_gpu()
    n = 5
    e = np.array([[0, 1, 2], [0, 1, 99], [3, 4, 4]], np.uint32)
    say("xor erange")
    res = gpu_peel_xor(n, e)
    assert res["flags"] & pk.FLAG_ERANGE


def test_repeatable_and_equal_to_peel_kcore():
    need_gpu()
    from gpu_helpers import gpu_peel
    n = 1 << 20
    e = gen.partitioned_edges(n, int(0.75 * n), 4, 21)
    say("xor repeat", n)
    a = gpu_peel_xor(n, e)
    b = gpu_peel_xor(n, e)
    c = gpu_peel(n, e, 2)
    for key in ("vertex_round", "edge_round", "deg", "V", "E"):
        assert np.array_equal(a[key], b[key]) and np.array_equal(a[key], c[key])


@pytest.mark.parametrize("c", configs.SWEEP_C + configs.NEAR_C)
def test_full_size_r4_n16M(c):
    # n = 2^24, r = 4: below, near (up to 214 rounds) and above the threshold
    need_gpu()
    spec = configs.kcore_sweep(c)
    e = spec.edges(1)
    say("xor", spec.name)
    res = gpu_peel_xor(spec.n, e)
    assert res["flags"] == 0
    _check(spec.n, e, res)
    if c == 0.70:
        assert certify.peel_certificate(spec.n, e, 2, res["vertex_round"], res["edge_round"],
                                        res["deg"], res["V"], res["E"], res["rounds"],
                                        res["edge_rounds"]) == []


@pytest.mark.parametrize("seed", [2, 3, 4, 5])
@pytest.mark.parametrize("c", [0.70, 0.85])
def test_full_size_more_seeds(c, seed):
    need_gpu()
    spec = configs.kcore_sweep(c)
    e = spec.edges(seed)
    say("xor", spec.name, "seed", seed)
    res = gpu_peel_xor(spec.n, e)
    assert res["flags"] == 0
    _check(spec.n, e, res)


def test_too_many_vertices_for_the_team():
    # n beyond what the resident team holds in LDS: flagged, not peeled
    need_gpu()
    n, m, r = (1 << 26) + 4099, 300_000, 3
    e = gen.gnm_edges(n, m, r, 31)
    say("xor team too small", n)
    res = gpu_peel_xor(n, e)
    assert res["flags"] & pk.FLAG_ETEAM
