"""GPU parity of hg_build + peel_kcore against the CPU oracle, bit for bit.

Every comparison is exact: vertex and edge removal rounds, per-round vertex and
edge counts, round counts, final degrees and the core size.  The CSR is
compared as per-vertex sorted edge lists (the order inside a list is free).
"""
import os

import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk

from oracle import certify, native
from workloads import configs, gen

from gpu_helpers import dev_u32, gpu_peel, host_u32, need_gpu, say

pytestmark = pytest.mark.gpu


def _check_csr(n, edges, res):
    m, r = edges.shape
    deg = np.bincount(edges.ravel().astype(np.int64), minlength=n)
    assert np.array_equal(res["deg0"], deg)
    off = host_u32(res["csr"].offsets)[: n + 1].astype(np.int64)
    assert off[0] == 0 and np.array_equal(np.diff(off), deg)
    inc = host_u32(res["csr"].inc)[: m * r].astype(np.int64)
    # each vertex's list is the multiset of edges that hold it: compare the
    # sorted (vertex, edge) keys of the lists with those of the edge rows
    got = np.sort(np.repeat(np.arange(n, dtype=np.int64), deg) * max(m, 1) + inc)
    want = np.sort(edges.ravel().astype(np.int64) * max(m, 1) + np.repeat(np.arange(m), r))
    assert np.array_equal(got, want)
    assert res["info"][0] == 0 and res["info"][1] == (deg.max() if n else 0)


def _check_against_oracle(n, edges, k, res, max_rounds=1 << 20):
    o = native.peel_rounds(n, edges, k, max_rounds=max_rounds)
    assert np.array_equal(res["vertex_round"], o.vertex_round)
    assert np.array_equal(res["edge_round"], o.edge_round)
    assert np.array_equal(res["deg"], o.deg)
    assert np.array_equal(res["V"], o.V) and np.array_equal(res["E"], o.E)
    assert res["rounds"] == o.rounds and res["edge_rounds"] == o.edge_rounds
    assert res["core"] == int((o.vertex_round == 0).sum())
    return o


@pytest.fixture(params=["default", "dense", "auto", "unfiltered", "retry"])
def rounds(request, monkeypatch):
    """Which rounds the owner engine runs: the default (all sparse: claims over the
    CSR, filtered by the dead-edge nibbles), all dense (edge scan against the
    frontier bitmap), chosen per round, sparse with every incidence of a
    frontier vertex claimed (the kernel that larger vertex ranges take), or that
    kernel taking over after the claim filter's kernel declined."""
    monkeypatch.delenv("PEEL_CLAIMS", raising=False)
    if request.param == "default":
        monkeypatch.delenv("PEEL_ROUNDS", raising=False)
    elif request.param in ("unfiltered", "retry"):
        monkeypatch.delenv("PEEL_ROUNDS", raising=False)
        monkeypatch.setenv("PEEL_CLAIMS", "all" if request.param == "unfiltered" else "retry")
    else:
        monkeypatch.setenv("PEEL_ROUNDS", request.param)
    return request.param


def test_small_hypergraphs_bit_exact(rounds):
    need_gpu()
    rng = np.random.default_rng(7)
    for i in range(40):
        r = int(rng.integers(2, 9))
        k = int(rng.integers(1, 5))
        n = int(rng.integers(r, 3000))
        m = int(rng.integers(0, 3 * n))
        e = rng.integers(0, n, size=(m, r)).astype(np.uint32)
        say("small", rounds, i, n, m, r, k)
        res = gpu_peel(n, e, k)
        assert res["flags"] == 0
        _check_csr(n, e, res)
        _check_against_oracle(n, e, k, res)


def test_degenerate_inputs(rounds):
    need_gpu()
    cases = [
        (1, 2, np.zeros((0, 3), np.uint32)),                       # one vertex, no edges
        (5, 2, np.zeros((0, 2), np.uint32)),                       # no edges
        (3, 1, np.array([[0, 1, 2]], np.uint32)),                  # k = 1
        (3, 2, np.array([[0, 1, 2], [0, 1, 2]], np.uint32)),       # duplicate edge: 2-core
        (4, 9, np.array([[0, 1, 2, 3]] * 5, np.uint32)),           # k above every degree
        (7, 2, np.array([[0, 1, 2], [0, 3, 4], [0, 5, 6]], np.uint32)),  # star
        (2, 2, np.array([[0, 0], [1, 1], [0, 1]], np.uint32)),     # repeated ids in an edge
        (8, 2, np.array([[j] * 8 for j in range(8)], np.uint32)),  # r = 8, loops
        # one CSR bucket with more incidences than the build stages in LDS
        (100, 3, np.random.default_rng(3).integers(0, 100, size=(12000, 4)).astype(np.uint32)),
        # degrees and k around and above 15, where the owner engine keeps a
        # vertex's degree in the global array instead of four bits of LDS
        (1000, 15, np.random.default_rng(4).integers(0, 1000, size=(3750, 4)).astype(np.uint32)),
        (300, 16, np.random.default_rng(5).integers(0, 300, size=(1200, 4)).astype(np.uint32)),
        (300, 20, np.random.default_rng(6).integers(0, 300, size=(2300, 4)).astype(np.uint32)),
        (300, 20, np.random.default_rng(7).integers(0, 300, size=(2350, 4)).astype(np.uint32)),
    ]
    for n, k, e in cases:
        say("degenerate", rounds, n, k, e.shape)
        res = gpu_peel(n, e, k)
        _check_csr(n, e, res)
        _check_against_oracle(n, e, k, res)


@pytest.mark.parametrize("which", ["n", "m"])
def test_build_three_level_path(which):
    # just past the two-level build's limits (2048 buckets of 8192 vertices,
    # 1024 tiles of 16384 edges): the three-level build with 8-byte pairs runs
    need_gpu()
    if which == "n":
        n, m, r, k = (1 << 24) + 4099, 300000, 3, 2
    else:
        n, m, r, k = 1 << 20, (1 << 24) + 777, 2, 22  # 7 rounds, a large 22-core
    e = gen.gnm_edges(n, m, r, 41)
    say("three-level build", n, m, r)
    res = gpu_peel(n, e, k)
    assert res["flags"] == 0
    _check_csr(n, e, res)
    _check_against_oracle(n, e, k, res)


def test_global_engine_bit_exact(monkeypatch):
    # the fallback engine (CAS claims and device-atomic degrees), which runs
    # when a workgroup's vertex or edge range does not fit in LDS, forced here
    need_gpu()
    monkeypatch.setenv("PEEL_ENGINE", "global")
    rng = np.random.default_rng(29)
    for i in range(12):
        r = int(rng.integers(2, 9))
        k = int(rng.integers(1, 5))
        n = int(rng.integers(r, 3000))
        e = rng.integers(0, n, size=(int(rng.integers(0, 3 * n)), r)).astype(np.uint32)
        say("global engine small", i, n, e.shape, k)
        _check_against_oracle(n, e, k, gpu_peel(n, e, k))
    n = (1 << 18) + 12345
    for r, k, c in [(4, 2, 0.7), (4, 2, 0.85), (3, 3, 1.7)]:
        e = gen.partitioned_edges(n, int(c * n), r, 23)
        say("global engine medium", r, k, c)
        _check_against_oracle(n, e, k, gpu_peel(n, e, k))
    spec = configs.kcore_sweep(0.70)
    e = spec.edges(1)
    say("global engine", spec.name)
    res = gpu_peel(spec.n, e, spec.k)
    assert res["flags"] == 0
    _check_against_oracle(spec.n, e, spec.k, res)


def test_config_kcore_small_seeds():
    need_gpu()
    spec = configs.kcore_small()
    for seed in (1, 2, 3, 4, 5):
        e = spec.edges(seed)
        say(spec.name, "seed", seed)
        res = gpu_peel(spec.n, e, spec.k)
        _check_csr(spec.n, e, res)
        _check_against_oracle(spec.n, e, spec.k, res)


@pytest.mark.parametrize("r,k,c", [(3, 2, 0.9), (4, 2, 0.7), (4, 2, 0.85), (3, 3, 1.4),
                                   (3, 3, 1.7), (2, 3, 1.2), (5, 2, 0.6), (6, 4, 2.0)])
def test_medium_models_bit_exact(r, k, c, rounds):
    need_gpu()
    n = (1 << 18) + 12345  # several tiles and a ragged tail
    for model in ("partitioned", "gnm"):
        e = (gen.partitioned_edges if model == "partitioned" else gen.gnm_edges)(n, int(c * n), r, 11)
        say("medium", rounds, model, n, r, k, c)
        res = gpu_peel(n, e, k)
        _check_against_oracle(n, e, k, res)


@pytest.mark.parametrize("k", [2, 3])
def test_list_bounds_blocks_with_hub_vertices(rounds, k):
    # a few vertices of degree ~300 among ordinary ones: the blocks of compact
    # list bounds that hold them have more than 255 incidences and are read
    # from the offsets array, the others from their one-byte offsets
    need_gpu()
    n = (1 << 16) + 77
    rng = np.random.default_rng(12)
    e = gen.partitioned_edges(n, int(0.7 * n), 4, 13)
    hubs = rng.choice(n, 40, replace=False).astype(np.uint32)
    extra = rng.integers(0, n, size=(40 * 300, 4)).astype(np.uint32)
    extra[:, 0] = np.repeat(hubs, 300)
    e = np.concatenate([e, extra])
    say("hub vertices", rounds, n, e.shape, k)
    res = gpu_peel(n, e, k)
    assert res["flags"] == 0
    _check_against_oracle(n, e, k, res)


def test_round_limit_leaves_consistent_state(rounds):
    need_gpu()
    n = 1 << 16
    e = gen.partitioned_edges(n, int(0.7 * n), 4, 5)
    for cap in (1, 3, 7):
        say("max_rounds", rounds, cap)
        res = gpu_peel(n, e, 2, max_rounds=cap)
        o = native.peel_rounds(n, e, 2, max_rounds=cap)
        assert o.status == native.EROUNDS and res["flags"] & 0x2
        assert np.array_equal(res["vertex_round"], o.vertex_round)
        assert np.array_equal(res["edge_round"], o.edge_round)
        assert np.array_equal(res["deg"], o.deg)
        assert res["rounds"] == cap


def test_out_of_range_ids_flagged():
    need_gpu()
    e = np.array([[0, 1, 2], [0, 1, 99]], np.uint32)
    say("erange")
    csr = pk.hg_build(dev_u32(e).view(2, 3), 5)
    torch.cuda.synchronize()
    info = host_u32(csr.info)
    assert info[0] & 0x1
    # the in-range incidences still form a consistent CSR
    assert host_u32(csr.offsets)[:6].tolist() == [0, 2, 4, 5, 5, 5]


def test_repeatable_across_runs():
    # Outputs are order-independent integers: two runs agree bit for bit.
    need_gpu()
    n = 1 << 20
    e = gen.partitioned_edges(n, int(0.75 * n), 4, 21)
    say("repeat", n)
    a = gpu_peel(n, e, 2)
    b = gpu_peel(n, e, 2)
    for key in ("vertex_round", "edge_round", "deg", "V", "E"):
        assert np.array_equal(a[key], b[key])


@pytest.mark.parametrize("c", configs.SWEEP_C)
def test_full_size_sweep_r4_n16M(c):
    # n = 2^24, r = 4, k = 2: the oracle computes the whole answer on the host.
    need_gpu()
    spec = configs.kcore_sweep(c)
    e = spec.edges(1)
    say(spec.name, "rounds", os.environ.get("PEEL_ROUNDS", "default"))
    res = gpu_peel(spec.n, e, spec.k)
    assert res["flags"] == 0
    _check_against_oracle(spec.n, e, spec.k, res)
    if c == 0.70:
        assert certify.peel_certificate(spec.n, e, spec.k, res["vertex_round"], res["edge_round"],
                                        res["deg"], res["V"], res["E"], res["rounds"],
                                        res["edge_rounds"]) == []


@pytest.mark.parametrize("c", configs.NEAR_C)
def test_full_size_near_threshold(c):
    # just below c*_{2,4}: tens to hundreds of rounds (Theorem 5), bit for bit
    need_gpu()
    spec = configs.kcore_sweep(c)
    e = spec.edges(1)
    say(spec.name, "near threshold")
    res = gpu_peel(spec.n, e, spec.k)
    assert res["flags"] == 0
    _check_against_oracle(spec.n, e, spec.k, res)


@pytest.mark.parametrize("c,mode", [(0.70, "dense"), (0.85, "auto"), (0.70, "unfiltered"),
                                    (0.772, "unfiltered"), (0.70, "retry")])
def test_full_size_forced_round_kind(c, mode, monkeypatch):
    # every round of one kind at full size, sparse rounds without the claim
    # filter, and the hand-over to the kernel without it when the claim
    # filter's kernel declines (as when too small a team forms for its LDS):
    # each gives the oracle's answer
    need_gpu()
    if mode in ("unfiltered", "retry"):
        monkeypatch.setenv("PEEL_CLAIMS", "all" if mode == "unfiltered" else "retry")
    else:
        monkeypatch.setenv("PEEL_ROUNDS", mode)
    spec = configs.kcore_sweep(c)
    e = spec.edges(1)
    say(spec.name, "rounds", mode)
    res = gpu_peel(spec.n, e, spec.k)
    assert res["flags"] == 0
    _check_against_oracle(spec.n, e, spec.k, res)


@pytest.mark.parametrize("which", ["lo", "hi"])
def test_full_size_k3_n4M(which):
    need_gpu()
    spec = configs.kcore_k3(which)
    e = spec.edges(1)
    say(spec.name)
    res = gpu_peel(spec.n, e, spec.k)
    _check_against_oracle(spec.n, e, spec.k, res)


@pytest.mark.parametrize("seed", [2, 3, 4, 5])
@pytest.mark.parametrize("c", [0.70, 0.85])
def test_full_size_more_seeds(c, seed):
    # n = 2^24, r = 4, k = 2 below and above the threshold, further seeds
    need_gpu()
    spec = configs.kcore_sweep(c)
    e = spec.edges(seed)
    say(spec.name, "seed", seed)
    res = gpu_peel(spec.n, e, spec.k)
    assert res["flags"] == 0
    _check_against_oracle(spec.n, e, spec.k, res)


@pytest.mark.parametrize("seed", [2, 3, 4, 5])
@pytest.mark.parametrize("which", ["lo", "hi"])
def test_full_size_k3_more_seeds(which, seed):
    need_gpu()
    spec = configs.kcore_k3(which)
    e = spec.edges(seed)
    say(spec.name, "seed", seed)
    res = gpu_peel(spec.n, e, spec.k)
    assert res["flags"] == 0
    _check_against_oracle(spec.n, e, spec.k, res)


def test_build_atomic_path_large_n():
    # n > 2^26: hg_build takes its per-incidence atomic path, and the peel its
    # global engine (a workgroup's vertex range no longer fits in LDS).
    need_gpu()
    n, m, r = (1 << 26) + 4099, 300_000, 3
    e = gen.gnm_edges(n, m, r, 31)
    # a few vertices of high degree, and ids at both ends of the range
    e[:40, 0] = n - 1
    e[40:80, 1] = 0
    e[80:95, 2] = 12345
    say("build atomic path", n, m)
    res = gpu_peel(n, e, 2)
    assert res["flags"] == 0
    _check_csr(n, e, res)
    _check_against_oracle(n, e, 2, res)
