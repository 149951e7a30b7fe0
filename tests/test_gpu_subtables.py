"""GPU parity of peel_kcore_subtables (peeling with subtables, Appendix B)
against the oracle's subround simulator, bit for bit: vertex and edge
subrounds, per-subround counts, subround totals, final degrees and the core."""
import numpy as np
import pytest

from oracle import native
from workloads import configs, gen

from gpu_helpers import gpu_peel, need_gpu, say

pytestmark = pytest.mark.gpu


def _check(n, e, k, res, max_rounds=1 << 20):
    o = native.peel_subrounds(n, e, k, max_rounds=max_rounds)
    assert np.array_equal(res["vertex_round"], o.vertex_round)
    assert np.array_equal(res["edge_round"], o.edge_round)
    assert np.array_equal(res["deg"], o.deg)
    assert np.array_equal(res["V"], o.V) and np.array_equal(res["E"], o.E)
    assert res["rounds"] == o.rounds and res["edge_rounds"] == o.edge_rounds
    assert res["core"] == int((o.vertex_round == 0).sum())
    return o


@pytest.fixture(params=["owner", "global"])
def engine(request, monkeypatch):
    """The owner engine (default) or the fallback global engine."""
    if request.param == "global":
        monkeypatch.setenv("PEEL_ENGINE", "global")
    else:
        monkeypatch.delenv("PEEL_ENGINE", raising=False)
    return request.param


def test_small_and_degenerate(engine):
    need_gpu()
    rng = np.random.default_rng(17)
    cases = [(1, 2, np.zeros((0, 3), np.uint32)), (5, 2, np.zeros((0, 2), np.uint32)),
             (3, 1, np.array([[0, 1, 2]], np.uint32)),
             (3, 2, np.array([[0, 1, 2], [0, 1, 2]], np.uint32)),
             (7, 2, np.array([[0, 1, 2], [0, 3, 4], [0, 5, 6]], np.uint32)),
             (2, 2, np.array([[0, 0], [1, 1], [0, 1]], np.uint32)),
             (1000, 15, np.random.default_rng(4).integers(0, 1000, size=(3750, 4)).astype(np.uint32)),
             (300, 20, np.random.default_rng(6).integers(0, 300, size=(2300, 4)).astype(np.uint32)),
             (300, 20, np.random.default_rng(7).integers(0, 300, size=(2350, 4)).astype(np.uint32))]
    for _ in range(30):
        r = int(rng.integers(2, 9))
        k = int(rng.integers(1, 5))
        n = int(rng.integers(r, 3000))
        m = int(rng.integers(0, 3 * n))
        cases.append((n, k, rng.integers(0, n, size=(m, r)).astype(np.uint32)))
    for i, (n, k, e) in enumerate(cases):
        say("subtables small", engine, i, n, e.shape, k)
        _check(n, e, k, gpu_peel(n, e, k, subtables=True))


@pytest.mark.parametrize("r,k,c", [(4, 2, 0.7), (4, 2, 0.85), (3, 2, 0.9), (3, 3, 1.7),
                                   (5, 2, 0.6), (2, 3, 1.2)])
def test_medium_models(r, k, c, engine):
    need_gpu()
    n = (1 << 18) + 12345
    for model in ("partitioned", "gnm"):
        fn = gen.partitioned_edges if model == "partitioned" else gen.gnm_edges
        e = fn(n, int(c * n), r, 23)
        say("subtables medium", engine, model, r, k, c)
        _check(n, e, k, gpu_peel(n, e, k, subtables=True))


def test_subround_limit(engine):
    need_gpu()
    n = 1 << 16
    e = gen.partitioned_edges(n, int(0.7 * n), 4, 5)
    for cap in (1, 2, 5, 13):
        say("subtables max_rounds", engine, cap)
        res = gpu_peel(n, e, 2, max_rounds=cap, subtables=True)
        o = native.peel_subrounds(n, e, 2, max_rounds=cap)
        assert o.status == native.EROUNDS and res["flags"] & 0x2
        assert np.array_equal(res["vertex_round"], o.vertex_round)
        assert np.array_equal(res["edge_round"], o.edge_round)
        assert np.array_equal(res["deg"], o.deg)
        assert res["rounds"] == o.rounds


@pytest.mark.parametrize("c", [0.70, 0.85])
def test_full_size_r4_n16M(c):
    need_gpu()
    spec = configs.kcore_sweep(c)
    e = spec.edges(1)
    say(spec.name, "subtables")
    res = gpu_peel(spec.n, e, spec.k, subtables=True)
    assert res["flags"] == 0
    o = _check(spec.n, e, spec.k, res)
    # the k-core is the one the plain rounds reach
    plain = native.peel_rounds(spec.n, e, spec.k)
    assert np.array_equal(o.vertex_round == 0, plain.vertex_round == 0)


def test_empty_subround_while_a_full_workgroup_waits():
    # Regression: one owner workgroup holds 2^16 vertices waiting for a later
    # subround (all of its range, in subtable 1) while subround 1 removes
    # nothing anywhere.  The run must go on to subround 2 and remove them.
    need_gpu()
    import torch
    T = torch.cuda.get_device_properties(0).multi_processor_count
    n, r, k = 1 << 24, 3, 2
    Vb = ((n + T - 1) // T + 31) & ~31
    base1, base2 = gen.subtable_bases(n, r)[1:3]
    s = (base1 + Vb - 1) // Vb
    assert (s + 1) * Vb <= base2
    iso = np.arange(s * Vb, (s + 1) * Vb, dtype=np.uint32)
    rest = np.setdiff1d(np.arange(n, dtype=np.uint32), iso)
    rng = np.random.default_rng(5)
    rng.shuffle(rest)
    whole = rest.size % 3 == 0
    rest = rest[: rest.size // 3 * 3].reshape(-1, 3)
    # every other vertex lies in two copies of one edge: degree 2, in the 2-core
    e = np.concatenate([rest, rest]).astype(np.uint32)
    say("subtables: empty subround, one workgroup waiting", n, e.shape, Vb)
    res = gpu_peel(n, e, k, subtables=True)
    assert res["flags"] == 0
    o = _check(n, e, k, res)
    if whole:
        assert o.rounds == 2 and (o.vertex_round[iso] == 2).all()
    if res["team"] == T:
        assert Vb == iso.size
