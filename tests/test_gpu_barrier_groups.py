"""The persistent kernels with every device-wide barrier in slot groups.

From its second barrier on, a run groups the barrier's arrivals by XCD, after
a census taken in the first barrier; when the census does not count the whole
team (a workgroup on an XCD past 7, say) every barrier keeps the slot groups
of the first.  PEEL_BARRIER=slots takes that path on purpose.  Each case is
compared with the oracle exactly as in the other parity tests.
"""
import numpy as np
import pytest

from oracle import native
from workloads import configs, gen

from gpu_helpers import gpu_peel, gpu_peel_xor, need_gpu, say
from test_gpu_iblt import check_list

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def slot_groups(monkeypatch):
    monkeypatch.setenv("PEEL_BARRIER", "slots")
    monkeypatch.delenv("PEEL_LIST_ENGINE", raising=False)
    monkeypatch.delenv("PEEL_ROUNDS", raising=False)
    monkeypatch.delenv("PEEL_CLAIMS", raising=False)


def _check_peel(n, e, k, res):
    o = native.peel_rounds(n, e, k)
    assert res["flags"] == 0
    assert np.array_equal(res["vertex_round"], o.vertex_round)
    assert np.array_equal(res["edge_round"], o.edge_round)
    assert np.array_equal(res["deg"], o.deg)
    assert np.array_equal(res["V"], o.V) and np.array_equal(res["E"], o.E)


@pytest.mark.parametrize("subtables", [False, True])
def test_peel_full_size(subtables):
    need_gpu()
    spec = configs.kcore_sweep(0.70)
    e = spec.edges(1)
    say("slot groups: peel", spec.name, "subtables", subtables)
    res = gpu_peel(spec.n, e, spec.k, subtables=subtables)
    if subtables:
        o = native.peel_subrounds(spec.n, e, spec.k)
        assert res["flags"] == 0
        assert np.array_equal(res["vertex_round"], o.vertex_round)
        assert np.array_equal(res["edge_round"], o.edge_round)
    else:
        _check_peel(spec.n, e, spec.k, res)


def test_peel_xor_medium():
    need_gpu()
    n = (1 << 20) + 333
    e = gen.partitioned_edges(n, int(0.75 * n), 4, 7)
    say("slot groups: xor peel", n)
    res = gpu_peel_xor(n, e)
    _check_peel(n, e, 2, res)


@pytest.mark.parametrize("engine", ["owner", "atomic"])
def test_list_full_size(engine, monkeypatch):
    need_gpu()
    if engine == "atomic":
        monkeypatch.setenv("PEEL_LIST_ENGINE", "atomic")
    spec = configs.iblt_main()
    keys = spec.keys(1)
    say("slot groups: list", engine)
    g, o = check_list(spec.ncells, spec.r, spec.table_seed(1), keys)
    assert g["listed"] == spec.nkeys and g["left"] == 0
