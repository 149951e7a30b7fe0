"""Host logic of the serving loop: the HBM-budget arena allocator."""
import numpy as np

from paper_1302_7014_amd.serve import Arena, Request


def test_arena_first_fit_and_merge():
    a = Arena(1 << 20, "cpu")
    rng = np.random.default_rng(0)
    live = []
    for step in range(2000):
        if live and (rng.random() < 0.5 or a.used > (1 << 19)):
            off, nb = live.pop(int(rng.integers(len(live))))
            a.free(off, nb)
        else:
            got = a.alloc(int(rng.integers(1, 20000)))
            if got is not None:
                live.append(got)
        # live blocks never overlap and stay inside the budget
        spans = sorted(live)
        for (o1, n1), (o2, _) in zip(spans, spans[1:]):
            assert o1 + n1 <= o2
        assert all(o % 256 == 0 and o + n <= a.budget for o, n in live)
        assert a.used == sum(n for _, n in live)
    for off, nb in live:
        a.free(off, nb)
    assert a.free_list == [(0, a.budget)] and a.used == 0
    assert a.peak <= a.budget


def test_arena_refuses_when_full():
    a = Arena(4096, "cpu")
    assert a.alloc(4096) == (0, 4096)
    assert a.alloc(1) is None
    a.free(0, 4096)
    assert a.alloc(100) == (0, 256)


def test_request_footprint():
    q = Request(0, 0.0, 3, 1000, 600, 1, 2)
    assert q.footprint(256) == sum((x + 255) // 256 * 256 for x in (32000, 8000, 4800, 2048, 64))
