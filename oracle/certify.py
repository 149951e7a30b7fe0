"""Checks that hold for any size (test infrastructure only).

``peel_certificate`` verifies, with vectorised numpy, that a claimed result of
round-synchronous peeling is *the* result.  Write vr(v) for the round that
removed v (infinity for a core vertex) and er(e) for the round that removed e.
The process of Section 1 / Section 3 is characterised by three facts:

  1. an edge dies in the first round that removes one of its vertices:
     er(e) = min over e's slots of vr;
  2. the degree of v at the start of round t is
     d_t(v) = #{incidences (e, v) : er(e) >= t}, non-increasing in t;
  3. a vertex is removed in the first round whose start degree is below k:
     vr(v) = min{t >= 1 : d_t(v) < k}, i.e. d_{vr}(v) < k and, for vr >= 2,
     d_{vr-1}(v) >= k; a core vertex has d_inf(v) >= k.

By induction on t, (1)-(3) determine vr and er uniquely, so an output that
satisfies them equals the process's output.  The final degree of a core vertex
is d_inf(v); a removed vertex ends at 0.
"""
from __future__ import annotations

import numpy as np

INF = np.int64(1) << 40


def _inf(a) -> np.ndarray:
    a = np.asarray(a).astype(np.int64)
    return np.where(a == 0, INF, a)


def peel_certificate(n: int, edges, k: int, vertex_round, edge_round, deg=None,
                     V=None, E=None, rounds=None, edge_rounds=None) -> list[str]:
    """Return the list of violated facts (empty when the result is the k-core peel)."""
    bad: list[str] = []
    e = np.asarray(edges)
    m, r = e.shape
    vr = _inf(vertex_round)
    er = _inf(edge_round)
    if vr.shape != (n,) or er.shape != (m,):
        return ["shape"]
    if m:
        er_expect = vr[e].min(axis=1)
        if not np.array_equal(er, er_expect):
            bad.append(f"edge rounds: {int((er != er_expect).sum())} edges differ from min vertex round")
    flat_v = e.ravel().astype(np.int64)
    flat_er = np.repeat(er, r)
    tv = vr[flat_v]
    d_now = np.bincount(flat_v, weights=(flat_er >= tv), minlength=n)
    d_prev = np.bincount(flat_v, weights=(flat_er >= tv - 1), minlength=n)
    removed = vr < INF
    if (d_now[removed] >= k).any():
        bad.append(f"{int((d_now[removed] >= k).sum())} removed vertices had start degree >= k")
    late = removed & (vr >= 2)
    if (d_prev[late] < k).any():
        bad.append(f"{int((d_prev[late] < k).sum())} vertices should have gone a round earlier")
    if (d_now[~removed] < k).any():
        bad.append(f"{int((d_now[~removed] < k).sum())} core vertices have core degree < k")
    if deg is not None:
        want = np.where(removed, 0, d_now).astype(np.int64)
        if not np.array_equal(np.asarray(deg).astype(np.int64), want):
            bad.append("final degrees")
    last_v = int(vr[removed].max()) if removed.any() else 0
    finite_e = er[er < INF]
    last_e = int(finite_e.max()) if finite_e.size else 0
    if V is not None:
        want = np.bincount(vr[removed], minlength=last_v + 1)[1:]
        if not np.array_equal(np.asarray(V).astype(np.int64), want):
            bad.append("per-round vertex counts")
    if E is not None:
        want = np.bincount(finite_e, minlength=last_v + 1)[1:]
        if not np.array_equal(np.asarray(E).astype(np.int64)[: want.size], want):
            bad.append("per-round edge counts")
    if rounds is not None and int(rounds) != last_v:
        bad.append(f"rounds {rounds} != {last_v}")
    if edge_rounds is not None and int(edge_rounds) != last_e:
        bad.append(f"edge rounds {edge_rounds} != {last_e}")
    return bad
