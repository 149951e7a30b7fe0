"""Pure-Python restatements for tiny inputs (test infrastructure only).

These recompute everything from scratch each round, with no incidence lists
and no incremental degrees, so they share no structure with the C oracle.
"""
from __future__ import annotations


def peel_rounds_naive(n: int, edges, k: int):
    """Round-synchronous peel (Section 1; Section 3) by full recomputation each round.

    Returns (vertex_round, edge_round, V, E) as Python lists; 0 = in the core.
    """
    edges = [tuple(int(x) for x in row) for row in edges]
    m = len(edges)
    vr = [0] * n
    er = [0] * m
    V, E = [], []
    t = 0
    while True:
        t += 1
        deg = [0] * n
        for i, row in enumerate(edges):
            if er[i] == 0:
                for u in row:
                    deg[u] += 1
        frontier = [v for v in range(n) if vr[v] == 0 and deg[v] < k]
        if not frontier:
            break
        for v in frontier:
            vr[v] = t
        dead = 0
        for i, row in enumerate(edges):
            if er[i] == 0 and any(vr[u] == t for u in row):
                er[i] = t
                dead += 1
        V.append(len(frontier))
        E.append(dead)
    return vr, er, V, E


def peel_subrounds_naive(n: int, edges, k: int, r: int):
    """Peeling with subtables (Appendix B) by full recomputation each subround.

    Subtable j holds the ids [lo_j, lo_{j+1}) of a near-equal split of 0..n-1 (the
    first n mod r one larger).  Subround s = (i-1) r + j + 1 removes the alive
    vertices of subtable j whose degree is below k at its start.  Stops after r
    empty subrounds in a row.  Returns (vertex_round, edge_round, V, E) with V, E
    listed up to the last subround that removed a vertex.
    """
    edges = [tuple(int(x) for x in row) for row in edges]
    m = len(edges)
    bounds = [0]
    for j in range(r):
        bounds.append(bounds[-1] + n // r + (1 if j < n % r else 0))
    vr = [0] * n
    er = [0] * m
    V, E = [], []
    s, empty = 0, 0
    while empty < r:
        s += 1
        j = (s - 1) % r
        deg = [0] * n
        for i, row in enumerate(edges):
            if er[i] == 0:
                for u in row:
                    deg[u] += 1
        frontier = [v for v in range(bounds[j], bounds[j + 1]) if vr[v] == 0 and deg[v] < k]
        if not frontier:
            empty += 1
            V.append(0)
            E.append(0)
            continue
        empty = 0
        for v in frontier:
            vr[v] = s
        dead = 0
        for i, row in enumerate(edges):
            if er[i] == 0 and any(vr[u] == s for u in row):
                er[i] = s
                dead += 1
        V.append(len(frontier))
        E.append(dead)
    last = max([i + 1 for i, x in enumerate(V) if x], default=0)
    return vr, er, V[:last], E[:last]
