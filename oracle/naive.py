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
