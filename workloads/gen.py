"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module only *draws inputs*: hypergraph edge lists and distinct 64-bit keys.
It holds none of the peeling or IBLT arithmetic; the CPU oracle and the HIP
library each implement that on their own.

Random numbers come from SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw ``i`` of stream ``seed`` is the SplitMix64 finaliser applied to
``seed + (i + 1) * 0x9e3779b97f4a7c15`` (the (i+1)-th output of a SplitMix64
state initialised to ``seed``).  An integer in ``[0, s)`` is taken from a
64-bit draw ``u`` by the multiply-shift map ``floor(u * s / 2^64)`` (Lemire,
"Fast random integer generation in an interval", ACM TOMACS 2019).

Two hypergraph models from the paper are provided:

* ``partitioned_edges`` -- the vertex set is split into ``r`` near-equal
  subtables and every edge takes one uniform vertex from each subtable
  (the partitioned model of Appendix B, "Parallel Peeling with Subtables",
  which is also the IBLT's layout in Section 5).
* ``gnm_edges`` -- G^r_{n,cn}: ``m`` edges, each a set of ``r`` distinct
  uniform vertices (Section 2, "Preliminaries").  A slot that repeats an
  earlier vertex of its edge is redrawn from the edge's next counter values.
"""
from __future__ import annotations

import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_C1 = np.uint64(0xBF58476D1CE4E5B9)
_C2 = np.uint64(0x94D049BB133111EB)
_MASK32 = np.uint64(0xFFFFFFFF)

# Independent streams for the different draws a workload makes from one seed.
_DOMAIN_EDGE = 0x243F6A8885A308D3
_DOMAIN_KEY = 0x13198A2E03707344
_DOMAIN_TABLE = 0xA4093822299F31D0
_DOMAIN_GNM = 0x082EFA98EC4E6C89

_CHUNK = 1 << 22


def _u64(x) -> np.uint64:
    return np.uint64(int(x) & 0xFFFFFFFFFFFFFFFF)


def mix64(z: np.ndarray) -> np.ndarray:
    """SplitMix64 output finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _C1
        z = (z ^ (z >> np.uint64(27))) * _C2
    return z ^ (z >> np.uint64(31))


def splitmix64(seed: int, idx: np.ndarray) -> np.ndarray:
    """Draw ``idx`` (uint64 array) of the SplitMix64 stream seeded with ``seed``."""
    idx = np.asarray(idx, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = _u64(seed) + (idx + np.uint64(1)) * GOLDEN
    return mix64(state)


def mulhi_reduce(u: np.ndarray, s) -> np.ndarray:
    """floor(u * s / 2^64) for uint64 ``u`` and 0 < s < 2^32, exactly."""
    u = np.asarray(u, dtype=np.uint64)
    s = np.asarray(s, dtype=np.uint64)
    hi = u >> np.uint64(32)
    lo = u & _MASK32
    # u*s = hi*s*2^32 + lo*s; both partial products fit in 64 bits for s < 2^32.
    return (hi * s + ((lo * s) >> np.uint64(32))) >> np.uint64(32)


def stream_seed(seed: int, domain: int) -> int:
    """A 64-bit stream seed for one kind of draw of a workload seed."""
    return int(splitmix64(seed ^ domain, np.zeros(1, np.uint64))[0])


def subtable_sizes(n: int, r: int) -> list[int]:
    """Near-equal split of ``n`` ids into ``r`` subtables (the first n mod r get one more)."""
    q, rem = divmod(n, r)
    return [q + (1 if j < rem else 0) for j in range(r)]


def subtable_bases(n: int, r: int) -> list[int]:
    out, acc = [], 0
    for s in subtable_sizes(n, r):
        out.append(acc)
        acc += s
    return out


def partitioned_edges(n: int, m: int, r: int, seed: int) -> np.ndarray:
    """``m`` edges, slot ``j`` of edge ``i`` uniform in subtable ``j``; returns (m, r) uint32."""
    if not (2 <= r <= 8) or n < r:
        raise ValueError("need 2 <= r <= 8 and n >= r")
    sizes = np.array(subtable_sizes(n, r), dtype=np.uint64)
    bases = np.array(subtable_bases(n, r), dtype=np.uint64)
    st = stream_seed(seed, _DOMAIN_EDGE)
    out = np.empty((m, r), dtype=np.uint32)
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        idx = np.arange(lo * r, hi * r, dtype=np.uint64)
        u = splitmix64(st, idx).reshape(hi - lo, r)
        v = bases[None, :] + mulhi_reduce(u, sizes[None, :])
        out[lo:hi] = v.astype(np.uint32)
    return out


def gnm_edges(n: int, m: int, r: int, seed: int) -> np.ndarray:
    """G^r_{n,cn}: ``m`` edges of ``r`` distinct uniform vertices; returns (m, r) uint32.

    Edge ``i`` owns the stream ``splitmix64(edge_seed, i)``; its slot draws are
    that stream's values 0, 1, 2, ... taken in order, skipping any vertex the
    edge already holds.
    """
    if not (2 <= r <= 8) or n < r:
        raise ValueError("need 2 <= r <= 8 and n >= r")
    st = stream_seed(seed, _DOMAIN_GNM)
    out = np.empty((m, r), dtype=np.uint32)
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        cnt = hi - lo
        eseed = splitmix64(st, np.arange(lo, hi, dtype=np.uint64))
        rows = np.empty((cnt, r), dtype=np.uint64)
        nxt = np.zeros(cnt, dtype=np.uint64)  # next draw index per edge
        for j in range(r):
            todo = np.arange(cnt)
            while todo.size:
                with np.errstate(over="ignore"):
                    state = eseed[todo] + (nxt[todo] + np.uint64(1)) * GOLDEN
                cand = mulhi_reduce(mix64(state), n)
                nxt[todo] += np.uint64(1)
                clash = np.zeros(todo.size, dtype=bool)
                for h in range(j):
                    clash |= rows[todo, h] == cand
                rows[todo[~clash], j] = cand[~clash]
                todo = todo[clash]
        out[lo:hi] = rows.astype(np.uint32)
    return out


def distinct_keys(m: int, seed: int) -> np.ndarray:
    """``m`` distinct uint64 keys: draws 0..m-1 of one SplitMix64 stream.

    Distinct because the finaliser is a bijection of 64-bit words and the
    states ``seed + (i+1)*golden`` are distinct for i < 2^64 (golden is odd).
    """
    st = stream_seed(seed, _DOMAIN_KEY)
    out = np.empty(m, dtype=np.uint64)
    for lo in range(0, m, _CHUNK):
        hi = min(m, lo + _CHUNK)
        out[lo:hi] = splitmix64(st, np.arange(lo, hi, dtype=np.uint64))
    return out


def table_seed(seed: int) -> int:
    """The hash-family seed an IBLT built for workload ``seed`` is given."""
    return stream_seed(seed, _DOMAIN_TABLE)


def _i64(x: int) -> int:
    """The int64 with the same bits as the 64-bit word x."""
    x &= 0xFFFFFFFFFFFFFFFF
    return x - (1 << 64) if x >> 63 else x


def _srl(z, k: int):
    """Logical right shift of an int64 torch tensor (bits as uint64)."""
    return (z >> k) & ((1 << (64 - k)) - 1)


def distinct_keys_torch(m: int, seed: int, device):
    """``distinct_keys(m, seed)`` computed with torch on ``device`` (int64 tensor of the
    same bits), for harnesses that must not spend host time on key generation."""
    import torch
    st = stream_seed(seed, _DOMAIN_KEY)
    z = torch.arange(1, m + 1, dtype=torch.int64, device=device)
    z = z * _i64(int(GOLDEN)) + _i64(st)
    z = (z ^ _srl(z, 30)) * _i64(int(_C1))
    z = (z ^ _srl(z, 27)) * _i64(int(_C2))
    return z ^ _srl(z, 31)
