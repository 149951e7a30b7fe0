"""The named synthetic workloads: sizes, models and seeds.

Hypergraph workloads (peeling to the k-core, Sections 1 and 3):
  * ``kcore_r3_k2_n64K``: r=3, k=2, n=2^16, m=round(0.70 n), partitioned edges.
  * ``kcore_r4_k2_n16M_c{c}``: r=4, k=2, n=2^24, c in {0.60, 0.70, 0.75, 0.80, 0.85}
    (c*_{2,4} ~ 0.7723 lies between 0.75 and 0.80), and just below the threshold
    c in {0.76, 0.77, 0.772}; partitioned edges.
  * ``kcore_r3_k3_n4M_{lo,hi}``: r=3, k=3, n=2^22 at 0.9 and 1.1 c*_{3,3}.

IBLT workloads (Section 5):
  * ``iblt_r3_N16M``: r=3 subtables over 2^24 cells, round(0.75 * 2^24 / 1.222)
    distinct keys (load ~0.614, below c*_{2,3} ~ 0.8185).
  * ``iblt_r{3,4}_N16M_load{0.75,0.83}``: the table shapes of the paper's Tables 5-6.

The thresholds come from ``manifest.json`` (written by ``make_manifest.py``).
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field

import numpy as np

from . import gen

_MANIFEST = os.path.join(os.path.dirname(os.path.abspath(__file__)), "manifest.json")


def manifest() -> dict:
    with open(_MANIFEST) as f:
        return json.load(f)


def cstar(k: int, r: int) -> float:
    return manifest()["cstar"][f"{k},{r}"]["cstar"]


@dataclass(frozen=True)
class HypergraphSpec:
    name: str
    n: int
    m: int
    r: int
    k: int
    model: str = "partitioned"  # or "gnm"
    seed: int = 1

    def edges(self, seed: int | None = None) -> np.ndarray:
        s = self.seed if seed is None else seed
        if self.model == "partitioned":
            return gen.partitioned_edges(self.n, self.m, self.r, s)
        if self.model == "gnm":
            return gen.gnm_edges(self.n, self.m, self.r, s)
        raise ValueError(self.model)


@dataclass(frozen=True)
class IbltSpec:
    name: str
    ncells: int
    nkeys: int
    r: int
    seed: int = 1

    def keys(self, seed: int | None = None) -> np.ndarray:
        return gen.distinct_keys(self.nkeys, self.seed if seed is None else seed)

    def table_seed(self, seed: int | None = None) -> int:
        return gen.table_seed(self.seed if seed is None else seed)


def kcore_small() -> HypergraphSpec:
    n = 1 << 16
    return HypergraphSpec("kcore_r3_k2_n64K", n, int(round(0.70 * n)), 3, 2)


SWEEP_C = (0.60, 0.70, 0.75, 0.80, 0.85)
# just below c*_{2,4} ~ 0.77228, where the rounds grow like 1/sqrt(c* - c) (Theorem 5)
NEAR_C = (0.76, 0.77, 0.772)


def kcore_sweep(c: float) -> HypergraphSpec:
    n = 1 << 24
    tag = f"{c:.2f}" if round(c, 2) == c else f"{c:.3f}"
    return HypergraphSpec(f"kcore_r4_k2_n16M_c{tag}", n, int(round(c * n)), 4, 2)


def kcore_k3(which: str) -> HypergraphSpec:
    d = manifest()["kcore_r3_k3_n4M"]
    key = {"lo": "m_0.9cstar", "hi": "m_1.1cstar"}[which]
    return HypergraphSpec(f"kcore_r3_k3_n4M_{which}", d["n"], d[key], 3, 3)


def iblt_main() -> IbltSpec:
    N = 1 << 24
    return IbltSpec("iblt_r3_N16M", N, int(round(0.75 * N / 1.222)), 3)


def iblt_paper(r: int, load: float) -> IbltSpec:
    N = 1 << 24
    return IbltSpec(f"iblt_r{r}_N16M_load{load:.2f}", N, int(round(load * N)), r)


@dataclass(frozen=True)
class BatchSpec:
    """Many independent IBLTs of uneven size (log-uniform cells, uniform load)."""
    name: str
    ntables: int
    r: int
    log2_lo: float
    log2_hi: float
    load_lo: float   # as a fraction of c*_{2,r}
    load_hi: float
    seed: int = 1
    tables: tuple = field(default=(), compare=False)
    hot_frac: float = 0.0  # a seeded share of tables drawn above threshold instead
    hot_lo: float = 1.0
    hot_hi: float = 1.2

    def draw(self, seed: int | None = None):
        """[(ncells, nkeys, key_seed, table_seed)] for every table."""
        s = self.seed if seed is None else seed
        st = gen.stream_seed(s, 0x452821E638D01377)
        idx = np.arange(3 * self.ntables, dtype=np.uint64)
        u = gen.splitmix64(st, idx).reshape(self.ntables, 3)
        unit = (u >> np.uint64(11)).astype(np.float64) / float(1 << 53)
        cs = cstar(2, self.r)
        if self.hot_frac > 0:
            # a stream of its own, so the other tables are those of the plain batch
            hs = gen.stream_seed(s, 0x9E3779B97F4A7C15)
            hu = gen.splitmix64(hs, np.arange(2 * self.ntables, dtype=np.uint64))
            hot = ((hu >> np.uint64(11)).astype(np.float64) / float(1 << 53)).reshape(self.ntables, 2)
        out = []
        for i in range(self.ntables):
            N = int(round(2.0 ** (self.log2_lo + (self.log2_hi - self.log2_lo) * unit[i, 0])))
            N = max(N, self.r)
            load = (self.load_lo + (self.load_hi - self.load_lo) * unit[i, 1]) * cs
            if self.hot_frac > 0 and hot[i, 0] < self.hot_frac:
                load = (self.hot_lo + (self.hot_hi - self.hot_lo) * hot[i, 1]) * cs
            m = int(round(load * N))
            kseed = int(u[i, 2])
            out.append((N, m, kseed, gen.table_seed(kseed)))
        return out


def batched_main() -> BatchSpec:
    return BatchSpec("iblt_batched_4096_r3", 4096, 3, 10.0, 20.0, 0.5, 0.8)


def batched_partial() -> BatchSpec:
    """The 4096-table batch with a seeded 5% of its tables at load 1.0-1.2 c*:
    those keep a 2-core, so the batch exercises partial listing."""
    return BatchSpec("iblt_batched_4096_r3_partial5", 4096, 3, 10.0, 20.0, 0.5, 0.8,
                     hot_frac=0.05, hot_lo=1.0, hot_hi=1.2)


def batched_few_large() -> BatchSpec:
    """16 tables of 2^20 cells at 0.7 c*: fewer tables than the GPU has CUs, the
    case a team of workgroups per table is for."""
    return BatchSpec("iblt_batched_16x1M_r3", 16, 3, 20.0, 20.0, 0.7, 0.7)


@dataclass(frozen=True)
class ServeSpec:
    """Poisson arrivals of IBLT list requests of mixed sizes (served decoding)."""
    name: str
    r_choices: tuple = (3, 4)
    log2_lo: float = 8.0
    log2_hi: float = 22.0
    load_lo: float = 0.4   # as a fraction of c*_{2,r}
    load_hi: float = 0.85
    budget_bytes: int = 64 << 30

    def requests(self, count: int, rate: float, seed: int):
        """[(arrival_s, r, ncells, nkeys, key_seed, table_seed)]; rate <= 0 = all at t=0."""
        st = gen.stream_seed(seed, 0x7C3B2A1908F7E6D5)
        u = gen.splitmix64(st, np.arange(5 * count, dtype=np.uint64)).reshape(count, 5)
        unit = (u >> np.uint64(11)).astype(np.float64) / float(1 << 53)
        out, t = [], 0.0
        for i in range(count):
            if rate > 0:
                t += -np.log(1.0 - unit[i, 0]) / rate
            r = self.r_choices[int(unit[i, 1] * len(self.r_choices)) % len(self.r_choices)]
            N = max(r, int(round(2.0 ** (self.log2_lo + (self.log2_hi - self.log2_lo) * unit[i, 2]))))
            load = (self.load_lo + (self.load_hi - self.load_lo) * unit[i, 3]) * cstar(2, r)
            ks = int(u[i, 4])
            out.append((t, r, N, int(round(load * N)), ks, gen.table_seed(ks)))
        return out


def served_main() -> ServeSpec:
    return ServeSpec("iblt_served_r34_N256-4M")
