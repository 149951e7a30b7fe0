"""ctypes front-end of the C oracle (``oracle/oracle.c``); test infrastructure only.

Each wrapper takes and returns numpy arrays.  The shared object is compiled
with gcc on first use (or by ``build()``), next to its source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE, ENOSPC, EROUNDS, ECORRUPT, ENOMEM = 0, -1, -2, -3, -4, -5, -7

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 into ``oracle/liboracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-std=gnu11", "-Wall", "-Wextra", "-shared", "-fPIC",
                        "-o", tmp, _SRC], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build(force=False)
        L = C.CDLL(_LIB)
        P = C.c_void_p
        u32, u64, i32 = C.c_uint32, C.c_uint64, C.c_int32
        L.orc_splitmix64.argtypes = [u64, u64]
        L.orc_splitmix64.restype = u64
        L.orc_peel_rounds.argtypes = [u32, u64, u32, u32, P, u32, P, P, P, P, P, P, P]
        L.orc_peel_subrounds.argtypes = [u32, u64, u32, u32, P, u32, P, P, P, P, P, P, P]
        L.orc_peel_queue.argtypes = [u32, u64, u32, u32, P, u64, P, P]
        L.orc_core_brute.argtypes = [u32, u64, u32, u32, P, P, P]
        L.orc_iblt_cells_of.argtypes = [u64, u32, u64, P, u64, P, P]
        L.orc_iblt_update.argtypes = [u64, u32, u64, P, P, P, P, u64, i32]
        L.orc_iblt_list_rounds.argtypes = [u64, u32, u64, P, P, P, P, u64, P, u32, P, P, P]
        L.orc_iblt_list_subrounds.argtypes = L.orc_iblt_list_rounds.argtypes
        L.orc_iblt_list_signed.argtypes = [u64, u32, u64, P, P, P, P, P, u64, P, u32, P, P, P]
        L.orc_iblt_list_seq.argtypes = [u64, u32, u64, P, P, P, P, u64, P]
        for f in ("orc_peel_rounds", "orc_peel_subrounds", "orc_peel_queue", "orc_core_brute", "orc_iblt_cells_of",
                  "orc_iblt_update", "orc_iblt_list_rounds", "orc_iblt_list_subrounds",
                  "orc_iblt_list_signed",
                  "orc_iblt_list_seq"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _edges(edges) -> np.ndarray:
    e = np.ascontiguousarray(edges, dtype=np.uint32)
    if e.ndim != 2:
        raise ValueError("edges must be (m, r)")
    return e


def splitmix64(seed: int, i: int) -> int:
    return int(lib().orc_splitmix64(seed, i))


@dataclass
class PeelResult:
    status: int
    vertex_round: np.ndarray  # uint32[n], 0 = in core
    edge_round: np.ndarray    # uint32[m], 0 = in core
    deg: np.ndarray           # uint32[n], core degree (0 for removed vertices)
    V: np.ndarray             # uint64[rounds], vertices removed per round
    E: np.ndarray             # uint64[rounds], edges removed per round
    rounds: int               # last round that removed a vertex
    edge_rounds: int          # last round that removed an edge


def peel_rounds(n: int, edges, k: int, max_rounds: int = 1 << 20) -> PeelResult:
    """Round-synchronous peel to the k-core (Section 1; Section 3)."""
    e = _edges(edges)
    m, r = e.shape
    vr = np.zeros(n, np.uint32)
    er = np.zeros(m, np.uint32)
    deg = np.zeros(n, np.uint32)
    cap = min(max_rounds, n) + 1
    V = np.zeros(cap, np.uint64)
    E = np.zeros(cap, np.uint64)
    R = C.c_uint32(0)
    Re = C.c_uint32(0)
    st = lib().orc_peel_rounds(n, m, r, k, _p(e), min(max_rounds, cap - 1), _p(vr), _p(er), _p(deg),
                               _p(V), _p(E), C.byref(R), C.byref(Re))
    if st not in (OK, EROUNDS):
        raise RuntimeError(f"orc_peel_rounds failed: {st}")
    return PeelResult(st, vr, er, deg, V[: R.value].copy(), E[: R.value].copy(), R.value, Re.value)


def peel_subrounds(n: int, edges, k: int, max_rounds: int = 1 << 20) -> PeelResult:
    """Peeling with subtables (Appendix B): r subrounds per round, subround (i, j)
    removing the vertices of subtable j below degree k.  Rounds in the result are
    subrounds, numbered (i-1) r + j from 1."""
    e = _edges(edges)
    m, r = e.shape
    vr = np.zeros(n, np.uint32)
    er = np.zeros(m, np.uint32)
    deg = np.zeros(n, np.uint32)
    cap = min(max_rounds, r * (n + 1)) + 1
    V = np.zeros(cap, np.uint64)
    E = np.zeros(cap, np.uint64)
    R = C.c_uint32(0)
    Re = C.c_uint32(0)
    st = lib().orc_peel_subrounds(n, m, r, k, _p(e), min(max_rounds, cap - 1), _p(vr), _p(er),
                                  _p(deg), _p(V), _p(E), C.byref(R), C.byref(Re))
    if st not in (OK, EROUNDS):
        raise RuntimeError(f"orc_peel_subrounds failed: {st}")
    return PeelResult(st, vr, er, deg, V[: R.value].copy(), E[: R.value].copy(), R.value, Re.value)


def peel_queue(n: int, edges, k: int, order_seed: int = 0):
    """Sequential peel (Section 1); returns (core_vertex, core_edge) bool masks."""
    e = _edges(edges)
    m, r = e.shape
    cv = np.zeros(n, np.uint8)
    ce = np.zeros(m, np.uint8)
    st = lib().orc_peel_queue(n, m, r, k, _p(e), order_seed, _p(cv), _p(ce))
    if st != OK:
        raise RuntimeError(f"orc_peel_queue failed: {st}")
    return cv.astype(bool), ce.astype(bool)


def core_brute(n: int, edges, k: int):
    """Exhaustive k-core of a tiny hypergraph (m <= 24); (core_vertex, core_edge)."""
    e = _edges(edges)
    m, r = e.shape
    cv = np.zeros(n, np.uint8)
    ce = np.zeros(max(m, 1), np.uint8)
    st = lib().orc_core_brute(n, m, r, k, _p(e), _p(cv), _p(ce))
    if st != OK:
        raise RuntimeError(f"orc_core_brute failed: {st}")
    return cv.astype(bool), ce[:m].astype(bool)


@dataclass
class IbltTable:
    """Structure-of-arrays IBLT cells as the oracle keeps them."""
    ncells: int
    r: int
    seed: int
    count: np.ndarray     # int32[ncells]
    key_sum: np.ndarray   # uint64[ncells]
    hash_sum: np.ndarray  # uint64[ncells]

    @classmethod
    def empty(cls, ncells: int, r: int, seed: int) -> "IbltTable":
        return cls(ncells, r, seed, np.zeros(ncells, np.int32), np.zeros(ncells, np.uint64),
                   np.zeros(ncells, np.uint64))

    def copy(self) -> "IbltTable":
        return IbltTable(self.ncells, self.r, self.seed, self.count.copy(), self.key_sum.copy(),
                         self.hash_sum.copy())

    def is_empty(self) -> bool:
        return not (self.count.any() or self.key_sum.any() or self.hash_sum.any())


def iblt_cells_of(ncells: int, r: int, seed: int, keys):
    """The r cells and the checksum of each key: ((nkeys, r) uint64, (nkeys,) uint64)."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    cells = np.zeros((k.size, r), np.uint64)
    chk = np.zeros(k.size, np.uint64)
    st = lib().orc_iblt_cells_of(ncells, r, seed, _p(k), k.size, _p(cells), _p(chk))
    if st != OK:
        raise RuntimeError(f"orc_iblt_cells_of failed: {st}")
    return cells, chk


def iblt_update(t: IbltTable, keys, sign: int = 1) -> IbltTable:
    """Insert (sign=+1) or delete (sign=-1) keys in place (Section 5, "Motivation")."""
    k = np.ascontiguousarray(keys, dtype=np.uint64)
    st = lib().orc_iblt_update(t.ncells, t.r, t.seed, _p(t.count), _p(t.key_sum), _p(t.hash_sum),
                               _p(k), k.size, sign)
    if st != OK:
        raise RuntimeError(f"orc_iblt_update failed: {st}")
    return t


def iblt_insert(ncells: int, r: int, seed: int, keys) -> IbltTable:
    return iblt_update(IbltTable.empty(ncells, r, seed), keys, +1)


@dataclass
class ListResult:
    status: int
    keys: np.ndarray     # uint64[n_listed], grouped by round, ascending within a round
    K: np.ndarray        # uint64[rounds], keys listed per round
    rounds: int
    corrupt: bool

    def per_round(self):
        out, off = [], 0
        for kk in self.K.tolist():
            out.append(self.keys[off: off + kk])
            off += kk
        return out


def iblt_list_rounds(t: IbltTable, max_rounds: int = 1 << 20, out_cap: int | None = None) -> ListResult:
    """Round-synchronous listing (Section 5); consumes ``t`` in place."""
    cap = t.ncells if out_cap is None else out_cap
    out = np.zeros(max(cap, 1), np.uint64)
    kcap = min(max_rounds, t.ncells) + 1
    K = np.zeros(kcap, np.uint64)
    nl = C.c_uint64(0)
    R = C.c_uint32(0)
    bad = C.c_int32(0)
    st = lib().orc_iblt_list_rounds(t.ncells, t.r, t.seed, _p(t.count), _p(t.key_sum), _p(t.hash_sum),
                                    _p(out), cap, _p(K), min(max_rounds, kcap - 1), C.byref(nl),
                                    C.byref(R), C.byref(bad))
    if st not in (OK, EROUNDS, ENOSPC):
        raise RuntimeError(f"orc_iblt_list_rounds failed: {st}")
    return ListResult(st, out[: nl.value].copy(), K[: R.value].copy(), R.value, bool(bad.value))


def iblt_list_subrounds(t: IbltTable, max_rounds: int = 1 << 20,
                        out_cap: int | None = None) -> ListResult:
    """Listing with subtables (Section 5; Appendix B): r subrounds per round, each
    listing the pure cells of one subtable; consumes ``t``.  Rounds in the result
    are subrounds, numbered (i-1) r + j from 1."""
    cap = t.ncells if out_cap is None else out_cap
    out = np.zeros(max(cap, 1), np.uint64)
    kcap = min(max_rounds, t.r * (t.ncells + 1)) + 1
    K = np.zeros(kcap, np.uint64)
    nl = C.c_uint64(0)
    R = C.c_uint32(0)
    bad = C.c_int32(0)
    st = lib().orc_iblt_list_subrounds(t.ncells, t.r, t.seed, _p(t.count), _p(t.key_sum),
                                       _p(t.hash_sum), _p(out), cap, _p(K),
                                       min(max_rounds, kcap - 1), C.byref(nl), C.byref(R),
                                       C.byref(bad))
    if st not in (OK, EROUNDS, ENOSPC):
        raise RuntimeError(f"orc_iblt_list_subrounds failed: {st}")
    return ListResult(st, out[: nl.value].copy(), K[: R.value].copy(), R.value, bool(bad.value))


@dataclass
class SignedListResult:
    status: int
    keys: np.ndarray     # uint64[n_listed], grouped by round, ascending within a round
    signs: np.ndarray    # int8[n_listed]: +1 inserted, -1 deleted
    K: np.ndarray        # uint64[rounds]
    rounds: int
    nonempty: int        # cells left non-zero

    def per_round(self):
        out, off = [], 0
        for kk in self.K.tolist():
            out.append((self.keys[off: off + kk], self.signs[off: off + kk]))
            off += kk
        return out


def iblt_list_signed(t: IbltTable, max_rounds: int = 1 << 20,
                     out_cap: int | None = None) -> SignedListResult:
    """Round-synchronous listing of a table holding deletions too (Section 5); pure =
    count +-1 with a matching checksum; consumes ``t``."""
    cap = t.ncells if out_cap is None else out_cap
    out = np.zeros(max(cap, 1), np.uint64)
    sg = np.zeros(max(cap, 1), np.int8)
    kcap = min(max_rounds, t.ncells) + 1
    K = np.zeros(kcap, np.uint64)
    nl = C.c_uint64(0)
    R = C.c_uint32(0)
    ne = C.c_uint64(0)
    st = lib().orc_iblt_list_signed(t.ncells, t.r, t.seed, _p(t.count), _p(t.key_sum),
                                    _p(t.hash_sum), _p(out), _p(sg), cap, _p(K),
                                    min(max_rounds, kcap - 1), C.byref(nl), C.byref(R),
                                    C.byref(ne))
    if st not in (OK, EROUNDS, ENOSPC):
        raise RuntimeError(f"orc_iblt_list_signed failed: {st}")
    n = nl.value
    return SignedListResult(st, out[:n].copy(), sg[:n].copy(), K[: R.value].copy(), R.value,
                            ne.value)


def iblt_list_seq(t: IbltTable) -> np.ndarray:
    """Sequential listing (one pure cell at a time); consumes ``t``; keys in discovery order."""
    out = np.zeros(max(t.ncells, 1), np.uint64)
    nl = C.c_uint64(0)
    st = lib().orc_iblt_list_seq(t.ncells, t.r, t.seed, _p(t.count), _p(t.key_sum), _p(t.hash_sum),
                                 _p(out), t.ncells, C.byref(nl))
    if st != OK:
        raise RuntimeError(f"orc_iblt_list_seq failed: {st}")
    return out[: nl.value].copy()
