"""Thin ctypes binding of ``libpeel.so`` (the C ABI in ``include/peel.h``).

Argument marshalling only: every step of the path runs in the HIP kernels.
PyTorch supplies device memory and the current stream.  Unsigned 32-bit and
64-bit device arrays travel as ``torch.int32`` / ``torch.int64`` tensors of the
same bit patterns; an IBLT table is an ``(ncells, 4)`` ``torch.int64`` tensor,
32 bytes per cell laid out as ``iblt_cell`` (count in the low half of column
0, key_sum in column 1, hash_sum in column 2).

There is no fallback: if the library is not built, or no GPU is present, the
calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpeel.so")

PEEL_OK, PEEL_EINVAL, PEEL_ERANGE, PEEL_ENOSPC, PEEL_EROUNDS, PEEL_ECORRUPT, PEEL_EHIP = (
    0, -1, -2, -3, -4, -5, -6)
FLAG_ERANGE, FLAG_EROUNDS, FLAG_ENOSPC, FLAG_ECORRUPT, FLAG_TIMEOUT, FLAG_EINVAL, FLAG_ETEAM = (
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20, 0x40)

# Every symbol include/peel.h declares.
EXPORTS = ("peel_strerror", "peel_abi_version", "hg_build_workspace", "hg_build",
           "peel_kcore_workspace", "peel_kcore", "peel_kcore_subtables",
           "peel_k2_xor_workspace", "peel_k2_xor", "iblt_insert",
           "iblt_update_workspace", "iblt_update",
           "iblt_delete", "iblt_list_workspace", "iblt_list", "iblt_list_subtables",
           "iblt_list_signed",
           "iblt_list_batched_workspace", "iblt_list_batched", "iblt_list_batched_noalloc")

_lib = None


class PeelError(RuntimeError):
    pass


class IbltDesc(C.Structure):
    _fields_ = [("ncells", C.c_uint64), ("r", C.c_uint32), ("workgroups", C.c_uint32),
                ("seed", C.c_uint64)]


def lib() -> C.CDLL:
    """Load libpeel.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise PeelError(f"{LIB_PATH} is not built: run `python -m paper_1302_7014_amd.build`")
        L = C.CDLL(LIB_PATH)
        P, u32, u64, sz = C.c_void_p, C.c_uint32, C.c_uint64, C.c_size_t
        L.peel_strerror.argtypes = [C.c_int32]
        L.peel_strerror.restype = C.c_char_p
        L.peel_abi_version.restype = C.c_int
        L.hg_build_workspace.argtypes = [u32, u64, u32]
        L.hg_build_workspace.restype = sz
        L.hg_build.argtypes = [P, u64, u32, u32, P, P, P, P, P, sz, P]
        L.peel_kcore_workspace.argtypes = [u32, u64, u32]
        L.peel_kcore_workspace.restype = sz
        L.peel_kcore.argtypes = [P, u64, u32, u32, u32, P, P, P, P, P, P, u32, P, P, sz, P]
        L.peel_kcore_subtables.argtypes = L.peel_kcore.argtypes
        L.peel_k2_xor_workspace.argtypes = [u32, u64, u32]
        L.peel_k2_xor_workspace.restype = sz
        L.peel_k2_xor.argtypes = [P, u64, u32, u32, P, P, P, P, u32, P, P, sz, P]
        L.iblt_insert.argtypes = [C.POINTER(IbltDesc), P, P, u64, P]
        L.iblt_list_workspace.argtypes = [C.POINTER(IbltDesc)]
        L.iblt_list_workspace.restype = sz
        L.iblt_list.argtypes = [C.POINTER(IbltDesc), P, P, u64, P, u32, P, P, sz, P]
        L.iblt_list_subtables.argtypes = L.iblt_list.argtypes
        L.iblt_list_signed.argtypes = [C.POINTER(IbltDesc), P, P, P, u64, P, u32, P, P, sz, P]
        L.iblt_delete.argtypes = L.iblt_insert.argtypes
        L.iblt_update_workspace.argtypes = [C.POINTER(IbltDesc), u64]
        L.iblt_update_workspace.restype = sz
        L.iblt_update.argtypes = [C.POINTER(IbltDesc), P, P, u64, C.c_int32, P, sz, P]
        L.iblt_list_batched_workspace.argtypes = [u32, u64]
        L.iblt_list_batched_workspace.restype = sz
        L.iblt_list_batched.argtypes = [P, u32, u64, u32, C.POINTER(BatchSchedule), P, sz, P]
        L.iblt_list_batched_noalloc.argtypes = [P, u32, u64, u32, C.POINTER(BatchSchedule), P]
        for f in ("hg_build", "peel_kcore", "peel_kcore_subtables", "peel_k2_xor", "iblt_insert",
                  "iblt_delete",
                  "iblt_update",
                  "iblt_list", "iblt_list_subtables", "iblt_list_signed", "iblt_list_batched",
                  "iblt_list_batched_noalloc"):
            getattr(L, f).restype = C.c_int32
        _lib = L
    return _lib


def _check(st: int, what: str) -> None:
    if st != PEEL_OK:
        raise PeelError(f"{what}: {lib().peel_strerror(st).decode()} ({st})")


def _ptr(t: torch.Tensor | None):
    if t is None:
        return None
    if not t.is_cuda:
        raise PeelError("device tensor expected")
    if not t.is_contiguous():
        raise PeelError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def _empty(n: int, dtype, device) -> torch.Tensor:
    return torch.empty(max(int(n), 1), dtype=dtype, device=device)


def workspace(nbytes: int, device) -> torch.Tensor:
    """A device workspace of at least ``nbytes`` (256-byte aligned by the allocator)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _call_ws(nbytes: int, device, stream) -> torch.Tensor:
    """A workspace a wrapper allocates for one call.  The allocator hands it out
    on the current stream; when the call runs on another stream the tensor is
    marked as used there, so that its memory is not reused before that stream
    has finished with it."""
    ws = workspace(nbytes, device)
    if stream is not None and stream != torch.cuda.current_stream(ws.device):
        ws.record_stream(stream)
    return ws


# ---------------------------------------------------------------------------
@dataclass
class Csr:
    offsets: torch.Tensor  # int32[n+1] (uint32 bits)
    inc: torch.Tensor      # int32[m*r]
    deg: torch.Tensor      # int32[n]
    info: torch.Tensor     # int32[2]: flags, max degree


def hg_build_workspace(n: int, m: int, r: int) -> int:
    return int(lib().hg_build_workspace(n, m, r))


def hg_build(edges: torch.Tensor, n: int, out: Csr | None = None, ws: torch.Tensor | None = None,
             stream=None) -> Csr:
    """CSR incidence of ``edges`` ((m, r) int32 device tensor of uint32 ids)."""
    m, r = edges.shape
    dev = edges.device
    if out is None:
        out = Csr(_empty(n + 1, torch.int32, dev), _empty(m * r, torch.int32, dev),
                  _empty(n, torch.int32, dev), _empty(2, torch.int32, dev))
    if ws is None:
        ws = _call_ws(hg_build_workspace(n, m, r), dev, stream)
    _check(lib().hg_build(_ptr(edges), m, r, n, _ptr(out.offsets), _ptr(out.inc), _ptr(out.deg),
                          _ptr(out.info), _ptr(ws), ws.numel(), _stream(stream)), "hg_build")
    return out


@dataclass
class PeelOut:
    deg: torch.Tensor           # int32[n]
    vertex_round: torch.Tensor  # int32[n]
    edge_round: torch.Tensor    # int32[m]
    round_stats: torch.Tensor   # int64[2*max_rounds]
    summary: torch.Tensor       # int32[8]: rounds, edge rounds, flags, core vertices, team


def peel_kcore_workspace(n: int, m: int, r: int) -> int:
    return int(lib().peel_kcore_workspace(n, m, r))


def peel_kcore(edges: torch.Tensor, n: int, k: int, csr: Csr, max_rounds: int = 4096,
               out: PeelOut | None = None, ws: torch.Tensor | None = None, stream=None,
               subtables: bool = False) -> PeelOut:
    """Round-synchronous peel to the k-core; ``csr.deg`` is consumed (see ``out.deg``).

    ``out.deg`` is ``csr.deg`` itself unless ``out`` brings its own degrees
    (then the caller copies the initial degrees into it).  ``subtables=True``
    calls peel_kcore_subtables: rounds are then subrounds.
    """
    m, r = edges.shape
    dev = edges.device
    if out is None:
        out = PeelOut(csr.deg, _empty(n, torch.int32, dev), _empty(m, torch.int32, dev),
                      _empty(2 * max_rounds, torch.int64, dev), _empty(8, torch.int32, dev))
    if ws is None:
        ws = _call_ws(peel_kcore_workspace(n, m, r), dev, stream)
    fn = lib().peel_kcore_subtables if subtables else lib().peel_kcore
    _check(fn(_ptr(edges), m, r, n, k, _ptr(csr.offsets), _ptr(csr.inc),
              _ptr(out.deg), _ptr(out.vertex_round), _ptr(out.edge_round),
              _ptr(out.round_stats), max_rounds, _ptr(out.summary), _ptr(ws),
              ws.numel(), _stream(stream)), "peel_kcore_subtables" if subtables else "peel_kcore")
    return out


def peel_k2_xor_workspace(n: int, m: int, r: int) -> int:
    return int(lib().peel_k2_xor_workspace(n, m, r))


def peel_k2_xor(edges: torch.Tensor, n: int, max_rounds: int = 4096,
                out: PeelOut | None = None, ws: torch.Tensor | None = None,
                stream=None) -> PeelOut:
    """Peel to the 2-core with no CSR (degrees and edge-id XORs per vertex);
    the same outputs as ``peel_kcore`` with k = 2.  ``out.deg`` receives the
    final degrees."""
    m, r = edges.shape
    dev = edges.device
    if out is None:
        out = PeelOut(_empty(n, torch.int32, dev), _empty(n, torch.int32, dev),
                      _empty(m, torch.int32, dev), _empty(2 * max_rounds, torch.int64, dev),
                      _empty(8, torch.int32, dev))
    if ws is None:
        ws = _call_ws(peel_k2_xor_workspace(n, m, r), dev, stream)
    _check(lib().peel_k2_xor(_ptr(edges), m, r, n, _ptr(out.deg), _ptr(out.vertex_round),
                             _ptr(out.edge_round), _ptr(out.round_stats), max_rounds,
                             _ptr(out.summary), _ptr(ws), ws.numel(), _stream(stream)),
           "peel_k2_xor")
    return out


def iblt_desc(ncells: int, r: int, seed: int, workgroups: int = 0) -> IbltDesc:
    """``workgroups``: iblt_list's persistent workgroups (0 = one per CU)."""
    return IbltDesc(ncells, r, workgroups, seed & 0xFFFFFFFFFFFFFFFF)


def iblt_table(ncells: int, device) -> torch.Tensor:
    """A zeroed table: (ncells, 4) int64, one 32-byte iblt_cell per row."""
    return torch.zeros((ncells, 4), dtype=torch.int64, device=device)


def iblt_insert(desc: IbltDesc, cells: torch.Tensor, keys: torch.Tensor, stream=None) -> None:
    """XOR ``keys`` (int64 device tensor of uint64 keys) into ``cells``."""
    _check(lib().iblt_insert(C.byref(desc), _ptr(cells), _ptr(keys), keys.numel(),
                             _stream(stream)), "iblt_insert")


def iblt_delete(desc: IbltDesc, cells: torch.Tensor, keys: torch.Tensor, stream=None) -> None:
    """Delete ``keys`` from ``cells`` (count down, same XORs)."""
    _check(lib().iblt_delete(C.byref(desc), _ptr(cells), _ptr(keys), keys.numel(),
                             _stream(stream)), "iblt_delete")


def iblt_update_workspace(desc: IbltDesc, nkeys: int) -> int:
    return int(lib().iblt_update_workspace(C.byref(desc), nkeys))


def iblt_update(desc: IbltDesc, cells: torch.Tensor, keys: torch.Tensor, sign: int = 1,
                ws: torch.Tensor | None = None, stream=None) -> None:
    """iblt_insert (sign=+1) or iblt_delete (sign=-1) by binning the keys per
    block of cells: the same cells, without a device atomic per update."""
    if ws is None:
        ws = _call_ws(iblt_update_workspace(desc, keys.numel()), cells.device, stream)
    _check(lib().iblt_update(C.byref(desc), _ptr(cells), _ptr(keys), keys.numel(), sign, _ptr(ws),
                             ws.numel(), _stream(stream)), "iblt_update")


@dataclass
class ListOut:
    keys: torch.Tensor         # int64[out_cap]
    round_stats: torch.Tensor  # int64[max_rounds]: keys listed per round
    summary: torch.Tensor      # int64[8]: listed, rounds, keys left, flags, team


def iblt_list_workspace(desc: IbltDesc) -> int:
    return int(lib().iblt_list_workspace(C.byref(desc)))


def iblt_list(desc: IbltDesc, cells: torch.Tensor, out_cap: int | None = None,
              max_rounds: int = 4096, out: ListOut | None = None, ws: torch.Tensor | None = None,
              stream=None, subtables: bool = False) -> ListOut:
    """Round-synchronous listing; consumes ``cells`` in place.  ``subtables=True``
    calls iblt_list_subtables: rounds are then subrounds."""
    dev = cells.device
    if out is None:
        cap = desc.ncells if out_cap is None else out_cap
        out = ListOut(_empty(cap, torch.int64, dev), _empty(max_rounds, torch.int64, dev),
                      _empty(8, torch.int64, dev))
    cap = out.keys.numel() if out_cap is None else out_cap
    if ws is None:
        ws = _call_ws(iblt_list_workspace(desc), dev, stream)
    fn = lib().iblt_list_subtables if subtables else lib().iblt_list
    _check(fn(C.byref(desc), _ptr(cells), _ptr(out.keys), cap, _ptr(out.round_stats),
              max_rounds, _ptr(out.summary), _ptr(ws), ws.numel(), _stream(stream)),
           "iblt_list_subtables" if subtables else "iblt_list")
    return out


@dataclass
class SignedListOut:
    keys: torch.Tensor         # int64[out_cap]
    signs: torch.Tensor        # int8[out_cap]
    round_stats: torch.Tensor  # int64[max_rounds]
    summary: torch.Tensor      # int64[8]; [2] = cells left non-zero


def iblt_list_signed(desc: IbltDesc, cells: torch.Tensor, out_cap: int | None = None,
                     max_rounds: int = 4096, out: SignedListOut | None = None,
                     ws: torch.Tensor | None = None, stream=None) -> SignedListOut:
    """Signed listing of a table that holds deletions too; consumes ``cells``."""
    dev = cells.device
    if out is None:
        cap = desc.ncells if out_cap is None else out_cap
        out = SignedListOut(_empty(cap, torch.int64, dev), _empty(cap, torch.int8, dev),
                            _empty(max_rounds, torch.int64, dev), _empty(8, torch.int64, dev))
    cap = out.keys.numel() if out_cap is None else out_cap
    if ws is None:
        ws = _call_ws(iblt_list_workspace(desc), dev, stream)
    _check(lib().iblt_list_signed(C.byref(desc), _ptr(cells), _ptr(out.keys), _ptr(out.signs), cap,
                                  _ptr(out.round_stats), max_rounds, _ptr(out.summary), _ptr(ws),
                                  ws.numel(), _stream(stream)), "iblt_list_signed")
    return out


# ---------------------------------------------------------------------------
# Batched listing.

BATCH_ENTRY = [("ncells", "<u8"), ("r", "<u4"), ("workgroups", "<u4"), ("seed", "<u8"),
               ("cells", "<u8"), ("out_keys", "<u8"), ("out_cap", "<u8"),
               ("round_stats", "<u8"), ("summary", "<u8")]


@dataclass
class BatchTable:
    """One table of a batch: its descriptor and device buffers."""
    desc: IbltDesc
    cells: torch.Tensor        # (ncells, 4) int64
    keys: torch.Tensor         # int64[out_cap]
    round_stats: torch.Tensor  # int64[max_rounds]
    summary: torch.Tensor      # int64[8]


def batch_table(desc: IbltDesc, cells: torch.Tensor, max_rounds: int,
                out_cap: int | None = None) -> BatchTable:
    dev = cells.device
    cap = desc.ncells if out_cap is None else out_cap
    return BatchTable(desc, cells, _empty(cap, torch.int64, dev),
                      _empty(max_rounds, torch.int64, dev), _empty(8, torch.int64, dev))


def batch_entries(tables: list[BatchTable], device) -> torch.Tensor:
    """Device array of iblt_batch_entry (64 bytes each) for ``tables``, in order."""
    import numpy as np
    arr = np.zeros(len(tables), dtype=np.dtype(BATCH_ENTRY))
    for i, t in enumerate(tables):
        d = t.desc
        if not (2 <= d.r <= 8 and d.r <= d.ncells < (1 << 32)):
            raise PeelError(f"batch table {i}: r={d.r}, ncells={d.ncells} out of range")
        if t.cells.numel() < 4 * d.ncells or t.cells.data_ptr() % 32:
            raise PeelError(f"batch table {i}: cells too small or not 32-byte aligned")
        arr[i] = (t.desc.ncells, t.desc.r, 0, t.desc.seed, t.cells.data_ptr(), t.keys.data_ptr(),
                  t.keys.numel(), t.round_stats.data_ptr(), t.summary.data_ptr())
    host = torch.from_numpy(arr.view(np.uint8).copy())
    return host.to(device)


def iblt_list_batched_workspace(ntables: int, max_cells: int) -> int:
    return int(lib().iblt_list_batched_workspace(ntables, max_cells))


IBLT_LDS_MAX_CELLS = 5120
# the most cells a workgroup of each size lists from LDS; a larger table is listed in place
IBLT_LDS_CELLS = {256: 2048, 512: 3072, 1024: 5120}


class BatchSchedule(C.Structure):
    """iblt_batch_schedule: threads per workgroup, the LDS-resident size limit,
    and the team ("tile") schedule for large tables."""
    _fields_ = [("block_threads", C.c_uint32), ("lds_max_cells", C.c_uint32),
                ("tile_min_cells", C.c_uint32), ("tile_workgroups", C.c_uint32)]


def iblt_list_batched(entries: torch.Tensor, ntables: int, max_cells: int, max_rounds: int,
                      block_threads: int = 0, lds_max_cells: int | None = None,
                      tile_min_cells: int = 0, tile_workgroups: int = 0,
                      ws: torch.Tensor | None = None, stream=None) -> None:
    """List every table of a batch in one launch (entries from ``batch_entries``).

    ``lds_max_cells``: tables of at most this many cells are listed from LDS
    (None = the library default, IBLT_LDS_MAX_CELLS; 0 = never), as far as the
    workgroup size holds them (IBLT_LDS_CELLS).  Tables of at
    least ``tile_min_cells`` cells are listed by teams of ``tile_workgroups``
    workgroups (0 or 1 = no teams)."""
    if ws is None:
        ws = _call_ws(iblt_list_batched_workspace(ntables, max_cells), entries.device, stream)
    sched = BatchSchedule(block_threads,
                          IBLT_LDS_MAX_CELLS if lds_max_cells is None else lds_max_cells,
                          tile_min_cells, tile_workgroups)
    _check(lib().iblt_list_batched(_ptr(entries), ntables, max_cells, max_rounds, C.byref(sched),
                                   _ptr(ws), ws.numel(), _stream(stream)), "iblt_list_batched")


IBLT_NOALLOC_MAX_CELLS = 16384


def iblt_list_batched_noalloc(entries: torch.Tensor, ntables: int, max_cells: int,
                              max_rounds: int, block_threads: int = 0,
                              lds_max_cells: int | None = None, tile_min_cells: int = 0,
                              tile_workgroups: int = 0, stream=None) -> None:
    """``iblt_list_batched`` without a workspace: the library's own static
    device scratch serves (max_cells <= IBLT_NOALLOC_MAX_CELLS).  Allocates
    nothing; calls that overlap on one device race on that scratch."""
    sched = BatchSchedule(block_threads,
                          IBLT_LDS_MAX_CELLS if lds_max_cells is None else lds_max_cells,
                          tile_min_cells, tile_workgroups)
    _check(lib().iblt_list_batched_noalloc(_ptr(entries), ntables, max_cells, max_rounds,
                                           C.byref(sched), _stream(stream)),
           "iblt_list_batched_noalloc")
