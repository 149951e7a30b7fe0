"""Shared helpers for the GPU parity tests: host <-> device conversion and the
calls into the library, always through the C ABI binding."""
from __future__ import annotations

import sys

import numpy as np
import pytest
import torch

import paper_1302_7014_amd as pk


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def say(*msg):
    print("[case]", *msg, flush=True)
    sys.stdout.flush()


def dev_u32(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint32).view(np.int32)).cuda()


def dev_u64(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.uint64).view(np.int64)).cuda()


def host_u32(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint32)


def host_u64(t: torch.Tensor) -> np.ndarray:
    return t.cpu().numpy().view(np.uint64)


def gpu_peel(n: int, edges: np.ndarray, k: int, max_rounds: int = 4096, subtables: bool = False):
    """hg_build + peel_kcore (or peel_kcore_subtables) on the GPU; returns numpy results."""
    e = dev_u32(edges.reshape(-1, edges.shape[1]) if edges.size else
                np.zeros((0, edges.shape[1]), np.uint32))
    e = e.view(edges.shape[0], edges.shape[1])
    csr = pk.hg_build(e, n)
    deg0 = host_u32(csr.deg)[:n].copy()
    info = host_u32(csr.info)
    out = pk.peel_kcore(e, n, k, csr, max_rounds=max_rounds, subtables=subtables)
    torch.cuda.synchronize()
    m = edges.shape[0]
    summ = host_u32(out.summary)
    stats = host_u64(out.round_stats)[: 2 * max_rounds].reshape(max_rounds, 2)
    R = int(summ[0])
    return {
        "csr": csr, "deg0": deg0, "info": info,
        "vertex_round": host_u32(out.vertex_round)[:n],
        "edge_round": host_u32(out.edge_round)[:m],
        "deg": host_u32(out.deg)[:n],
        "V": stats[:R, 0].copy(), "E": stats[:R, 1].copy(), "stats": stats,
        "rounds": R, "edge_rounds": int(summ[1]), "flags": int(summ[2]), "core": int(summ[3]),
        "team": int(summ[4]),
    }


def table_to_numpy(cells: torch.Tensor):
    """(count int32, key_sum uint64, hash_sum uint64, reserved ok) of a device table."""
    h = cells.cpu().numpy()
    count = h.view(np.int32).reshape(-1, 8)[:, 0].copy()
    res0 = h.view(np.int32).reshape(-1, 8)[:, 1]
    ks = h[:, 1].view(np.uint64).copy()
    hs = h[:, 2].view(np.uint64).copy()
    reserved_ok = bool((res0 == 0).all() and (h[:, 3] == 0).all())
    return count, ks, hs, reserved_ok


def gpu_peel_xor(n: int, edges: np.ndarray, max_rounds: int = 4096):
    """peel_k2_xor on the GPU (no CSR); returns numpy results like gpu_peel."""
    e = dev_u32(edges.reshape(-1, edges.shape[1]) if edges.size else
                np.zeros((0, edges.shape[1]), np.uint32))
    e = e.view(edges.shape[0], edges.shape[1])
    out = pk.peel_k2_xor(e, n, max_rounds=max_rounds)
    torch.cuda.synchronize()
    m = edges.shape[0]
    summ = host_u32(out.summary)
    stats = host_u64(out.round_stats)[: 2 * max_rounds].reshape(max_rounds, 2)
    R = int(summ[0])
    return {
        "vertex_round": host_u32(out.vertex_round)[:n],
        "edge_round": host_u32(out.edge_round)[:m],
        "deg": host_u32(out.deg)[:n],
        "V": stats[:R, 0].copy(), "E": stats[:R, 1].copy(), "stats": stats,
        "rounds": R, "edge_rounds": int(summ[1]), "flags": int(summ[2]), "core": int(summ[3]),
        "team": int(summ[4]),
    }
