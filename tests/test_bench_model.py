"""The bench's algorithmic byte models against the closed forms and the
figures they must give at the benchmark shapes, and its host description.
No GPU is used."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_peel_bytes_fully_peeled_is_16n_plus_16rm():
    # every vertex and edge removed: 8n + 8n + 4 r m + m (8 + 4r + 8(r-1)) = 16n + 16rm
    rng = np.random.default_rng(5)
    n, m, r = 1000, 700, 4
    edges = rng.integers(0, n, size=(m, r), dtype=np.uint32)
    deg0 = np.bincount(edges.ravel(), minlength=n).astype(np.uint32)
    vr = np.ones(n, np.uint32)
    er = np.ones(m, np.uint32)
    assert bench.peel_bytes(n, r, edges, deg0, vr, er) == 16 * n + 16 * r * m


def test_peel_bytes_counts_only_what_was_removed():
    n, m, r = 10, 4, 3
    edges = np.array([[0, 1, 2], [2, 3, 4], [5, 6, 7], [7, 8, 9]], np.uint32)
    deg0 = np.bincount(edges.ravel(), minlength=n).astype(np.uint32)
    vr = np.zeros(n, np.uint32)
    er = np.zeros(m, np.uint32)
    vr[[0, 1]] = 1  # two vertices of degree 1 leave with edge 0
    er[0] = 1
    want = 8 * n + 8 * 2 + 4 * 2 + 1 * (8 + 4 * r + 8 * (r - 1))
    assert bench.peel_bytes(n, r, edges, deg0, vr, er) == want


def test_byte_models_at_the_benchmark_shapes():
    n, m, r = 1 << 24, 11_744_051, 4
    # peel, fully peeled (c = 0.70 peels everything): 1.020 GB
    deg0 = np.zeros(n, np.uint32)
    deg0[0] = r * m
    full = bench.peel_bytes(n, r, None, deg0, np.ones(n, np.uint32), np.ones(m, np.uint32))
    assert full == 1_020_054_720
    assert abs(bench.build_bytes(n, m, r) / 1e9 - 1.450) < 5e-4
    N, keys = 1 << 24, 10_296_982
    assert abs(bench.iblt_list_bytes(N, 3, keys) / 1e9 - 1.591) < 5e-4
    assert bench.iblt_insert_bytes(keys, 3) == keys * 128


def test_host_description():
    h = bench.host_cpu()
    assert isinstance(h["model"], str)
    assert h["nproc"] >= 1 and 1 <= h["usable"] <= h["nproc"]


def test_cpu_baseline_on_the_small_workload():
    from workloads import configs
    spec = configs.kcore_small()
    cb = bench.cpu_baseline(spec, spec.edges(1))
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0
    # c = 0.70 < c*: both the round-synchronous and the serial peel remove every edge
    assert cb["serial_queue"]["value"] > 0
    assert str(spec.m) in cb["sample"]
