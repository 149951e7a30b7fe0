"""Host-side checks of the C ABI: the library loads, exports what peel.h declares,
and rejects bad arguments before touching a GPU.  No kernel runs here."""
import ctypes as C
import os
import re

import pytest

import paper_1302_7014_amd as pk
from paper_1302_7014_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "peel.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b([a-z_][a-z0-9_]*)\s*\(", src)) - {"sizeof", "defined"})


@pytest.fixture(scope="module")
def L():
    return pk.lib()


def test_exports_every_declared_symbol(L):
    names = _declared()
    assert set(names) == set(binding.EXPORTS)
    for name in names:
        assert hasattr(L, name), name


def test_version_and_strerror(L):
    assert L.peel_abi_version() == 7
    for code in range(-6, 1):
        assert L.peel_strerror(code)
    assert L.peel_strerror(-99) == b"unknown status"


def test_workspace_queries(L):
    assert L.hg_build_workspace(1 << 24, 11744051, 4) >= (1 << 24) * 4
    assert L.peel_kcore_workspace(1 << 24, 11744051, 4) >= 2 * (1 << 24) * 4
    d = pk.iblt_desc(1 << 24, 3, 7)
    assert L.iblt_list_workspace(C.byref(d)) >= 2 * (1 << 24) * 4
    bad = pk.iblt_desc(2, 3, 7)  # fewer cells than subtables
    assert L.iblt_list_workspace(C.byref(bad)) == 0


def test_argument_errors_are_reported_on_the_host(L):
    P = C.c_void_p
    dummy = P(0x1000)
    # r out of range
    assert L.hg_build(dummy, 10, 1, 10, dummy, dummy, dummy, dummy, dummy, 1 << 20, None) == pk.binding.PEEL_EINVAL
    assert L.hg_build(dummy, 10, 9, 10, dummy, dummy, dummy, dummy, dummy, 1 << 20, None) == pk.binding.PEEL_EINVAL
    # m*r >= 2^32
    assert L.hg_build(dummy, 1 << 31, 2, 10, dummy, dummy, dummy, dummy, dummy, 1 << 20, None) == pk.binding.PEEL_EINVAL
    # workspace too small
    assert L.hg_build(dummy, 10, 3, 10, dummy, dummy, dummy, dummy, dummy, 1, None) == pk.binding.PEEL_ENOSPC
    # k = 0, max_rounds = 0, n = 0
    args = [dummy, 10, 3, 10, 0, dummy, dummy, dummy, dummy, dummy, dummy, 8, dummy, dummy, 1 << 20, None]
    assert L.peel_kcore(*args) == pk.binding.PEEL_EINVAL
    args[4], args[11] = 2, 0
    assert L.peel_kcore(*args) == pk.binding.PEEL_EINVAL
    args[11], args[3] = 8, 0
    assert L.peel_kcore(*args) == pk.binding.PEEL_EINVAL
    d = pk.iblt_desc(100, 9, 1)
    assert L.iblt_insert(C.byref(d), dummy, dummy, 5, None) == pk.binding.PEEL_EINVAL
    d = pk.iblt_desc(100, 3, 1)
    assert L.iblt_list(C.byref(d), dummy, dummy, 10, dummy, 8, dummy, dummy, 1, None) == pk.binding.PEEL_ENOSPC
    assert L.iblt_list(C.byref(d), dummy, dummy, 10, dummy, 0, dummy, dummy, 1 << 20, None) == pk.binding.PEEL_EINVAL


def test_batched_schedule_is_checked_on_the_host(L):
    src = open(os.path.join(ROOT, "include", "peel.h")).read()
    assert int(re.search(r"#define IBLT_LDS_MAX_CELLS (\d+)u", src).group(1)) == pk.IBLT_LDS_MAX_CELLS
    assert C.sizeof(pk.BatchSchedule) == 16
    P = C.c_void_p
    dummy = P(0x1000)
    for bt, lds in [(128, 0), (300, 0), (512, pk.IBLT_LDS_MAX_CELLS + 1)]:
        s = pk.BatchSchedule(bt, lds)
        assert L.iblt_list_batched(dummy, 4, 1000, 8, C.byref(s), dummy, 1 << 30, None) == pk.binding.PEEL_EINVAL
    s = pk.BatchSchedule(512, 0, 1 << 18, 65)  # teams of more than 64 workgroups
    assert L.iblt_list_batched(dummy, 4, 1000, 8, C.byref(s), dummy, 1 << 30, None) == pk.binding.PEEL_EINVAL
    assert L.iblt_list_batched(dummy, 4, 1000, 0, None, dummy, 1 << 30, None) == pk.binding.PEEL_EINVAL


def test_oracle_and_library_share_no_code():
    # The oracle never imports or includes the library, and the library never
    # imports, includes or loads anything of the oracle.
    lib_dir = os.path.join(ROOT, "paper_1302_7014_amd")
    bad_lib = re.compile(r"(^|\n)\s*(import|from)\s+oracle\b|liboracle|oracle\.c|oracle/")
    for dirpath, _, files in os.walk(lib_dir):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert not bad_lib.search(txt), f
    bad_orc = re.compile(r"(^|\n)\s*(import|from)\s+paper_1302_7014_amd\b|#\s*include\s*\"(peel\.h|common\.hpp|host\.hpp)|libpeel")
    for f in os.listdir(os.path.join(ROOT, "oracle")):
        if f.endswith((".py", ".c", ".h")):
            txt = open(os.path.join(ROOT, "oracle", f)).read()
            assert not bad_orc.search(txt), f


def test_binned_update_is_checked_on_the_host(L):
    P = C.c_void_p
    dummy = P(0x1000)
    d = pk.iblt_desc(1 << 24, 3, 7)
    # the sorted entries (10 bytes per key and subtable) dominate the workspace
    nk = 10_296_982
    assert L.iblt_update_workspace(C.byref(d), nk) >= 3 * nk * 10
    big = pk.iblt_desc((1 << 24) + 1, 3, 7)  # past the binned limit: atomic path, no workspace
    assert L.iblt_update_workspace(C.byref(big), nk) == 256
    bad = pk.iblt_desc(2, 3, 7)
    assert L.iblt_update_workspace(C.byref(bad), nk) == 0
    for sign in (0, 2, -2):
        assert L.iblt_update(C.byref(d), dummy, dummy, 5, sign, dummy, 1 << 30, None) == pk.binding.PEEL_EINVAL
    assert L.iblt_update(C.byref(d), P(0x1010), dummy, 5, 1, dummy, 1 << 30, None) == pk.binding.PEEL_EINVAL
    assert L.iblt_update(C.byref(d), dummy, dummy, nk, 1, None, 1 << 30, None) == pk.binding.PEEL_EINVAL
    assert L.iblt_update(C.byref(d), dummy, dummy, nk, 1, dummy, 1024, None) == pk.binding.PEEL_ENOSPC
    assert L.iblt_update(C.byref(d), dummy, dummy, 0, 1, None, 0, None) == pk.binding.PEEL_OK


def test_noalloc_batched_limit_is_checked_on_the_host(L):
    # past its static scratch the no-allocation listing refuses before any launch
    src = open(os.path.join(ROOT, "include", "peel.h")).read()
    lim = int(re.search(r"#define IBLT_NOALLOC_MAX_CELLS (\d+)u", src).group(1))
    assert lim == pk.IBLT_NOALLOC_MAX_CELLS
    dummy = C.c_void_p(0x1000)
    assert L.iblt_list_batched_noalloc(dummy, 4, lim + 1, 8, None, None) == pk.binding.PEEL_ENOSPC
    assert L.iblt_list_batched_noalloc(dummy, 4, 1 << 40, 8, None, None) == pk.binding.PEEL_ENOSPC
