"""Round-synchronous parallel peeling on MI355X (gfx950).

Paper: J. Jiang, M. Mitzenmacher, J. Thaler, "Parallel Peeling Algorithms".
The HIP kernels live in ``libpeel.so`` behind the C ABI of ``include/peel.h``;
``binding`` is its thin Python face (PyTorch for device memory and streams).
"""
from .binding import (  # noqa: F401
    EXPORTS, FLAG_ECORRUPT, FLAG_EINVAL, FLAG_ENOSPC, FLAG_ERANGE, FLAG_EROUNDS, FLAG_ETEAM,
    FLAG_TIMEOUT,
    IBLT_LDS_CELLS, IBLT_LDS_MAX_CELLS, IBLT_NOALLOC_MAX_CELLS, BatchSchedule, BatchTable, Csr, IbltDesc,
    ListOut, PeelError, PeelOut, SignedListOut, batch_entries, batch_table, hg_build,
    hg_build_workspace, iblt_delete, iblt_desc, iblt_insert, iblt_list, iblt_list_batched,
    iblt_list_batched_noalloc, iblt_list_batched_workspace, iblt_list_signed, iblt_list_workspace,
    iblt_table, iblt_update, iblt_update_workspace, lib, peel_k2_xor, peel_k2_xor_workspace,
    peel_kcore, peel_kcore_workspace, workspace)
