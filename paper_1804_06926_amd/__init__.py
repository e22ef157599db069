"""Exact triangle counting on one MI355X (gfx950).

A thin Python binding of ``libtc_mi355x.so`` (C ABI in ``include/tc.h``). Every
step of the counting path runs in the library's HIP kernels; this module only
marshals arguments. PyTorch provides device memory and the stream.

If the library is not built the functions raise ``RuntimeError``: there is no
CPU fallback.
"""
from ._lib import (  # noqa: F401
    FORCE_BITMAP,
    FORCE_BSEARCH,
    FORCE_MERGE,
    SELECT_HEURISTIC,
    SELECT_LEARNED,
    TCError,
    build_csr,
    count_triangles,
    edge_counts,
    last_stats,
    library_path,
    radix_sort_u64,
    stage_names,
    workspace_size,
)
