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
    SELECTOR_NUM_FEATURES,
    SELECTOR_NUM_PARAMS,
    TCError,
    bucket_features,
    build_csr,
    clustering,
    count_triangles,
    count_triangles_async,
    count_triangles_noalloc,
    NOALLOC_SCRATCH_BYTES,
    count_triangles_formulation,
    FORMULATIONS,
    count_triangles_batch,
    edge_counts,
    edge_support,
    last_stats,
    list_triangles,
    library_path,
    profile_buckets,
    profile_choices,
    profile_selected,
    radix_sort_u64,
    radix_partition_u64,
    sort_runs_u64,
    selector_forward,
    selector_get_params,
    selector_load,
    selector_save,
    selector_gradient,
    selector_set_params,
    selector_get_tile_params,
    selector_set_tile_params,
    selector_train_step,
    set_tile_shapes,
    stage_names,
    workspace_size,
)
