"""The no-allocation entry point (tc_count_triangles_noalloc), called through the C
ABI, against the entry point it varies (tc_count_triangles_async on a workspace the
caller allocates) and the oracle: two calls in a row on the fixed per-GPU scratch, the
second on a smaller graph (the scratch keeps the first call's contents), then a graph
too large for the scratch, rejected before anything is queued."""
import ctypes
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu

TC_ERR_WORKSPACE = 3


@pytest.fixture(scope="module")
def tc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1804_06926_amd import _lib
    if not os.path.exists(_lib.library_path()):
        import __graft_entry__
        __graft_entry__.build()
    import paper_1804_06926_amd
    return paper_1804_06926_amd


def _abi(tc):
    from paper_1804_06926_amd import _lib
    lib = _lib._load()
    vp = ctypes.c_void_p
    lib.tc_count_triangles_noalloc.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(_lib.Options),
                                               vp, vp]
    lib.tc_count_triangles_noalloc.restype = ctypes.c_int
    return _lib, lib


def _noalloc(tc, d, n, select):
    """One call of tc_count_triangles_noalloc; returns (status, result[2], t[v])."""
    import torch
    _lib, lib = _abi(tc)
    ctx, _ = _lib._ctx(d.device)
    res = torch.full((2,), -7, dtype=torch.int64, device=d.device)
    pv = torch.full((n,), -7, dtype=torch.int64, device=d.device)
    o = _lib._options(select, False)
    st = lib.tc_count_triangles_noalloc(ctx, d.data_ptr(), d.shape[0], n, ctypes.byref(o), res.data_ptr(),
                                        pv.data_ptr())
    torch.cuda.synchronize()
    return st, res.cpu().numpy(), pv.cpu().numpy()


def _async(tc, d, n, select):
    import torch
    res = torch.full((2,), -7, dtype=torch.int64, device=d.device)
    pv = torch.full((n,), -7, dtype=torch.int64, device=d.device)
    tc.count_triangles_async(d, n, result=res, per_vertex=pv, select=select)
    torch.cuda.synchronize()
    return res.cpu().numpy(), pv.cpu().numpy()


def test_noalloc_equals_async_entry_point_on_two_calls(tc):
    import torch
    graphs = [("rmat16 (raw draws)", graphgen.rmat(16, 16, seed=3), 1 << 16),
              ("er4096", graphgen.erdos_renyi(4096, 32768, seed=1804), 4096)]
    assert graphs[1][1].shape[0] < graphs[0][1].shape[0]   # the second call is smaller
    for sel in (tc.SELECT_HEURISTIC, tc.FORCE_MERGE, tc.FORCE_BSEARCH, tc.FORCE_BITMAP):
        for name, e, n in graphs:
            print(f"[noalloc] {name} select={sel}", flush=True)
            assert tc.workspace_size(e.shape[0], n) <= tc.NOALLOC_SCRATCH_BYTES
            d = torch.from_numpy(e).cuda()
            st, res, pv = _noalloc(tc, d, n, sel)
            assert st == 0
            ref_res, ref_pv = _async(tc, d, n, sel)
            T, t = oracle.count_triangles(e, n, per_vertex=True)
            assert res[1] == 0 and ref_res[1] == 0
            assert int(res[0]) == int(ref_res[0]) == T
            np.testing.assert_array_equal(pv, ref_pv)
            np.testing.assert_array_equal(pv.astype(np.uint64), t)


def test_noalloc_rejects_graphs_beyond_the_scratch(tc):
    import torch
    n = 1 << 22
    E = 3 << 20
    assert tc.workspace_size(E, n) > tc.NOALLOC_SCRATCH_BYTES
    d = torch.zeros((E, 2), dtype=torch.int32, device="cuda")   # a real buffer of E pairs
    st, res, _ = _noalloc(tc, d, n, tc.SELECT_HEURISTIC)
    assert st == TC_ERR_WORKSPACE
    assert np.all(res == -7)   # nothing was queued
    # the scratch still serves a small graph afterwards
    e = graphgen.erdos_renyi(4096, 32768, seed=1804)
    st, res, _ = _noalloc(tc, torch.from_numpy(e).cuda(), 4096, tc.SELECT_HEURISTIC)
    assert st == 0 and res[1] == 0 and int(res[0]) == oracle.count_triangles(e, 4096)
