"""The size limits of the boundary at their edges: a graph with m just below the
documented edge limit (the internal CSR and CSC positions are 32-bit), the limit
itself exceeded (rejected on the host before any launch), and vertex ids wider
than 27 bits (the degree stage's full-sort path)."""
import ctypes
import os
from math import comb

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]

K_MAX_EDGES = (1 << 31) - (1 << 20)   # num_edges above this: TC_ERR_UNSUPPORTED
TC_ERR_UNSUPPORTED = 5


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


def test_edge_limit_boundary_with_clique_union(tc):
    """1,064,699 disjoint copies of K_64: 2,146,433,184 pairs, every one a distinct edge
    (1,888 below the limit), on 68,140,736 vertices. T = copies * C(64, 3) =
    44,359,619,136 and every t[v] = C(63, 2); pairs alternate direction."""
    import torch
    k = 64
    copies = K_MAX_EDGES // comb(k, 2)
    a, b = np.triu_indices(k, 1)
    base = np.stack([a, b], axis=1).astype(np.int32)
    base[1::2] = base[1::2, ::-1]
    E = copies * base.shape[0]
    assert K_MAX_EDGES - comb(k, 2) < E <= K_MAX_EDGES
    n = copies * k
    print(f"[limits] clique union: E={E} n={n}", flush=True)
    e = np.empty((copies, base.shape[0], 2), dtype=np.int32)
    np.add(base[None, :, :], (np.arange(copies, dtype=np.int32) * k)[:, None, None], out=e)
    d = torch.from_numpy(e.reshape(-1, 2)).cuda()
    del e
    T, t = tc.count_triangles(d, n, per_vertex=True)
    assert T == copies * comb(k, 3)
    assert bool((t == comb(k - 1, 2)).all())
    del t
    st = tc.last_stats()
    assert st["m"] == E
    del d
    torch.cuda.empty_cache()


def test_edge_limit_exceeded_is_rejected_before_any_launch(tc):
    import torch
    from paper_1804_06926_amd import _lib
    lib = _lib._load()
    d = torch.zeros((16, 2), dtype=torch.int32, device="cuda")
    ctx, _ = _lib._ctx(d.device)
    o = _lib._options(tc.SELECT_HEURISTIC, False)
    count = ctypes.c_uint64(7)
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st = lib.tc_count_triangles(ctx, d.data_ptr(), K_MAX_EDGES + 1, 4, ws.data_ptr(), ws.numel(), ctypes.byref(o),
                                ctypes.byref(count), None)
    assert st == TC_ERR_UNSUPPORTED and count.value == 7
    out = ctypes.c_size_t()
    assert lib.tc_workspace_size(K_MAX_EDGES + 1, 4, ctypes.byref(o), ctypes.byref(out)) == TC_ERR_UNSUPPORTED
    assert lib.tc_workspace_size(K_MAX_EDGES, 4, ctypes.byref(o), ctypes.byref(out)) == 0


def test_vertex_ids_wider_than_27_bits(tc):
    """n = 2^27 + 1 (28-bit ids): the degree stage counts by a full sort of the
    endpoints. A Chung-Lu graph of 3^7 * 100 vertices with its ids spread over the
    whole range, loops and repeats added: T and t[v] of the touched vertices equal the
    oracle's, and every untouched vertex has t = 0."""
    import torch
    n = (1 << 27) + 1
    small = 218_700
    e = graphgen.chung_lu(small, 1_500_000, seed=31)
    stride = (n - 1) // small
    e = (e.astype(np.int64) * stride + 3).astype(np.int32)
    assert e.max() < n and int(e.max()) >= 1 << 26
    e = np.concatenate([e, e[:1000], np.array([[5, 5], [n - 1, n - 1]], dtype=np.int32)])
    T_ref, t_ref = oracle.count_triangles(e, n, per_vertex=True, threads=2)   # per-thread t arrays of n entries
    d = torch.from_numpy(e).cuda()
    for sel in (tc.SELECT_HEURISTIC, tc.FORCE_MERGE, tc.FORCE_BITMAP):
        T, t = tc.count_triangles(d, n, per_vertex=True, select=sel)
        assert T == T_ref, sel
        np.testing.assert_array_equal(t.cpu().numpy().astype(np.uint64), t_ref)
    del d
