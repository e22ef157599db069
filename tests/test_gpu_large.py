"""Parity at the full workload sizes: R-MAT scale 24, the random geometric graph on
2^23 vertices and the batch of 4096 Chung-Lu graphs.

The oracle cannot count these whole within a test's time, so the GPU outputs
are checked on samples the oracle computes one by one (t[v] by definition,
oriented per-edge counts by definition, per-graph counts of sampled graphs) and
through properties that hold at any size (sum of t[v] = 3T; the three
strategies agree edge by edge; the batch's counts add up to the union's count).
"""
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]


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


def _check_large(tc, name, e, n, degree):
    import torch
    print(f"[{name}] E={e.shape[0]} n={n}: GPU counts", flush=True)
    d = torch.from_numpy(e).cuda()
    T = tc.count_triangles(d, n)
    T2, t = tc.count_triangles(d, n, per_vertex=True)
    t = t.cpu().numpy().astype(np.uint64)
    assert T2 == T and int(t.sum()) == 3 * T
    edges_by_kernel = {}
    for sel in (tc.FORCE_MERGE, tc.FORCE_BSEARCH, tc.FORCE_BITMAP):
        print(f"[{name}] per-edge counts, strategy {sel}", flush=True)
        pairs, counts, T3 = tc.edge_counts(d, n, select=sel)
        assert T3 == T
        edges_by_kernel[sel] = (pairs.cpu().numpy(), counts.cpu().numpy())
    p0, c0 = edges_by_kernel[tc.FORCE_MERGE]
    for sel in (tc.FORCE_BSEARCH, tc.FORCE_BITMAP):
        np.testing.assert_array_equal(edges_by_kernel[sel][0], p0)
        np.testing.assert_array_equal(edges_by_kernel[sel][1], c0)
    assert int(c0.astype(np.int64).sum()) == T
    del d
    print(f"[{name}] oracle graph", flush=True)
    g = oracle.Graph(e, n)
    assert g.m == p0.shape[0]
    rng = np.random.default_rng(2024)
    deg = g.degrees()
    top = np.argsort(deg)[-40:]
    some = rng.choice(np.nonzero(deg > 0)[0], 200, replace=False)
    low = rng.choice(n, 20, replace=False)
    vs = np.unique(np.concatenate([top, some, low])).astype(np.int32)
    print(f"[{name}] oracle t[v] for {vs.size} vertices", flush=True)
    np.testing.assert_array_equal(g.vertex_triangles(vs), t[vs])
    idx = rng.choice(p0.shape[0], 3000, replace=False)
    print(f"[{name}] oracle per-edge counts for {idx.size} edges", flush=True)
    np.testing.assert_array_equal(g.pair_counts(p0[idx], degree).astype(np.int64), c0[idx].astype(np.int64))
    return T


def test_rmat24_sampled(tc):
    n = 1 << 24
    e = graphgen.rmat(24, 16, seed=1)
    # raw R-MAT draws repeat pairs: the GPU orders by input-pair degree
    _check_large(tc, "rmat24", e, n, "input")


def test_rgg23_sampled(tc):
    n = 1 << 23
    e = graphgen.rgg(n, 32.0, seed=5)
    _check_large(tc, "rgg23", e, n, "simple")


def test_chung_lu_batch_4096_sampled(tc):
    import torch
    print("[batch] generating 4096 Chung-Lu graphs", flush=True)
    e, off, nv = graphgen.chung_lu_batch(4096)
    d = torch.from_numpy(e).cuda()
    print(f"[batch] E={e.shape[0]}: batched count", flush=True)
    got = tc.count_triangles_batch(d, off, nv)
    again = tc.count_triangles_batch(d, off, nv)   # graph replay
    np.testing.assert_array_equal(got, again)
    # the union counted as one graph (vertex ids shifted) gives the sum
    base = np.zeros(nv.size, dtype=np.int64)
    np.cumsum(nv[:-1].astype(np.int64), out=base[1:])
    shift = np.repeat(base, np.diff(off)).astype(np.int32)
    union = e + shift[:, None]
    N = int(nv.astype(np.int64).sum())
    print("[batch] union count", flush=True)
    T_union = tc.count_triangles(torch.from_numpy(union).cuda(), N)
    assert int(got.astype(np.int64).sum()) == T_union
    del union
    rng = np.random.default_rng(7)
    sizes = np.diff(off)
    sample = np.unique(np.concatenate([np.argsort(sizes)[-6:], np.argsort(sizes)[:6],
                                       rng.choice(nv.size, 36, replace=False)]))
    print(f"[batch] oracle on {sample.size} graphs", flush=True)
    for g in sample:
        ref = oracle.count_triangles(e[off[g]:off[g + 1]], int(nv[g]))
        assert int(got[g]) == ref, g


def test_formulations_rmat20_against_oracle(tc):
    """The benchmark graph (R-MAT 20) through every formulation and strategy:
    T equal to the oracle's, and the sums 3T (full lists), 2T (sum of C) and T."""
    import torch
    n = 1 << 20
    e = graphgen.rmat(20, 16, seed=1)
    print("[rmat20] oracle T", flush=True)
    T = oracle.count_triangles(e, n)
    d = torch.from_numpy(e).cuda()
    for form, k in (("filtered", 1), ("full", 3), ("matrix", 2), ("matrix_upper", 1)):
        for sel in (tc.SELECT_HEURISTIC, tc.FORCE_MERGE, tc.FORCE_BSEARCH, tc.FORCE_BITMAP):
            print(f"[rmat20] formulation={form} select={sel}", flush=True)
            assert tc.count_triangles_formulation(d, n, form, select=sel) == (T, k * T)


def test_formulations_rmat24_sums(tc):
    """R-MAT 24 (heuristic selection): every formulation's T equals the filtered
    count (itself checked on samples above) and the sums are 3T, 2T and T."""
    import torch
    n = 1 << 24
    e = graphgen.rmat(24, 16, seed=1)
    d = torch.from_numpy(e).cuda()
    print("[rmat24] filtered", flush=True)
    T = tc.count_triangles(d, n)
    for form, k in (("full", 3), ("matrix", 2), ("matrix_upper", 1)):
        print(f"[rmat24] formulation={form}", flush=True)
        assert tc.count_triangles_formulation(d, n, form) == (T, k * T)
