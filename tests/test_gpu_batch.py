"""Batched counting on the GPU: per-graph counts equal the oracle's, graph
capture/replay gives the same counts as direct launches, tile shapes never
change counts."""
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


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


def _small_batch(G=64, seed=3):
    e, off, n = graphgen.chung_lu_batch(G, 1e2, 2e4, seed=seed)
    return e, off, n


def _oracle_counts(e, off, n):
    return np.array([oracle.count_triangles(e[off[g]:off[g + 1]], int(n[g])) for g in range(len(n))],
                    dtype=np.uint64)


def test_batch_matches_oracle_per_graph(tc):
    import torch
    e, off, n = _small_batch()
    ref = _oracle_counts(e, off, n)
    d = torch.from_numpy(e).cuda()
    got = tc.count_triangles_batch(d, off, n, graph=False)
    np.testing.assert_array_equal(got, ref)
    assert ref.sum() > 0


def test_graph_replay_matches_eager_and_survives_interleaved_work(tc):
    """Replays of the captured graph, with eager counting calls between them,
    each give the eager per-graph counts."""
    import torch
    e, off, n = _small_batch(48, 7)
    d = torch.from_numpy(e).cuda()
    eager = tc.count_triangles_batch(d, off, n, graph=False)
    other = graphgen.rmat(12, 16, seed=9)
    other_T = oracle.count_triangles(other, 4096)
    do = torch.from_numpy(other).cuda()
    for _ in range(4):
        np.testing.assert_array_equal(tc.count_triangles_batch(d, off, n, graph=True), eager)
        assert tc.count_triangles(do, 4096) == other_T
        torch.cuda.synchronize()


def test_batch_edge_cases(tc):
    import torch
    # empty graphs inside the batch, a graph without pairs at the end
    parts = [graphgen.complete(5), np.zeros((0, 2), np.int32), graphgen.wheel(6), graphgen.cycle(3),
             np.zeros((0, 2), np.int32)]
    nv = np.array([5, 3, 7, 3, 4], dtype=np.int32)
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    np.cumsum([p.shape[0] for p in parts], out=off[1:])
    d = torch.from_numpy(np.concatenate(parts).astype(np.int32)).cuda()
    got = tc.count_triangles_batch(d, off, nv, graph=False)
    np.testing.assert_array_equal(got, np.array([10, 0, 6, 1, 0], dtype=np.uint64))
    # a local id beyond its own graph is an error even if the union has that vertex
    bad = np.array([[0, 1], [1, 2], [0, 3]], dtype=np.int32)
    with pytest.raises(tc.TCError) as ei:
        tc.count_triangles_batch(torch.from_numpy(bad).cuda(), np.array([0, 3, 3]), np.array([3, 4], np.int32),
                                 graph=False)
    assert ei.value.status == 2
    # no pairs at all
    z = tc.count_triangles_batch(torch.zeros((0, 2), dtype=torch.int32, device="cuda:0"), np.zeros(3, np.int64),
                                 np.array([1, 2], np.int32))
    assert z.tolist() == [0, 0]


@pytest.mark.parametrize("sel", ["heuristic", "merge", "bsearch", "bitmap"])
def test_batch_every_strategy(tc, sel):
    import torch
    e, off, n = _small_batch(32, 11)
    ref = _oracle_counts(e, off, n)
    s = {"heuristic": tc.SELECT_HEURISTIC, "merge": tc.FORCE_MERGE, "bsearch": tc.FORCE_BSEARCH,
         "bitmap": tc.FORCE_BITMAP}[sel]
    got = tc.count_triangles_batch(torch.from_numpy(e).cuda(), off, n, select=s, graph=True)
    np.testing.assert_array_equal(got, ref)


def test_tile_shapes_never_change_counts(tc):
    import torch
    n = 1 << 14
    e = graphgen.rmat(14, 16, seed=13)
    ref = oracle.count_triangles(e, n)
    d = torch.from_numpy(e).cuda()
    rng = np.random.default_rng(0)
    for K in (16, 48, 100, 512):
        tc.set_tile_shapes(chunk=np.full(256, K), group=2 ** rng.integers(0, 7, 256))
        for s in (tc.SELECT_HEURISTIC, tc.FORCE_MERGE, tc.FORCE_BSEARCH, tc.FORCE_BITMAP):
            assert tc.count_triangles(d, n, select=s) == ref, (K, s)
    tc.set_tile_shapes(None, None)
