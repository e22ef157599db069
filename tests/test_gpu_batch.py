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


def test_autotuner_end_to_end_on_a_small_batch(tc, tmp_path):
    """The tile-shape autotuner run for real: tune on the union of a small batch (every
    busy bucket timed at each candidate size through tc_profile_selected), save the
    result to a cache file, install it from there, and count the batch with it: every
    per-graph count equals the oracle's, replayed and launched directly."""
    import torch
    from paper_1804_06926_amd import autotune
    e, off, nv = graphgen.chung_lu_batch(96, 1e3, 5e4, seed=19)
    ref = _oracle_counts(e, off, nv)
    base = np.zeros(nv.size, dtype=np.int64)
    np.cumsum(nv[:-1].astype(np.int64), out=base[1:])
    union = e + np.repeat(base, np.diff(off)).astype(np.int32)[:, None]
    N = int(nv.astype(np.int64).sum())
    du = torch.from_numpy(np.ascontiguousarray(union)).cuda()
    best, table = autotune.tune(du, N, repeats=2, candidates=(32, 128, 512))
    busy = np.nonzero(tc.last_stats()["bucket_vertices"][:255])[0]
    assert busy.size > 0
    for b in busy:   # every busy bucket was timed at every size and got one of them
        assert np.all(table[:, b] > 0), b
        assert best[b] in (32, 128, 512), (b, best[b])
    assert np.all(best[[b for b in range(256) if b not in set(busy.tolist())]] == 0)
    cache = str(tmp_path / "shapes.json")
    key = autotune.device_key(tc.SELECT_HEURISTIC)
    autotune.save(best, key, cache)
    np.testing.assert_array_equal(autotune.load(key, cache), best)
    d = torch.from_numpy(e).cuda()
    try:
        assert autotune.apply_cached(tc.SELECT_HEURISTIC, path=cache)
        np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv), ref)
        np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv), ref)
        np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv, graph=False), ref)
        st = tc.last_stats()
        for b in busy:   # the tuned sizes are the ones the layout used (bitmap tiles cap at 512)
            if st["bucket_vertices"][b]:
                assert st["bucket_chunk"][b] == best[b], (b, st["bucket_chunk"][b], best[b])
    finally:
        tc.set_tile_shapes(None, None)


def test_captured_graph_serves_other_batches_of_the_same_sizes(tc):
    """The captured graph is keyed on the batch's totals (pairs, vertices, graphs), the
    selection and the workspace; the edge list's address and the per-graph offsets
    reach the device before each launch. Batches with other contents, at another
    address, and with the same totals split differently between the graphs, replay it
    and still give the oracle's per-graph counts."""
    import torch
    G = 24
    rng = np.random.default_rng(8)
    nv = rng.integers(40, 400, size=G).astype(np.int32)
    E = (nv.astype(np.int64) * rng.integers(3, 9, size=G)).astype(np.int64)

    def batch(nv, E, seed):
        off = np.zeros(G + 1, dtype=np.int64)
        np.cumsum(E, out=off[1:])
        e = np.concatenate([graphgen.chung_lu(int(nv[g]), int(E[g]), seed=seed + g) for g in range(G)])
        return e.astype(np.int32), off, nv

    # same sizes, other contents; then the same totals split differently
    nv2, E2 = nv[::-1].copy(), E[::-1].copy()
    batches = [batch(nv, E, 100), batch(nv, E, 500), batch(nv2, E2, 900), batch(nv, E, 100)]
    for i, (e, off, n) in enumerate(batches):
        ref = _oracle_counts(e, off, n)
        d = torch.from_numpy(e).cuda()   # a new buffer each time
        np.testing.assert_array_equal(tc.count_triangles_batch(d, off, n, graph=True), ref, err_msg=str(i))
        del d
