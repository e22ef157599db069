"""Whole-graph parity at the full workload sizes: R-MAT scale 24 (T above 2^32),
the random geometric graph on 2^23 vertices and the batch of 4096 Chung-Lu
graphs.

Expected values are the oracle's (forward algorithm, Section 3.2 / Algorithm 2),
written by tests/golden/make_large_golden.py, which calls only the seeded
generators and the oracle. Vectors too large to store (t[v], the per-edge
intersection sizes, the kept edges) are compared whole through the SHA-256 of
their bytes; on a mismatch the test re-runs the oracle to name the first
differing entries.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "large_counts.json")


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


@pytest.fixture(scope="module")
def gold():
    with open(GOLDEN) as f:
        return json.load(f)


def _sha(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _canonical(pairs, counts):
    """GPU per-edge output (original-id pairs in CSR order) in canonical pair order
    (a << 32 | b, a < b, ascending): (keys uint64, counts uint32) numpy arrays."""
    import torch
    p = pairs.to(torch.int64)
    key = (torch.minimum(p[:, 0], p[:, 1]) << 32) | torch.maximum(p[:, 0], p[:, 1])
    del p
    sk, perm = torch.sort(key)
    c = counts[perm]
    return sk.cpu().numpy().astype("<u8"), c.cpu().numpy().astype("<u4")


def _modes(tc):
    from paper_1804_06926_amd import selector
    modes = [("heuristic", tc.SELECT_HEURISTIC), ("merge", tc.FORCE_MERGE), ("bsearch", tc.FORCE_BSEARCH),
             ("bitmap", tc.FORCE_BITMAP)]
    if selector.load_default():
        modes.insert(1, ("learned", tc.SELECT_LEARNED))
    return modes


def _check_whole(tc, name, e, n, ref):
    import torch
    assert e.shape[0] == ref["raw_pairs"]
    d = torch.from_numpy(e).cuda()
    for mname, sel in _modes(tc):
        print(f"[{name}] T, selection {mname}", flush=True)
        assert tc.count_triangles(d, n, select=sel) == ref["triangles"], mname
    print(f"[{name}] t[v]", flush=True)
    T, t = tc.count_triangles(d, n, per_vertex=True)
    assert T == ref["triangles"]
    t = t.cpu().numpy().astype("<u8")
    assert int(t.sum()) == ref["t_sum"] == 3 * ref["triangles"]
    if _sha(t) != ref["t_sha256_u64le"]:
        _, t_ref = oracle.count_triangles(e, n, per_vertex=True)
        bad = np.nonzero(t != t_ref)[0]
        pytest.fail(f"{name}: t[v] differs at {bad.size} vertices, first {bad[:10].tolist()}")
    print(f"[{name}] per-edge counts, heuristic", flush=True)
    pairs0, counts0, T0 = tc.edge_counts(d, n)
    assert T0 == ref["triangles"] and pairs0.shape[0] == ref["m"]
    keys, c = _canonical(pairs0, counts0)
    assert _sha(keys) == ref["edge_keys_sha256_u64le"], f"{name}: kept edges differ from the oracle's"
    assert int(c.astype(np.uint64).sum()) == ref["edge_counts_sum"]
    if _sha(c) != ref["edge_counts_sha256_u32le"]:
        c_ref = oracle.Graph(e, n).forward_edge_counts(ref["edge_counts_degree"])
        bad = np.nonzero(c != c_ref)[0]
        pytest.fail(f"{name}: per-edge counts differ at {bad.size} edges, first {bad[:10].tolist()}")
    del keys, c
    # the CSR (and so the output order) does not depend on the selection: every other
    # strategy must give the same arrays, entry by entry
    for mname, sel in _modes(tc)[1:]:
        print(f"[{name}] per-edge counts, selection {mname}", flush=True)
        pairs, counts, T1 = tc.edge_counts(d, n, select=sel)
        assert T1 == ref["triangles"], mname
        assert torch.equal(pairs, pairs0), mname
        assert torch.equal(counts, counts0), mname
        del pairs, counts


def test_rmat24_whole_graph(tc, gold):
    """R-MAT scale 24 seed 1: T = 10,287,651,446 (above 2^32) and every t[v] and every
    per-edge count, for every selection mode. The raw draws repeat pairs, so the
    per-edge counts follow the input-pair degree order (the oracle's "input" reading)."""
    ref = gold["rmat24"]
    assert ref["triangles"] > 1 << 32
    _check_whole(tc, "rmat24", graphgen.rmat(24, 16, seed=1), 1 << 24, ref)


def test_rgg23_whole_graph(tc, gold):
    """Random geometric graph, 2^23 vertices, average degree 32, seed 5 (held out from
    selector training): T, every t[v] and every per-edge count, every selection mode."""
    ref = gold["rgg23"]
    _check_whole(tc, "rgg23", graphgen.rgg(1 << 23, 32.0, seed=5), 1 << 23, ref)


def test_chung_lu_batch_4096_every_graph(tc, gold):
    """All 4096 per-graph counts of the batch against the oracle's: captured-graph call,
    its replay, a direct launch, the learned mode, and the shipped autotuned tile shapes."""
    import torch
    from paper_1804_06926_amd import autotune, selector
    ref = np.array(gold["clbatch"]["counts"], dtype=np.uint64)
    print("[batch] generating 4096 Chung-Lu graphs", flush=True)
    e, off, nv = graphgen.chung_lu_batch(4096)
    assert e.shape[0] == gold["clbatch"]["raw_pairs"] and nv.size == ref.size
    d = torch.from_numpy(e).cuda()
    try:
        for tuned in (False, True):
            if tuned:
                assert autotune.apply_cached(tc.SELECT_HEURISTIC), "no shipped tile shapes for this device"
            print(f"[batch] tuned tiles={tuned}: captured graph, replay, direct launch", flush=True)
            np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv), ref)
            np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv), ref)   # replay
            np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv, graph=False), ref)
        if selector.load_default():
            print("[batch] learned selection", flush=True)
            np.testing.assert_array_equal(tc.count_triangles_batch(d, off, nv, select=tc.SELECT_LEARNED), ref)
    finally:
        tc.set_tile_shapes(None, None)


def test_formulations_rmat20_against_oracle(tc):
    """R-MAT 20 through every formulation and strategy: T equal to the oracle's, and
    the sums 3T (full lists), 2T (sum of C) and T."""
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


def test_formulations_rmat24_against_oracle(tc, gold):
    """R-MAT 24 (heuristic selection): every formulation gives the oracle's T, with the
    sums 3T, 2T and T."""
    import torch
    T = gold["rmat24"]["triangles"]
    n = 1 << 24
    d = torch.from_numpy(graphgen.rmat(24, 16, seed=1)).cuda()
    for form, k in (("filtered", 1), ("full", 3), ("matrix", 2), ("matrix_upper", 1)):
        print(f"[rmat24] formulation={form}", flush=True)
        assert tc.count_triangles_formulation(d, n, form) == (T, k * T)
