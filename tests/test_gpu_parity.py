"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Every count is an integer, so every comparison is exact equality.
"""
import os

import numpy as np
import pytest

import graphgen
import oracle
from oracle import stages

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def dev(e):
    import torch
    return torch.from_numpy(np.ascontiguousarray(np.asarray(e, dtype=np.int32).reshape(-1, 2))).to("cuda:0")


def _fig4():
    from tests.conftest import load_golden_matrices
    A = load_golden_matrices("fig4_matrix_example.txt")["A"]
    i, j = np.nonzero(np.triu(A, 1))
    return np.stack([i, j], 1).astype(np.int32), 7


def _dirty(e, n, seed):
    rng = np.random.default_rng(seed)
    k = max(1, e.shape[0] // 7)
    dup = e[rng.integers(0, e.shape[0], k)][:, ::-1]
    loops = np.repeat(rng.integers(0, n, (k // 3 + 1, 1)), 2, axis=1)
    return graphgen.shuffle_edges(np.concatenate([e, dup, loops]).astype(np.int32), seed)


def _repeated(e, n, seed):
    """Three pairs repeated 1500, 3000 and 10000 times: after orientation their rows hold that
    many keys, so the row sort takes its one-wave, whole-block and radix paths."""
    rng = np.random.default_rng(seed)
    pick = e[e[:, 0] != e[:, 1]][rng.integers(0, e.shape[0] // 2, 3)]
    reps = [np.repeat(pick[k:k + 1], c, axis=0) for k, c in enumerate((1500, 3000, 10000))]
    return graphgen.shuffle_edges(np.concatenate([e] + reps).astype(np.int32), seed)


CASES = {
    "fig4": _fig4,
    "repeated_rows": lambda: (_repeated(graphgen.rmat(12, 16, seed=5), 4096, 5), 4096),
    # the same past 2^21 vertices (orientation by partition passes)
    "repeated_rows_22bit": lambda: (_repeated(graphgen.chung_lu(4_100_000, 1_000_000, seed=18), 4_100_000, 18),
                                    4_100_000),
    "k5": lambda: (graphgen.complete(5), 5),
    "k40": lambda: (graphgen.complete(40), 40),
    "bipartite": lambda: (graphgen.complete_bipartite(17, 23), 40),
    "grid": lambda: (graphgen.grid2d(37, 29), 37 * 29),
    "wheel6": lambda: (graphgen.wheel(6), 7),
    "friendship": lambda: (graphgen.friendship(12), 25),
    "tripartite": lambda: (graphgen.complete_tripartite(5, 7, 9), 21),
    "star": lambda: (graphgen.star(3000), 3001),
    "er_4096_32768": lambda: (graphgen.erdos_renyi(4096, 32768, seed=1804), 4096),
    "rmat12_dirty": lambda: (_dirty(graphgen.rmat(12, 16, seed=3), 4096, 3), 4096),
    "chung_lu": lambda: (graphgen.chung_lu(20000, 160000, seed=4), 20000),
    "rgg_16k": lambda: (graphgen.rgg(1 << 14, avg_degree=24, seed=6), 1 << 14),
    "isolated_tail": lambda: (graphgen.complete(30), 5000),
    # ids over 22 bits: the degree count uses its widest LDS buckets (2^14 vertices)
    "sparse_22bit": lambda: (_dirty(graphgen.chung_lu(4_100_000, 2_000_000, seed=12), 4_100_000, 12), 4_100_000),
    # ids of 23 bits: one 8-bit partition pass, buckets of 2^15 vertices (128 KB LDS histogram)
    "sparse_23bit": lambda: (_dirty(graphgen.chung_lu(6_000_000, 1_500_000, seed=17), 6_000_000, 17), 6_000_000),
    # ids of 24 bits: one 8-bit partition pass, buckets of 2^16 vertices counted in two parts
    "sparse_24bit": lambda: (_dirty(graphgen.chung_lu(12_000_000, 1_500_000, seed=16), 12_000_000, 16), 12_000_000),
    # ids over 25 bits: two partition passes, buckets of 2^14 vertices
    "sparse_25bit": lambda: (graphgen.chung_lu(20_000_000, 1_500_000, seed=15), 20_000_000),
    # ids over 12 bits: no partition pass, one bucket counted by several blocks
    "dense_12bit": lambda: (graphgen.erdos_renyi(4000, 300_000, seed=13), 4000),
    # ids over 13 bits: a one-bit partition, two buckets counted by several blocks each
    "dense_13bit": lambda: (graphgen.erdos_renyi(6000, 400_000, seed=14), 6000),
    # short-list buckets of millions of in-edges: edge-centric tiles of up to 2048 in-edges,
    # vertex groups capped by the LDS stage
    "rgg_1m": lambda: (graphgen.rgg(1 << 20, avg_degree=16, seed=61), 1 << 20),
    "uniform_4m": lambda: (np.random.Generator(np.random.PCG64(62)).integers(0, 1 << 18, size=(4 << 20, 2),
                                                                            dtype=np.int32), 1 << 18),
}

SELECTS = ["heuristic", "merge", "bsearch", "bitmap"]


def _sel(tc, name):
    return {"heuristic": tc.SELECT_HEURISTIC, "merge": tc.FORCE_MERGE, "bsearch": tc.FORCE_BSEARCH,
            "bitmap": tc.FORCE_BITMAP}[name]


@pytest.mark.parametrize("sel", SELECTS)
@pytest.mark.parametrize("case", sorted(CASES))
def test_count_and_per_vertex(tc, case, sel):
    e, n = CASES[case]()
    print(f"case={case} select={sel} E={e.shape[0]} n={n}", flush=True)
    ref_T, ref_t = oracle.count_triangles(e, n, per_vertex=True)
    T = tc.count_triangles(dev(e), n, select=_sel(tc, sel))
    assert T == ref_T
    T2, t = tc.count_triangles(dev(e), n, per_vertex=True, select=_sel(tc, sel))
    assert T2 == ref_T
    np.testing.assert_array_equal(t.cpu().numpy().astype(np.uint64), ref_t)


def test_empty_inputs(tc):
    import torch
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda:0")
    assert tc.count_triangles(empty, 0) == 0
    T, t = tc.count_triangles(empty, 9, per_vertex=True)
    assert T == 0 and t.cpu().numpy().tolist() == [0] * 9
    assert tc.count_triangles(dev([[2, 2], [3, 3]]), 4) == 0
    assert tc.count_triangles(dev([[0, 1]]), 2) == 0
    assert tc.count_triangles(dev([[0, 1], [1, 2], [2, 0]]), 3) == 1


def test_vertex_range_error(tc):
    with pytest.raises(tc.TCError) as ei:
        tc.count_triangles(dev([[0, 1], [1, 7]]), 5)
    assert ei.value.status == 2
    with pytest.raises(tc.TCError) as ei:
        tc.count_triangles(dev([[0, 1], [-3, 2]]), 5)
    assert ei.value.status == 2
    # the context stays usable after an error
    assert tc.count_triangles(dev([[0, 1], [1, 2], [2, 0]]), 3) == 1


def test_async_calls_queue_without_waiting(tc):
    """Several asynchronous calls queued back to back on one stream and one
    workspace, each with its own result slot, then one synchronisation: every
    slot holds the oracle's T, the range status is reported on the device, and
    an empty input gives zeros."""
    import torch
    cases = [(graphgen.rmat(s, 16, seed=40 + s), 1 << s) for s in (10, 13, 15)]
    cases.append((graphgen.erdos_renyi(4096, 32768, seed=1804), 4096))
    ws = torch.empty(max(tc.workspace_size(e.shape[0], n) for e, n in cases), dtype=torch.uint8, device="cuda:0")
    res = torch.full((len(cases) + 2, 2), -1, dtype=torch.int64, device="cuda:0")
    pv = torch.full((1 << 15,), -1, dtype=torch.int64, device="cuda:0")
    dev_cases = [(dev(e), n) for e, n in cases]
    for k, (d, n) in enumerate(dev_cases):
        tc.count_triangles_async(d, n, result=res[k], per_vertex=pv if n == 1 << 15 else None, workspace=ws)
    tc.count_triangles_async(dev([[0, 1], [1, 9]]), 5, result=res[len(cases)], workspace=ws)
    tc.count_triangles_async(torch.zeros((0, 2), dtype=torch.int32, device="cuda:0"), 3, result=res[-1],
                             workspace=ws)
    torch.cuda.synchronize()
    got = res.cpu().numpy()
    for k, (e, n) in enumerate(cases):
        assert got[k].tolist() == [oracle.count_triangles(e, n), 0], k
    assert got[len(cases)][1] == 2
    assert got[-1].tolist() == [0, 0]
    _, ref_t = oracle.count_triangles(cases[2][0], cases[2][1], per_vertex=True)
    np.testing.assert_array_equal(pv.cpu().numpy().astype(np.uint64), ref_t)


@pytest.mark.parametrize("case", ["fig4", "k40", "wheel6", "friendship", "star", "rmat12_dirty", "chung_lu",
                                  "rgg_16k", "isolated_tail"])
def test_clustering_matches_oracle(tc, case):
    """Each coefficient and the transitivity are one correctly rounded float64
    division of the same exact integers on both sides, so they agree exactly."""
    from oracle.measures import clustering
    e, n = CASES[case]()
    print(f"case={case} E={e.shape[0]} n={n}", flush=True)
    r_coeff, r_T, r_W, r_tr, r_t = clustering(e, n)
    coeff, T, W, tr, t = tc.clustering(dev(e), n, per_vertex=True)
    assert (T, W, tr) == (r_T, r_W, r_tr)
    np.testing.assert_array_equal(coeff.cpu().numpy(), r_coeff)
    np.testing.assert_array_equal(t.cpu().numpy().astype(np.uint64), r_t)
    # without the per-vertex output requested
    coeff2, T2, W2, tr2 = tc.clustering(dev(e), n, select=tc.FORCE_BITMAP)
    assert (T2, W2, tr2) == (r_T, r_W, r_tr)
    np.testing.assert_array_equal(coeff2.cpu().numpy(), r_coeff)


def test_clustering_empty(tc):
    import torch
    coeff, T, W, tr = tc.clustering(torch.zeros((0, 2), dtype=torch.int32, device="cuda:0"), 5)
    assert (T, W, tr) == (0, 0, 0.0) and coeff.cpu().numpy().tolist() == [0.0] * 5


def _canon_keys(pairs):
    a = pairs[:, 0].astype(np.int64)
    b = pairs[:, 1].astype(np.int64)
    return (np.minimum(a, b) << 32) | np.maximum(a, b)


@pytest.mark.parametrize("sel", SELECTS)
def test_per_edge_counts_match_oracle(tc, sel):
    n = 1 << 13
    e = _dirty(graphgen.rmat(13, 16, seed=21), n, 21)
    g = oracle.Graph(e, n)
    # the input has repeated pairs: the GPU orders by input-pair degree
    ref = g.oriented_edge_counts(degree="input")
    ref_keys = _canon_keys(g.edges())
    pairs, counts, T = tc.edge_counts(dev(e), n, select=_sel(tc, sel))
    pairs = pairs.cpu().numpy()
    counts = counts.cpu().numpy().astype(np.int64)
    assert pairs.shape[0] == g.m
    keys = _canon_keys(pairs)
    o = np.argsort(keys)
    np.testing.assert_array_equal(keys[o], ref_keys)
    np.testing.assert_array_equal(counts[o], ref.astype(np.int64))
    assert T == g.count() == int(counts.sum())
    # orientation: u before v in (input degree, id) order
    deg = stages.input_degrees(e, n)
    u, v = pairs[:, 0], pairs[:, 1]
    assert np.all((deg[u] < deg[v]) | ((deg[u] == deg[v]) & (u < v)))


@pytest.mark.parametrize("sel", SELECTS)
@pytest.mark.parametrize("case", ["fig4", "k40", "wheel6", "friendship", "rmat12_dirty", "chung_lu", "rgg_16k",
                                  "er_4096_32768"])
def test_edge_support_matches_oracle(tc, case, sel):
    """Support of every kept edge (triangles containing it) against the oracle,
    matched by canonical pair: the edge set is unique, the order may differ."""
    e, n = CASES[case]()
    print(f"case={case} select={sel} E={e.shape[0]} n={n}", flush=True)
    g = oracle.Graph(e, n)
    ref = g.edge_support()
    ref_keys = _canon_keys(g.edges())
    pairs, sup, T = tc.edge_support(dev(e), n, select=_sel(tc, sel))
    keys = _canon_keys(pairs.cpu().numpy())
    o = np.argsort(keys)
    np.testing.assert_array_equal(keys[o], ref_keys)
    np.testing.assert_array_equal(sup.cpu().numpy()[o].astype(np.uint32), ref)
    assert T == g.count() and int(ref.astype(np.int64).sum()) == 3 * T


@pytest.mark.parametrize("sel", SELECTS)
@pytest.mark.parametrize("case", ["fig4", "k40", "wheel6", "friendship", "tripartite", "rmat12_dirty", "chung_lu",
                                  "rgg_16k", "er_4096_32768", "bipartite"])
def test_list_triangles(tc, case, sel):
    """The listed triples are exactly the triangles: as many as the oracle counts,
    each one a triangle of the simple graph, no two the same; each ordered
    u before v before w in (input degree, id) order and grouped by edge (u, v)."""
    e, n = CASES[case]()
    print(f"case={case} select={sel} E={e.shape[0]} n={n}", flush=True)
    g = oracle.Graph(e, n)
    T = g.count()
    tri = tc.list_triangles(dev(e), n, select=_sel(tc, sel)).cpu().numpy().astype(np.int64)
    assert tri.shape == (T, 3)
    if T == 0:
        return
    keys = set(_canon_keys(g.edges()).tolist())
    u, v, w = tri[:, 0], tri[:, 1], tri[:, 2]
    for a_, b_ in ((u, v), (v, w), (u, w)):
        assert (a_ != b_).all()
        assert all(k in keys for k in _canon_keys(np.stack([a_, b_], 1)).tolist())
    srt = np.sort(tri, axis=1)
    assert np.unique(srt, axis=0).shape[0] == T
    deg = stages.input_degrees(e, n).astype(np.int64)
    ku, kv, kw = deg[u] * n + u, deg[v] * n + v, deg[w] * n + w
    assert (ku < kv).all() and (kv < kw).all()
    pair = u * n + v
    change = np.nonzero(np.diff(pair))[0]
    starts = np.concatenate([[0], change + 1])
    assert np.unique(pair[starts]).shape[0] == starts.shape[0]   # each edge's triangles are contiguous


def test_list_triangles_empty(tc):
    import torch
    assert tc.list_triangles(torch.zeros((0, 2), dtype=torch.int32, device="cuda:0"), 4).shape == (0, 3)
    assert tc.list_triangles(dev(graphgen.star(20)), 21).shape == (0, 3)


def test_csr_export_matches_definition(tc):
    n = 1 << 12
    e = _dirty(graphgen.rmat(12, 16, seed=5), n, 5)
    rank, off, col = tc.build_csr(dev(e), n)
    r_rank, r_off, r_col, _ = stages.oriented_csr(e, n, degree="input")
    np.testing.assert_array_equal(rank.cpu().numpy(), r_rank)
    np.testing.assert_array_equal(off.cpu().numpy(), r_off)
    np.testing.assert_array_equal(col.cpu().numpy(), r_col)


@pytest.mark.parametrize("count,bits", [(c, b) for c in (1, 2047, 2048, 2049, 4097, 100003)
                                        for b in ((0, 64), (0, 20), (32, 45), (7, 13))]
                         # either side of the switch from 2048- to 4096-key tiles (2^22 keys)
                         + [((1 << 22) - 1, (0, 20)), ((1 << 22) + 4097, (0, 64))]
                         # more than 8192 tiles of 4096 keys (several digit-row segments), ragged last tile
                         + [(8 * 1024 * 4096 + 4096 * 5 + 77, (0, 64)), (8 * 1024 * 4096 + 4096 * 5 + 77, (7, 13))]
                         # 8192-key tiles of 64-bit sorts from 2^26 keys: more than 8192 of them, ragged
                         + [((1 << 26) + 8192 * 3 + 77, (0, 64))]
                         # two to four passes at that size: the passes after the first look back
                         # over the tiles before them instead of reading a count table
                         + [((1 << 26) + 8192 * 3 + 77, (0, 32)), ((1 << 26) + 8192 * 3 + 77, (7, 29)),
                            ((1 << 26) + 5, (40, 56))])
def test_radix_sort_is_stable_and_exact(tc, count, bits):
    import torch
    rng = np.random.default_rng(count + bits[0])
    keys = rng.integers(0, 2**63, count, dtype=np.int64)
    keys[: count // 3] &= 0xFFFF   # many equal digits (one dominant digit in the upper passes)
    d = torch.from_numpy(keys.copy()).to("cuda:0")
    tc.radix_sort_u64(d, bits[0], bits[1])
    lo, hi = bits
    u = keys.view(np.uint64)
    digit = (u >> np.uint64(lo)) & np.uint64((1 << (hi - lo)) - 1 if hi - lo < 64 else 0xFFFFFFFFFFFFFFFF)
    ref = keys[np.argsort(digit, kind="stable")]
    np.testing.assert_array_equal(d.cpu().numpy(), ref)


@pytest.mark.parametrize("count,shift,bits,dist",
                         [(c, sh, b, "mixed") for c in (1, 2047, 2049, 100003) for sh, b in ((0, 8), (7, 6), (56, 8), (3, 1))]
                         + [(100003, 32, 8, "equal"), (4097, 0, 8, "equal"), (100003, 40, 8, "skewed"),
                            # 4096-key tiles (from 2^22 keys) and 8192-key tiles (from 2^26), ragged last tiles
                            ((1 << 22) + 4097, 24, 8, "mixed"), ((1 << 26) + 8192 * 3 + 77, 0, 8, "mixed"),
                            ((1 << 26) + 8192 * 3 + 77, 40, 8, "skewed")])
def test_radix_partition_groups_by_digit(tc, count, shift, bits, dist):
    """tc_radix_partition_u64 (the builder's partitioning pass, ranks by LDS atomics): the output is a
    permutation of the input whose digits never decrease, so every key lies in its digit's group,
    the groups in ascending order; what is unique (the digit sequence and the multiset) is
    compared with a sort on the CPU, the order inside a group is not."""
    import torch
    rng = np.random.default_rng(count + 31 * shift + bits)
    keys = rng.integers(0, 2**63, count, dtype=np.int64) * 2 + rng.integers(0, 2, count)
    if dist == "mixed":
        keys[: count // 3] &= 0xFFFF   # a third with high digits zero
    elif dist == "equal":
        keys[:] = keys[0]              # every lane of every wave on one counter
    elif dist == "skewed":             # nine in ten keys on one digit, the rest spread
        keys[rng.random(count) < 0.9] &= ~np.int64(((1 << bits) - 1) << shift)
    out = tc.radix_partition_u64(torch.from_numpy(keys.copy()).to("cuda:0"), shift, bits).cpu().numpy()
    u, o = keys.view(np.uint64), out.view(np.uint64)
    mask = np.uint64((1 << bits) - 1)
    np.testing.assert_array_equal(np.sort((o >> np.uint64(shift)) & mask), (o >> np.uint64(shift)) & mask)
    np.testing.assert_array_equal(np.sort((u >> np.uint64(shift)) & mask), (o >> np.uint64(shift)) & mask)
    np.testing.assert_array_equal(np.sort(o), np.sort(u))


def test_radix_partition_rejects_bad_arguments(tc):
    import torch
    k = torch.zeros(16, dtype=torch.int64, device="cuda:0")
    for shift, bits in ((0, 0), (0, 9), (60, 8), (-1, 4)):
        with pytest.raises(tc.TCError) as ei:
            tc.radix_partition_u64(k, shift, bits)
        assert ei.value.status == 1   # TC_ERR_INVALID_ARG
    assert tc.radix_partition_u64(k[:0], 0, 8).numel() == 0


def _run_lengths(kind, rng):
    if kind == "singletons":
        return [1] * 5000
    if kind == "short":
        return rng.integers(1, 65, 3000).tolist()
    if kind == "windows":        # spans of short runs past 64 slots
        return rng.integers(1, 130, 1500).tolist()
    if kind == "edges":          # either side of every length class
        return [64, 65, 2048, 2049, 1, 2, 127, 128, 4095, 4096, 4097, 63, 1, 8192, 3]
    if kind == "huge":           # one run over many tiles, between short ones
        return rng.integers(1, 40, 200).tolist() + [300_000] + rng.integers(1, 300, 200).tolist()
    if kind == "overflow":       # a 2048-key run from the last position of a tile: its overflow
        return ([1] * 4095 + [2048]) * 3 + [2000, 1, 2048]   # reaches the end of the block's LDS span
    if kind == "powerlaw":       # row lengths like a degree-ordered R-MAT out-list
        return np.minimum((rng.pareto(1.2, 120_000) * 4 + 1).astype(np.int64), 5000).tolist()
    raise ValueError(kind)


@pytest.mark.parametrize("shift,kind", [(24, "singletons"), (24, "short"), (24, "windows"), (24, "edges"),
                                        (20, "huge"), (24, "powerlaw"), (32, "powerlaw"), (7, "windows"),
                                        (1, "edges"), (13, "short"), (24, "one"), (24, "overflow"),
                                        (32, "overflow")])
def test_sort_runs_sorts_every_run(tc, shift, kind):
    """tc_sort_runs_u64 on keys grouped by their high bits gives np.sort of them (runs of every length
    class, duplicates inside runs, ragged last tile)."""
    import torch
    rng = np.random.default_rng(shift * 7 + len(kind))
    lens = np.asarray([1] if kind == "one" else _run_lengths(kind, rng), dtype=np.int64)
    high = np.cumsum(rng.integers(1, 4, lens.size)).astype(np.uint64)
    hv = np.repeat(high, lens)
    low = rng.integers(0, 1 << shift, hv.size, dtype=np.uint64)
    few = np.repeat(rng.random(lens.size) < 0.3, lens)   # some runs with many repeated keys
    low[few] %= np.uint64(5)
    keys = (hv << np.uint64(shift)) | low
    d = torch.from_numpy(keys.view(np.int64).copy()).to("cuda:0")
    tc.sort_runs_u64(d, shift)
    np.testing.assert_array_equal(d.cpu().numpy().view(np.uint64), np.sort(keys))


def test_per_edge_counts_clean_input_simple_degree(tc):
    """Without repeated pairs, input degree and simple degree coincide."""
    n = 1 << 12
    g0 = oracle.Graph(graphgen.rmat(12, 8, seed=31), n)
    e = graphgen.shuffle_edges(g0.edges(), 4)
    g = oracle.Graph(e, n)
    ref = g.oriented_edge_counts(degree="simple")
    pairs, counts, T = tc.edge_counts(dev(e), n)
    keys = _canon_keys(pairs.cpu().numpy())
    o = np.argsort(keys)
    np.testing.assert_array_equal(keys[o], _canon_keys(g.edges()))
    np.testing.assert_array_equal(counts.cpu().numpy()[o].astype(np.int64), ref.astype(np.int64))


def test_rmat20_all_kernels_agree_per_edge(tc):
    """R-MAT scale 20 (edge factor 16): oracle total and per-vertex counts; the three
    intersection strategies forced one at a time agree edge by edge."""
    n = 1 << 20
    e = graphgen.rmat(20, 16, seed=1)
    print(f"rmat20 E={e.shape[0]}", flush=True)
    ref_T, ref_t = oracle.count_triangles(e, n, per_vertex=True)
    d = dev(e)
    T, t = tc.count_triangles(d, n, per_vertex=True)
    assert T == ref_T
    np.testing.assert_array_equal(t.cpu().numpy().astype(np.uint64), ref_t)
    base = None
    for sel in ("merge", "bsearch", "bitmap"):
        pairs, counts, T2 = tc.edge_counts(d, n, select=_sel(tc, sel))
        assert T2 == ref_T
        cur = (pairs.cpu().numpy(), counts.cpu().numpy())
        if base is None:
            base = cur
        else:
            np.testing.assert_array_equal(cur[0], base[0])
            np.testing.assert_array_equal(cur[1], base[1])


# ---------------------------------------------------------------- the other formulations
FORM_CASES = sorted(CASES) + ["spread_hubs", "rmat18"]
_form_ref = {}


def _form_case(case):
    if case == "spread_hubs":
        return graphgen.spread_hubs(), 1 << 21
    if case == "rmat18":
        return graphgen.rmat(18, 16, seed=9), 1 << 18
    return CASES[case]()


def _form_oracle(case, e, n):
    """(T, full sum, sum of C, upper sum of C) from the oracle, once per case."""
    if case not in _form_ref:
        G = oracle.Graph(e, n)
        _form_ref[case] = (G.count(), G.full_sum(), G.matrix_sum(), G.matrix_sum(upper=True))
    return _form_ref[case]


@pytest.mark.parametrize("sel", SELECTS)
@pytest.mark.parametrize("case", FORM_CASES)
def test_formulations_match_oracle(tc, case, sel):
    """Full lists (sum 3T), Algorithm 3 (sum of C = 2T), its upper-triangle
    form (T) and the filtered form, each against the oracle's own sums."""
    e, n = _form_case(case)
    T, full, mat, upper = _form_oracle(case, e, n)
    d = dev(e)
    for form, want in (("filtered", T), ("full", full), ("matrix", mat), ("matrix_upper", upper)):
        print(f"case={case} select={sel} formulation={form} E={e.shape[0]} n={n}", flush=True)
        got = tc.count_triangles_formulation(d, n, form, select=_sel(tc, sel))
        assert got == (T, want), form


def test_formulations_empty_and_errors(tc):
    import torch
    empty = torch.zeros((0, 2), dtype=torch.int32, device="cuda:0")
    for form in tc.FORMULATIONS:
        assert tc.count_triangles_formulation(empty, 4, form) == (0, 0)
        assert tc.count_triangles_formulation(dev([[1, 1], [2, 2]]), 3, form) == (0, 0)
        assert tc.count_triangles_formulation(dev([[0, 1], [1, 2], [2, 0]]), 3, form)[0] == 1
        with pytest.raises(tc.TCError) as ei:
            tc.count_triangles_formulation(dev([[0, 1], [1, 6]]), 4, form)
        assert ei.value.status == 2
    with pytest.raises(ValueError):
        tc.count_triangles_formulation(dev([[0, 1]]), 2, "dense")


# ---------------------------------------------------------------- merge-path diagonal splits
def _straddles(L, g):
    """Lane boundaries k (1..g-1) at which the merge-path split of two equal lists of
    length L falls between the equal pair a_i = b_i. With A = B the merge (A first on
    ties) is a0 b0 a1 b1 ..., so the boundary at diagonal d = floor(2 L k / g) separates
    a pair exactly when d is odd."""
    return {k for k in range(1, g) if ((2 * L * k) // g) % 2 == 1}


@pytest.mark.parametrize("n", [130, 4200])
def test_merge_path_matches_split_at_every_lane_boundary(tc, n):
    """K_n (all degrees n - 1, so rank = id): every in-edge (u -> v) has the tail
    {v+1 .. n-1} = N+(v), two equal lists of every length 1 .. n - 2. For each group
    size g = 2 .. 64 (forced through the tile shapes on every bucket) the host first
    checks that some list length puts an equal pair across every lane boundary
    k = 1 .. g - 1; the forced merge-path kernel must then give T = C(n, 3) and every
    per-edge count c(u -> v) = n - 1 - v. n = 4200 makes the middle lists longer than
    the kernel's LDS stage, so the unstaged call site is covered as well."""
    import torch
    from math import comb
    e = graphgen.complete(n)
    d = dev(e)
    if n <= 200:
        assert oracle.count_triangles(e, n) == comb(n, 3)
    try:
        for g in (1, 2, 4, 8, 16, 32, 64):
            covered = set().union(*(_straddles(L, g) for L in range(1, n - 1)))
            assert covered == set(range(1, g)), (g, sorted(set(range(1, g)) - covered))
            tc.set_tile_shapes(group=np.full(256, g))
            print(f"K_{n}: merge path, {g} lanes per in-edge", flush=True)
            assert tc.count_triangles(d, n, select=tc.FORCE_MERGE) == comb(n, 3), g
            pairs, counts, T = tc.edge_counts(d, n, select=tc.FORCE_MERGE)
            p = pairs.cpu().numpy()
            assert np.all(p[:, 0] < p[:, 1])   # rank = id
            np.testing.assert_array_equal(counts.cpu().numpy(), n - 1 - p[:, 1])
    finally:
        tc.set_tile_shapes(None, None)


# ---------------------------------------------------------------- dynamic grouping (buckets)
@pytest.mark.parametrize("case,degree", [("k40", "simple"), ("rmat12_dirty", "input"), ("chung_lu", "input"),
                                         ("rgg_16k", "simple"), ("er_4096_32768", "simple")])
def test_bucket_statistics_match_oracle(tc, case, degree):
    """Per-bucket vertices, in-edges with work, out-edges and work (the grouping of the
    middle vertices, Section 4.2) equal the oracle's stage definition on its own
    degree-ordered CSR. Inputs with repeated pairs (the R-MAT and Chung-Lu draws) are
    oriented by the input-pair degree, as the library orients them."""
    e, n = CASES[case]()
    rank, off, col, src = stages.oriented_csr(e, n, degree=degree)
    ref = stages.bucket_totals(off, col)
    tc.count_triangles(dev(e), n)
    st = tc.last_stats()
    np.testing.assert_array_equal(st["bucket_vertices"][:255].astype(np.int64), ref["vertices"][:255])
    np.testing.assert_array_equal(st["bucket_in_edges"][:255].astype(np.int64), ref["in_edges"][:255])
    np.testing.assert_array_equal(st["bucket_out_edges"][:255].astype(np.int64), ref["out_edges"][:255])
    np.testing.assert_array_equal(st["bucket_work"][:255].astype(np.int64), ref["work"][:255])
    busy = np.nonzero(ref["vertices"][:255])[0]
    feat = tc.bucket_features()
    np.testing.assert_allclose(feat[busy, 2], np.log2(1.0 + ref["windows"][busy]).astype(np.float32) / 32.0,
                               rtol=1e-6)
