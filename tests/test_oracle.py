"""Pins for the CPU oracle: it is checked against things other than itself.

Each check ties the forward-algorithm oracle to an independent fact: the
paper's worked example, brute force over vertex triples, the trace of A^3,
closed forms of structured graphs, invariances of the exact count, and
third-party libraries run as black boxes (networkx, scipy.sparse).
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import dense, stages
from tests.conftest import load_golden_matrices


def _count(e, n, **kw):
    return oracle.count_triangles(e, n, **kw)


# ---------------------------------------------------------------- Figure 4
def test_fig4_matrix_formulation_reproduces_printed_matrices():
    g = load_golden_matrices("fig4_matrix_example.txt")
    T, L, U, B, C = dense.masked_product(g["A"])
    np.testing.assert_array_equal(L, g["L"])
    np.testing.assert_array_equal(U, g["U"])
    np.testing.assert_array_equal(B, g["B"])
    np.testing.assert_array_equal(C, g["C"])
    assert T == int(g["T"][0, 0]) == 3


def test_fig4_forward_oracle_and_brute_force():
    A = load_golden_matrices("fig4_matrix_example.txt")["A"]
    i, j = np.nonzero(np.triu(A, 1))
    e = np.stack([i, j], 1).astype(np.int32)
    assert e.shape[0] == 10
    T, t = _count(e, 7, per_vertex=True)
    Tb, tb = dense.brute_force(e, 7)
    assert T == Tb == 3
    np.testing.assert_array_equal(t, tb)
    for order in (oracle.ORDER_DEG_ID, oracle.ORDER_PAPER, oracle.ORDER_ID):
        assert _count(e, 7, order=order) == 3


# ---------------------------------------------------------------- brute force
@pytest.mark.parametrize("seed", range(6))
def test_brute_force_random_small(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(3, 40))
    p = [0.05, 0.2, 0.5, 0.9][seed % 4]
    A = np.triu(rng.random((n, n)) < p, 1)
    i, j = np.nonzero(A)
    e = np.stack([i, j], 1).astype(np.int32)
    T, t = _count(e, n, per_vertex=True)
    Tb, tb = dense.brute_force(e, n)
    assert T == Tb
    np.testing.assert_array_equal(t, tb)


def test_empty_and_trivial():
    assert _count(np.zeros((0, 2), np.int32), 0) == 0
    assert _count(np.zeros((0, 2), np.int32), 10) == 0
    assert _count(np.array([[0, 1]], np.int32), 2) == 0
    assert _count(np.array([[3, 3]], np.int32), 4) == 0
    T, t = _count(np.array([[0, 1], [1, 2], [2, 0]], np.int32), 5, per_vertex=True)
    assert T == 1 and t.tolist() == [1, 1, 1, 0, 0]


def test_vertex_range_error():
    with pytest.raises(oracle.VertexRangeError):
        oracle.Graph(np.array([[0, 5]], np.int32), 5)
    with pytest.raises(oracle.VertexRangeError):
        oracle.Graph(np.array([[-1, 2]], np.int32), 5)


# ---------------------------------------------------------------- closed forms
@pytest.mark.parametrize("n", [3, 4, 5, 17, 64])
def test_complete_graph(n):
    T, t = _count(graphgen.complete(n), n, per_vertex=True)
    assert T == math.comb(n, 3)
    assert np.all(t == math.comb(n - 1, 2))


@pytest.mark.parametrize("a,b", [(1, 1), (3, 5), (20, 31)])
def test_complete_bipartite_is_triangle_free(a, b):
    assert _count(graphgen.complete_bipartite(a, b), a + b) == 0


def test_grid_and_long_cycles_are_triangle_free():
    assert _count(graphgen.grid2d(30, 41), 30 * 41) == 0
    for k in (4, 5, 9, 100):
        assert _count(graphgen.cycle(k), k) == 0
    assert _count(graphgen.cycle(3), 3) == 1


@pytest.mark.parametrize("k", [4, 5, 6, 50])
def test_wheel(k):
    T, t = _count(graphgen.wheel(k), k + 1, per_vertex=True)
    assert T == k
    assert t[0] == k and np.all(t[1:] == 2)


def test_wheel_with_three_rim_vertices_is_k4():
    assert _count(graphgen.wheel(3), 4) == 4


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (2, 3, 4), (7, 5, 9)])
def test_complete_tripartite(a, b, c):
    assert _count(graphgen.complete_tripartite(a, b, c), a + b + c) == a * b * c


@pytest.mark.parametrize("k", [1, 2, 10])
def test_friendship(k):
    T, t = _count(graphgen.friendship(k), 2 * k + 1, per_vertex=True)
    assert T == k and t[0] == k and np.all(t[1:] == 1)


def test_star_is_triangle_free():
    assert _count(graphgen.star(1000), 1001) == 0


# ---------------------------------------------------------------- trace(A^3)
@pytest.mark.parametrize("maker", ["er", "rmat", "dense"])
def test_trace_of_cube(maker):
    if maker == "er":
        n, e = 600, graphgen.erdos_renyi(600, 6000, seed=3)
    elif maker == "rmat":
        n, e = 512, graphgen.rmat(9, 16, seed=4)
    else:
        n = 200
        rng = np.random.default_rng(5)
        i, j = np.nonzero(np.triu(rng.random((n, n)) < 0.6, 1))
        e = np.stack([i, j], 1).astype(np.int32)
    T, t = _count(e, n, per_vertex=True)
    Tt, tt = dense.trace_count(e, n)
    assert T == Tt
    np.testing.assert_array_equal(t, tt)
    assert int(t.sum()) == 3 * T


# ---------------------------------------------------------------- invariances
def _rmat_small(scale=11, seed=9):
    return graphgen.rmat(scale, 16, seed=seed), 1 << scale


def test_relabel_shuffle_flip_duplicates_loops_isolated():
    e, n = _rmat_small()
    T, t = _count(e, n, per_vertex=True)
    assert T > 0
    rng = np.random.default_rng(1)
    p = rng.permutation(n).astype(np.int32)
    T2, t2 = _count(p[e], n, per_vertex=True)
    assert T2 == T
    np.testing.assert_array_equal(t2[p], t)
    assert _count(graphgen.shuffle_edges(e, 77), n) == T
    dirty = np.concatenate([e, e[::3, ::-1], np.stack([np.arange(50), np.arange(50)], 1).astype(np.int32)])
    assert _count(graphgen.shuffle_edges(dirty, 5), n) == T
    T3, t3 = _count(e, n + 1000, per_vertex=True)
    assert T3 == T and np.all(t3[n:] == 0)


def test_orientation_independence():
    e, n = _rmat_small(12, 3)
    res = {o: _count(e, n, per_vertex=True, order=o) for o in (0, 1, 2)}
    assert res[0][0] == res[1][0] == res[2][0]
    np.testing.assert_array_equal(res[0][1], res[1][1])
    np.testing.assert_array_equal(res[0][1], res[2][1])


def test_disjoint_union_is_additive():
    e1, n1 = _rmat_small(10, 1)
    e2 = graphgen.chung_lu(3000, 20000, seed=2)
    n2 = 3000
    T1, T2 = _count(e1, n1), _count(e2, n2)
    u = np.concatenate([e1, e2 + n1])
    assert _count(u, n1 + n2) == T1 + T2


def test_thread_count_does_not_change_result():
    e, n = _rmat_small(14, 2)
    T1, t1 = oracle.count_triangles(e, n, per_vertex=True, threads=1)
    T8, t8 = oracle.count_triangles(e, n, per_vertex=True, threads=8)
    assert T1 == T8
    np.testing.assert_array_equal(t1, t8)


# ---------------------------------------------------------------- definition-level functions
def test_vertex_triangles_definition_matches_forward():
    e, n = _rmat_small(13, 6)
    g = oracle.Graph(e, n)
    T, t = g.count(per_vertex=True)
    np.testing.assert_array_equal(g.vertex_triangles(np.arange(n)), t)


def test_oriented_edge_counts_match_sets_and_sum_to_T():
    e, n = _rmat_small(10, 8)
    g = oracle.Graph(e, n)
    c = g.oriented_edge_counts()
    assert int(c.sum()) == g.count()
    rank, off, col, src = stages.oriented_csr(e, n)
    ref = stages.oriented_counts(off, col, src)
    inv = np.empty(n, dtype=np.int64)
    inv[rank] = np.arange(n)
    a, b = inv[src], inv[col]
    keys = (np.minimum(a, b) << 32) | np.maximum(a, b)
    o = np.argsort(keys)
    np.testing.assert_array_equal(c, ref[o])


def test_oriented_counts_input_degree_mode():
    e, n = _rmat_small(10, 8)
    dirty = np.concatenate([e, e[: e.shape[0] // 4, ::-1]]).astype(np.int32)
    g = oracle.Graph(dirty, n)
    c = g.oriented_edge_counts(degree="input")
    assert int(c.sum()) == g.count()
    rank, off, col, src = stages.oriented_csr(dirty, n, degree="input")
    ref = stages.oriented_counts(off, col, src)
    inv = np.empty(n, dtype=np.int64)
    inv[rank] = np.arange(n)
    a, b = inv[src], inv[col]
    o = np.argsort((np.minimum(a, b) << 32) | np.maximum(a, b))
    np.testing.assert_array_equal(c, ref[o])
    # clean input: both degree definitions agree
    g2 = oracle.Graph(e, n)
    assert np.array_equal(g2.oriented_edge_counts("simple"), oracle.Graph(g2.edges(), n).oriented_edge_counts("input"))


def test_pair_counts_match_full_oriented_counts():
    e, n = _rmat_small(11, 12)
    dirty = np.concatenate([e, e[::5, ::-1]]).astype(np.int32)
    g = oracle.Graph(dirty, n)
    for mode in ("simple", "input"):
        full = g.oriented_edge_counts(mode)
        pe = g.edges()
        rng = np.random.default_rng(1)
        idx = rng.choice(g.m, 500, replace=False)
        q = pe[idx][:, ::-1].copy()   # reversed order must not matter
        np.testing.assert_array_equal(g.pair_counts(q, mode), full[idx])
    assert g.pair_counts(np.array([[0, 0]]))[0] == 0


def test_edge_support():
    e, n = _rmat_small(9, 10)
    g = oracle.Graph(e, n)
    s = g.edge_support()
    assert int(s.sum()) == 3 * g.count()
    A = dense.adjacency(e, n)
    A2 = A @ A
    pe = g.edges()
    np.testing.assert_array_equal(s, A2[pe[:, 0], pe[:, 1]])


# ---------------------------------------------------------------- third-party libraries as black boxes
def test_networkx_triangles():
    nx = pytest.importorskip("networkx")
    e = graphgen.chung_lu(20000, 120000, seed=12)
    n = 20000
    G = nx.Graph()
    G.add_nodes_from(range(n))
    G.add_edges_from((int(a), int(b)) for a, b in e if a != b)
    tri = nx.triangles(G)
    ref = np.array([tri[v] for v in range(n)], dtype=np.uint64)
    T, t = _count(e, n, per_vertex=True)
    np.testing.assert_array_equal(t, ref)
    assert T == int(ref.sum()) // 3


def test_scipy_sparse_matrix_formulation():
    sp = pytest.importorskip("scipy.sparse")
    e, n = graphgen.rmat(14, 16, seed=13), 1 << 14
    pairs = stages.simple_graph(e, n)
    A = sp.coo_matrix((np.ones(pairs.shape[0]), (pairs[:, 0], pairs[:, 1])), shape=(n, n)).tocsr()
    A = (A + A.T).tocsr()
    L, U = sp.tril(A, -1).tocsr(), sp.triu(A, 1).tocsr()
    C = (L @ U).multiply(A)
    assert int(round(C.sum())) % 2 == 0
    assert _count(e, n) == int(round(C.sum())) // 2


# ---------------------------------------------------------------- stage definitions
def test_stage_definitions_on_small_graph():
    e, n = _rmat_small(10, 21)
    rank, off, col, src = stages.oriented_csr(e, n)
    assert np.all(src < col)
    assert np.all(np.diff(off) >= 0) and off[-1] == col.shape[0]
    for u in range(n):
        row = col[off[u]:off[u + 1]]
        assert np.all(np.diff(row) > 0)
    assert sorted(rank.tolist()) == list(range(n))
    din, dout, b = stages.middle_buckets(off, col)
    assert b.max() <= stages.NO_BUCKET
    assert np.all((b == stages.NO_BUCKET) == ((din == 0) | (dout == 0)))
    np.testing.assert_array_equal(dout, np.diff(off))


def test_middle_buckets_k4_by_hand():
    # K4: all degrees 3, so rank = id; rows 0 -> {1,2,3}, 1 -> {2,3}, 2 -> {3}.
    # Tails: (0->1): {2,3}; (0->2): {3}; (1->2): {3}; (0->3), (1->3), (2->3): empty.
    rank, off, col, src = stages.oriented_csr(graphgen.complete(4), 4)
    din, dout, b = stages.middle_buckets(off, col)
    assert din.tolist() == [0, 1, 2, 0]
    assert dout.tolist() == [3, 2, 1, 0]
    # vertex 1: 16*log2(1) + log2(2) = 1; vertex 2: 16*log2(2) + log2(1) = 16
    assert b.tolist() == [255, 1, 16, 255]


def test_middle_buckets_complete_graph_closed_form():
    # K_n, rank = id: row v = {v+1 .. n-1}; an in-edge (u -> v) has the tail
    # {v+1 .. n-1}, non-empty iff v < n - 1; so d_in(v) = v, d_out(v) = n - 1 - v.
    n = 40
    rank, off, col, src = stages.oriented_csr(graphgen.complete(n), n)
    din, dout, b = stages.middle_buckets(off, col)
    for v in range(n):
        assert dout[v] == n - 1 - v
        assert din[v] == (v if v < n - 1 else 0)
        if 1 <= v <= n - 2:
            assert b[v] == 16 * int(np.log2(v)) + int(np.log2(n - 1 - v)), v
        else:
            assert b[v] == 255
    tot = stages.bucket_totals(off, col)
    busy = range(1, n - 1)
    assert tot["vertices"].sum() == n - 2
    assert tot["in_edges"].sum() == sum(busy)
    assert tot["out_edges"].sum() == sum(n - 1 - v for v in busy)
    assert tot["work"].sum() == sum(v * (n - 1 - v) for v in busy)
    assert tot["windows"].sum() == n - 2   # every middle list lies inside one 2^17-id window
    # 8-id windows: N+(v) = {v+1 .. 39} spans ((39 - ((v+1) rounded down to 32)) >> 3) + 1
    # windows: 5 for v + 1 < 32 (vertices 1..30), 1 for v + 1 >= 32 (vertices 31..38)
    assert stages.bucket_totals(off, col, window_log2=3)["windows"].sum() == 30 * 5 + 8 * 1


def test_middle_buckets_in_degree_cap():
    # 2^15 vertices u_i joined to both v and w (ids 0 and 1), and v joined to w:
    # deg(u_i) = 2, deg(v) = deg(w) = 2^15 + 1, v before w by id. Each u_i -> v has the
    # tail {w}, so d_in(v) = 2^15 and d_out(v) = 1: bucket 16 * min(14, 15) + 0 = 224.
    k = 1 << 15
    u = np.arange(2, 2 + k, dtype=np.int32)
    e = np.concatenate([np.stack([u, np.zeros(k, np.int32)], 1), np.stack([u, np.ones(k, np.int32)], 1),
                        np.array([[0, 1]], np.int32)])
    rank, off, col, src = stages.oriented_csr(e, k + 2)
    din, dout, b = stages.middle_buckets(off, col)
    rv = rank[0]
    assert (din[rv], dout[rv], b[rv]) == (k, 1, 224)
    assert np.count_nonzero(b != 255) == 1


def test_forward_edge_counts_match_definition():
    """The forward algorithm's per-edge intersection sizes equal the definition-level per-edge
    counts (common neighbours after both endpoints), for both degree readings."""
    e, n = _rmat_small(12, 31)
    dirty = np.concatenate([e, e[::3, ::-1], np.array([[5, 5], [7, 7]], np.int32)]).astype(np.int32)
    for edges, modes in ((e, ("simple", "input")), (dirty, ("simple", "input"))):
        g = oracle.Graph(edges, n)
        for mode in modes:
            f = g.forward_edge_counts(mode)
            np.testing.assert_array_equal(f, g.oriented_edge_counts(mode))
            assert int(f.astype(np.int64).sum()) == g.count()


def test_forward_per_vertex_thread_private_sums():
    """t[v] from the forward algorithm (per-thread sums) equals t[v] by definition
    at 1 and at 8 threads."""
    e, n = _rmat_small(13, 41)
    ref = oracle.Graph(e, n, threads=1).vertex_triangles(np.arange(n))
    for th in (1, 8):
        T, t = oracle.Graph(e, n, threads=th).count(per_vertex=True)
        np.testing.assert_array_equal(t, ref)
        assert int(t.sum()) == 3 * T


@pytest.mark.parametrize("stride", [1, 2, 3, 7])
def test_forward_row_sample_counts_triangles_of_sampled_earliest_vertices(stride):
    """The row-sampled forward count (the CPU baseline's bounded sample) finds exactly the
    triangles whose earliest vertex in the (degree, id) order is a sampled row, by brute
    force over triples; its edge total is the out-degrees of the sampled rows."""
    import itertools
    e = graphgen.erdos_renyi(36, 220, seed=40 + stride)
    n = 36
    g = oracle.Graph(e, n, threads=2)
    deg = g.degrees()
    adj = [set() for _ in range(n)]
    for a, b in g.edges():
        adj[a].add(b)
        adj[b].add(a)
    want = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if b in adj[a] and c in adj[a] and c in adj[b]:
            first = min((a, b, c), key=lambda x: (deg[x], x))
            want += first % stride == 0
    out_deg = np.zeros(n, dtype=np.int64)
    for a, b in g.edges():
        out_deg[a if (deg[a], a) < (deg[b], b) else b] += 1
    T, edges = g.count_rows(stride)
    assert T == want
    assert edges == int(out_deg[::stride].sum())
    if stride == 1:
        assert T == g.count()
    with pytest.raises(ValueError):
        g.count_rows(0)


def test_one_call_entry_matches_the_graph_path():
    """tc_oracle_count (edge list to T in one C call) gives the closed form on K_n and the same T
    and t[v] as the graph path on dirty R-MAT input; an id out of range is refused."""
    assert oracle.tc_oracle_count(graphgen.complete(12), 12) == 220   # C(12, 3)
    e = graphgen.rmat(11, 8, seed=9)
    e = np.concatenate([e, e[:100, ::-1], np.array([[3, 3], [5, 5]], np.int32)])
    T, t = oracle.tc_oracle_count(e, 2048, per_vertex=True)
    T2, t2 = oracle.count_triangles(e, 2048, per_vertex=True)
    assert T == T2 and np.array_equal(t, t2)
    assert oracle.tc_oracle_count(np.array([[0, 5]], np.int32), 5) is None
    assert oracle.tc_oracle_count(np.zeros((0, 2), np.int32), 0) == 0
