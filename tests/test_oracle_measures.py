"""Pins of the oracle's clustering coefficient and transitivity (no GPU):
closed forms on structured graphs, brute force on small random graphs, and
networkx as an independent library."""
import math

import numpy as np
import pytest

import graphgen
from oracle.measures import clustering


@pytest.mark.parametrize("n", [3, 4, 9])
def test_complete_graph_is_fully_clustered(n):
    coeff, T, W, tr, _ = clustering(graphgen.complete(n), n)
    assert np.all(coeff == 1.0) and tr == 1.0
    assert T == math.comb(n, 3) and W == n * math.comb(n - 1, 2)


def test_star_and_bipartite_have_no_clustering():
    for e, n in ((graphgen.star(50), 51), (graphgen.complete_bipartite(6, 9), 15)):
        coeff, T, W, tr, _ = clustering(e, n)
        assert T == 0 and tr == 0.0 and np.all(coeff == 0.0) and W > 0


@pytest.mark.parametrize("k", [4, 5, 12])
def test_wheel_closed_form(k):
    # vertex 0 is the hub (degree k, k triangles); each rim vertex has degree 3 and 2 triangles
    coeff, T, W, tr, _ = clustering(graphgen.wheel(k), k + 1)
    assert coeff[0] == k / math.comb(k, 2)
    assert np.all(coeff[1:] == 2 / 3)
    assert W == math.comb(k, 2) + 3 * k and tr == 3.0 * k / W


@pytest.mark.parametrize("k", [1, 3, 10])
def test_friendship_closed_form(k):
    # F_k: hub of degree 2k in k triangles; blades of degree 2 in one triangle each
    coeff, T, W, tr, _ = clustering(graphgen.friendship(k), 2 * k + 1)
    assert coeff[0] == 1.0 / (2 * k - 1)
    assert np.all(coeff[1:] == 1.0)
    assert W == k * (2 * k + 1) and tr == 3.0 / (2 * k + 1)


def test_isolated_and_pendant_vertices_are_zero():
    e = np.array([[0, 1], [1, 2], [2, 0], [2, 3]], dtype=np.int32)
    coeff, T, W, tr, _ = clustering(e, 6)
    assert coeff.tolist() == [1.0, 1.0, 1.0 / 3.0, 0.0, 0.0, 0.0]
    assert W == 1 + 1 + 3 and T == 1 and tr == 3.0 / 5.0


@pytest.mark.parametrize("seed", range(4))
def test_brute_force_on_small_random_graphs(seed):
    rng = np.random.default_rng(seed)
    n = 24
    A = np.triu(rng.random((n, n)) < 0.3, 1)
    A = (A | A.T).astype(np.int64)
    i, j = np.nonzero(np.triu(A, 1))
    e = np.stack([i, j], 1).astype(np.int32)
    coeff, T, W, tr, t = clustering(e, n)
    tri = np.zeros(n, dtype=np.int64)
    for a in range(n):
        for b in range(a + 1, n):
            for c in range(b + 1, n):
                if A[a, b] and A[b, c] and A[a, c]:
                    tri[[a, b, c]] += 1
    d = A.sum(1)
    for v in range(n):
        want = tri[v] / (d[v] * (d[v] - 1) // 2) if d[v] >= 2 else 0.0
        assert coeff[v] == want, v
    assert T == int(tri.sum()) // 3 and W == int(sum(x * (x - 1) // 2 for x in d))
    np.testing.assert_array_equal(t, tri.astype(np.uint64))


def test_loops_and_repeats_do_not_change_degrees():
    e = graphgen.erdos_renyi(300, 2000, seed=9)
    dirty = np.concatenate([e, e[:500, ::-1], np.array([[5, 5], [7, 7]], dtype=np.int32)])
    a, b = clustering(e, 300), clustering(graphgen.shuffle_edges(dirty.astype(np.int32), 1), 300)
    np.testing.assert_array_equal(a[0], b[0])
    assert a[1:4] == b[1:4]


def test_networkx_clustering_and_transitivity():
    nx = pytest.importorskip("networkx")
    for e, n in ((graphgen.rmat(11, 16, seed=8), 1 << 11), (graphgen.rgg(3000, avg_degree=16, seed=2), 3000)):
        G = nx.Graph()
        G.add_nodes_from(range(n))
        G.add_edges_from((int(a), int(b)) for a, b in e if a != b)
        coeff, T, W, tr, _ = clustering(e, n)
        ref = nx.clustering(G)
        # both are one correctly rounded division of the same exact ratio
        np.testing.assert_array_equal(coeff, np.array([ref[v] for v in range(n)], dtype=np.float64))
        assert tr == nx.transitivity(G)
