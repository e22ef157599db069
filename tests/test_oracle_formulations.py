"""Pins for the oracle's matrix formulation (Algorithm 3, row by row) and its
full-list variant of the intersection method.

Each is tied to facts other than itself: the printed matrices of the worked
example (Figure 4), the dense Algorithm 3 with numpy matrix products, brute
force over vertex triples, closed forms of structured graphs, and the
invariance of the sums under the row order.
"""
import math

import numpy as np
import pytest

import graphgen
import oracle
from oracle import dense
from tests.conftest import load_golden_matrices


def _edges_of(A):
    i, j = np.nonzero(np.triu(A, 1))
    return np.stack([i, j], 1).astype(np.int32)


def _random_graph(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(4, 36))
    p = [0.1, 0.25, 0.5, 0.85][seed % 4]
    A = np.triu(rng.random((n, n)) < p, 1).astype(np.int64)
    return A + A.T, n


# ---------------------------------------------------------------- Figure 4
def test_fig4_row_sums_match_the_printed_C():
    g = load_golden_matrices("fig4_matrix_example.txt")
    e = _edges_of(g["A"])
    s, rs = oracle.Graph(e, 7).matrix_sum(order=oracle.ORDER_ID, row_sums=True)
    np.testing.assert_array_equal(rs, g["C"].sum(axis=1))
    assert s == int(g["C"].sum()) == 6
    assert s // 2 == int(g["T"][0, 0]) == 3


def test_fig4_upper_mask_and_full_sum():
    g = load_golden_matrices("fig4_matrix_example.txt")
    G = oracle.Graph(_edges_of(g["A"]), 7)
    assert G.matrix_sum(order=oracle.ORDER_ID, upper=True) == int(np.triu(g["C"], 1).sum()) == 3
    assert G.full_sum() == 9   # three triangles, each seen at three edges


# ---------------------------------------------------------------- dense Algorithm 3
@pytest.mark.parametrize("seed", range(8))
def test_rows_match_dense_algorithm_3_in_id_order(seed):
    A, n = _random_graph(seed)
    _, _, _, _, C = dense.masked_product(A)
    s, rs = oracle.Graph(_edges_of(A), n).matrix_sum(order=oracle.ORDER_ID, row_sums=True)
    np.testing.assert_array_equal(rs, C.sum(axis=1))
    assert s == int(C.sum())
    assert oracle.Graph(_edges_of(A), n).matrix_sum(order=oracle.ORDER_ID, upper=True) == int(np.triu(C, 1).sum())


@pytest.mark.parametrize("seed", range(8))
def test_rows_match_dense_algorithm_3_with_nnz_permutation(seed):
    A, n = _random_graph(seed)
    _, _, _, _, C = dense.masked_product(A, dense.nnz_rank(A))
    s, rs = oracle.Graph(_edges_of(A), n).matrix_sum(order=oracle.ORDER_DEG_ID, row_sums=True)
    np.testing.assert_array_equal(rs, C.sum(axis=1))
    assert s == int(C.sum())
    # the order changes C, never the count: T = trace(A^3) / 6 in both orders
    Tt, _ = dense.trace_count(_edges_of(A), n)
    assert dense.masked_product(A)[0] == dense.masked_product(A, dense.nnz_rank(A))[0] == Tt


# ---------------------------------------------------------------- brute force and invariants
@pytest.mark.parametrize("seed", range(8))
def test_sums_are_multiples_of_the_brute_force_count(seed):
    A, n = _random_graph(seed)
    e = _edges_of(A)
    Tb, _ = dense.brute_force(e, n)
    G = oracle.Graph(e, n)
    for order in (oracle.ORDER_DEG_ID, oracle.ORDER_ID):
        assert G.matrix_sum(order=order) == 2 * Tb
        assert G.matrix_sum(order=order, upper=True) == Tb
    assert G.full_sum() == 3 * Tb


def test_full_sum_is_the_sum_of_brute_force_edge_triangles():
    A, n = _random_graph(3)
    e = _edges_of(A)
    per_edge = [sum(1 for w in range(n) if A[a, w] and A[b, w]) for a, b in e]
    assert oracle.Graph(e, n).full_sum() == sum(per_edge)


@pytest.mark.parametrize("n", [3, 4, 7, 12])
def test_complete_graph_closed_forms(n):
    e = np.array([(a, b) for a in range(n) for b in range(a + 1, n)], dtype=np.int32)
    G = oracle.Graph(e, n)
    T = math.comb(n, 3)
    assert G.full_sum() == math.comb(n, 2) * (n - 2) == 3 * T
    assert G.matrix_sum() == 2 * T
    assert G.matrix_sum(upper=True) == T


def test_star_and_bipartite_are_zero():
    star = np.array([(0, i) for i in range(1, 30)], dtype=np.int32)
    kab = np.array([(a, 10 + b) for a in range(10) for b in range(12)], dtype=np.int32)
    for e, n in ((star, 30), (kab, 22)):
        G = oracle.Graph(e, n)
        assert G.full_sum() == 0 and G.matrix_sum() == 0 and G.matrix_sum(upper=True) == 0


@pytest.mark.parametrize("k", [4, 9, 33])
def test_wheel_closed_form(k):
    # hub 0 and a k-cycle 1..k: k triangles
    e = [(0, i) for i in range(1, k + 1)] + [(i, i % k + 1) for i in range(1, k + 1)]
    G = oracle.Graph(np.array(e, dtype=np.int32), k + 1)
    assert G.full_sum() == 3 * k
    assert G.matrix_sum() == 2 * k
    assert G.matrix_sum(upper=True) == k


def test_loops_and_repeats_are_ignored():
    rng = np.random.default_rng(5)
    e = graphgen.erdos_renyi(300, 2500, seed=5)
    dirty = np.concatenate([e, e[::-1, ::-1], np.stack([np.arange(40), np.arange(40)], 1).astype(np.int32)])
    dirty = dirty[rng.permutation(dirty.shape[0])]
    a, b = oracle.Graph(e, 300), oracle.Graph(dirty, 300)
    assert a.full_sum() == b.full_sum()
    assert a.matrix_sum() == b.matrix_sum()


def test_rmat_sums_agree_with_the_forward_oracle():
    e = graphgen.rmat(12, 16, seed=3)
    n = 1 << 12
    T = oracle.count_triangles(e, n)
    G = oracle.Graph(e, n)
    assert G.full_sum() == 3 * T
    assert G.matrix_sum() == 2 * T
    assert G.matrix_sum(upper=True) == T
