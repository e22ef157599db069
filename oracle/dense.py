"""Dense and brute-force triangle counts for small graphs. TEST INFRASTRUCTURE ONLY.

Three formulations that share nothing with the forward algorithm in
``tc_oracle.cpp``, so each can pin it:

* ``brute_force``: every vertex triple is tested (pure Python, n <= ~64).
* ``trace_count``: T = trace(A^3) / 6 and t = diag(A^3) / 2 with int64 matrix
  products (A^3)_vv counts closed walks of length 3 through v, i.e. twice the
  triangles at v.
* ``masked_product``: the matrix formulation of Section 3.3 written as its
  definition, C = A o (L U) for a vertex order: L keeps the entries A[i, k]
  with k before i, U the entries A[k, j] with k before j, so (L U)[i, j]
  counts the common neighbours k of i and j that come before both, and
  C[i, j] counts them for the edges ij alone; every triangle is seen at its
  two later edges, once from each end, so T = (1/2) sum C. (The printed last
  line of Algorithm 3 sums A rather than C; the caption of the worked example,
  Figure 4, sums C, which is the reading taken here.)
"""
from __future__ import annotations

import itertools

import numpy as np


def adjacency(edges: np.ndarray, n: int) -> np.ndarray:
    """Dense symmetric 0/1 int64 adjacency of the simple graph (loops dropped, repeats merged)."""
    A = np.zeros((n, n), dtype=np.int64)
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    for a, b in e:
        if a != b:
            A[a, b] = 1
            A[b, a] = 1
    return A


def brute_force(edges: np.ndarray, n: int):
    """(T, t) by testing all C(n,3) vertex triples."""
    A = adjacency(edges, n)
    t = np.zeros(n, dtype=np.uint64)
    T = 0
    for a, b, c in itertools.combinations(range(n), 3):
        if A[a, b] and A[b, c] and A[a, c]:
            T += 1
            t[a] += 1
            t[b] += 1
            t[c] += 1
    return T, t


def trace_count(edges: np.ndarray, n: int):
    """(T, t) from the cube of the dense adjacency matrix."""
    A = adjacency(edges, n)
    A3 = A @ A @ A
    d = np.diag(A3)
    assert np.all(d % 2 == 0)
    T2 = int(d.sum())
    assert T2 % 6 == 0
    return T2 // 6, (d // 2).astype(np.uint64)


def masked_product(A: np.ndarray, rank=None):
    """C = A o (L U) on a dense adjacency matrix, for the vertex order `rank`
    (rank[v] = position of v; default: id order, where L and U are the strict
    lower and upper triangles of A). Returns (T, L, U, B, C) with B = L U,
    all in the original vertex labels, and T = (1/2) sum C.
    """
    A = np.asarray(A, dtype=np.int64)
    n = A.shape[0]
    r = np.arange(n) if rank is None else np.asarray(rank)
    before = (r[None, :] < r[:, None]).astype(np.int64)   # before[i, k]: k comes before i
    L = A * before                # L[i, k] = A[i, k] when k is before i
    U = A * before.T              # U[k, j] = A[k, j] when k is before j
    B = L @ U
    C = A * B
    s = int(C.sum())
    assert s % 2 == 0
    return s // 2, L, U, B, C


def nnz_rank(A: np.ndarray) -> np.ndarray:
    """Position of each vertex when rows are ordered by increasing number of
    nonzeros, ties by id (the row order Algorithm 3 asks for)."""
    p = np.argsort(np.asarray(A).sum(axis=1), kind="stable")
    r = np.empty_like(p)
    r[p] = np.arange(p.size)
    return r
