"""Dense and brute-force triangle counts for small graphs. TEST INFRASTRUCTURE ONLY.

Three formulations that share nothing with the forward algorithm in
``tc_oracle.cpp``, so each can pin it:

* ``brute_force``: every vertex triple is tested (pure Python, n <= ~64).
* ``trace_count``: T = trace(A^3) / 6 and t = diag(A^3) / 2 with int64 matrix
  products (A^3)_vv counts closed walks of length 3 through v, i.e. twice the
  triangles at v.
* ``matrix_formulation``: the paper's Algorithm 3 (Section 3.3): split A into
  its strictly lower and strictly upper triangles L and U, B = L U,
  C = A o B (Hadamard product), T = (1/2) sum C. The printed last line of the
  algorithm sums A rather than C; the figure caption of the worked example
  (Figure 4) sums C, which is the reading taken here.
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


def matrix_formulation(A: np.ndarray, permute_by_nnz: bool = False):
    """Algorithm 3 on a dense adjacency matrix. Returns (T, L, U, B, C).

    With permute_by_nnz, rows and columns are first reordered by increasing
    number of nonzeros (stable), as the algorithm's first step says; the
    worked example of Figure 4 is shown without that permutation.
    """
    A = np.asarray(A, dtype=np.int64)
    if permute_by_nnz:
        p = np.argsort(A.sum(axis=1), kind="stable")
        A = A[np.ix_(p, p)]
    L = np.tril(A, -1)
    U = np.triu(A, 1)
    B = L @ U
    C = A * B
    s = int(C.sum())
    assert s % 2 == 0
    return s // 2, L, U, B, C
