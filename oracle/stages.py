"""Plain numpy definitions of the intermediate products of the counting path.
TEST INFRASTRUCTURE ONLY.

Each function is the definition of one step of the forward algorithm as the
GPU path stages it (Section 3.2 and Section 4.2), written with numpy library
primitives (sort, unique, bincount, lexsort) and no blocking or fusion:

* ``simple_graph``   canonical, loop-free, de-duplicated pairs (a < b).
* ``degree_order``   rank of every vertex in (degree, id) ascending order.
* ``oriented_csr``   each edge kept once, directed from the lower to the higher
                     rank, as a CSR over ranks with ascending rows.
* ``edge_tails``     for kept edge e = (u -> v) at position p of row u, the
                     candidates of the intersection are the entries of row u
                     after p (they alone exceed v); its length and the length
                     of row v define the edge's degree-pair bucket.
* ``oriented_counts`` the per-edge intersection sizes, by sets.
"""
from __future__ import annotations

import numpy as np


def simple_graph(edges: np.ndarray, n: int) -> np.ndarray:
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    if e.size and (e.min() < 0 or e.max() >= n):
        raise ValueError("vertex id outside [0, n)")
    a = np.minimum(e[:, 0], e[:, 1])
    b = np.maximum(e[:, 0], e[:, 1])
    keep = a != b
    k = np.unique((a[keep] << 32) | b[keep])
    return np.stack([k >> 32, k & 0xFFFFFFFF], 1).astype(np.int64)


def degrees(pairs: np.ndarray, n: int) -> np.ndarray:
    return (np.bincount(pairs[:, 0], minlength=n) + np.bincount(pairs[:, 1], minlength=n)).astype(np.int64)


def degree_order(deg: np.ndarray) -> np.ndarray:
    """rank[v] = position of v when vertices are sorted by (degree, id)."""
    n = deg.shape[0]
    order = np.lexsort((np.arange(n), deg))
    rank = np.empty(n, dtype=np.int64)
    rank[order] = np.arange(n)
    return rank


def input_degrees(edges: np.ndarray, n: int) -> np.ndarray:
    """Number of input pairs at each vertex, self-loops dropped, repeated pairs counted."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    e = e[e[:, 0] != e[:, 1]]
    return (np.bincount(e[:, 0], minlength=n) + np.bincount(e[:, 1], minlength=n)).astype(np.int64)


def oriented_csr(edges: np.ndarray, n: int, degree: str = "simple"):
    """(rank, offsets int64[n+1], col int64[m], src int64[m]) of the degree-ordered graph.

    degree="simple" orders by the simple graph's degrees, degree="input" by the
    number of input pairs at each vertex (identical when the input has no repeats).
    """
    pairs = simple_graph(edges, n)
    deg = degrees(pairs, n) if degree == "simple" else input_degrees(edges, n)
    rank = degree_order(deg)
    ra, rb = rank[pairs[:, 0]], rank[pairs[:, 1]]
    src, dst = np.minimum(ra, rb), np.maximum(ra, rb)
    o = np.lexsort((dst, src))
    src, dst = src[o], dst[o]
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(np.bincount(src, minlength=n), out=off[1:])
    return rank, off, dst, src


def edge_tails(off: np.ndarray, col: np.ndarray, src: np.ndarray):
    """(tail_len, dplus_v) per kept edge in CSR order."""
    m = col.shape[0]
    e = np.arange(m, dtype=np.int64)
    tail = off[src + 1] - e - 1
    dplus = np.diff(off)
    return tail, dplus[col]


def bucket_of(tail: np.ndarray, dv: np.ndarray) -> np.ndarray:
    """Degree-pair bucket 16 * l(tail) + l(d+ v), l(x) = min(15, floor(log2 x)); -1 when either is 0."""
    def lg(x):
        x = np.asarray(x, dtype=np.int64)
        out = np.full(x.shape, -1, dtype=np.int64)
        pos = x > 0
        out[pos] = np.minimum(15, np.floor(np.log2(x[pos])).astype(np.int64))
        return out
    lt, lv = lg(tail), lg(dv)
    b = 16 * lt + lv
    b[(lt < 0) | (lv < 0)] = -1
    return b


def oriented_counts(off: np.ndarray, col: np.ndarray, src: np.ndarray) -> np.ndarray:
    """|N+(u) intersected with N+(v)| for each kept edge u -> v, by Python sets (small graphs)."""
    n = off.shape[0] - 1
    rows = [set(col[off[v]:off[v + 1]].tolist()) for v in range(n)]
    return np.array([len(rows[u] & rows[v]) for u, v in zip(src.tolist(), col.tolist())], dtype=np.int64)
