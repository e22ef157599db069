"""Plain numpy definitions of the intermediate products of the counting path.
TEST INFRASTRUCTURE ONLY.

Each function is the definition of one step of the forward algorithm as the
GPU path stages it (Section 3.2 and Section 4.2), written with numpy library
primitives (sort, unique, bincount, lexsort) and no blocking or fusion:

* ``simple_graph``   canonical, loop-free, de-duplicated pairs (a < b).
* ``degree_order``   rank of every vertex in (degree, id) ascending order.
* ``oriented_csr``   each edge kept once, directed from the lower to the higher
                     rank, as a CSR over ranks with ascending rows.
* ``middle_buckets`` the dynamic grouping (Section 4.2) by middle vertex: for
                     kept edge e = (u -> v) at position p of row u, only the
                     entries of row u after p (its tail) can be common
                     out-neighbours of u and v; v's in-edges with a non-empty
                     tail and its out-degree give v's degree-pair bucket.
* ``bucket_totals``  per-bucket sums of those quantities.
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


NO_BUCKET = 255


def _floor_log2(x: np.ndarray) -> np.ndarray:
    """floor(log2 x) of positive integers, exactly (bit length - 1)."""
    x = np.asarray(x, dtype=np.int64)
    out = np.zeros(x.shape, dtype=np.int64)
    y = x.copy()
    while np.any(y > 1):
        big = y > 1
        out[big] += 1
        y[big] >>= 1
    return out


def middle_buckets(off: np.ndarray, col: np.ndarray):
    """(d_in, d_out, bucket) per vertex of the oriented CSR (over ranks).

    d_in(v): kept edges (u -> v) whose tail in row u (the entries after v) is
    non-empty; d_out(v) = |N+(v)|. A vertex with both positive falls in bucket
    16 * min(14, floor(log2 d_in)) + min(15, floor(log2 d_out)); every other
    vertex in NO_BUCKET (255): it has no intersection work as a middle vertex.
    """
    off = np.asarray(off, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    n = off.shape[0] - 1
    m = col.shape[0]
    dout = np.diff(off)
    src = np.repeat(np.arange(n, dtype=np.int64), dout)
    tail = off[src + 1] - np.arange(m, dtype=np.int64) - 1   # entries of row u after the edge
    din = np.bincount(col[tail > 0], minlength=n).astype(np.int64)
    bucket = np.full(n, NO_BUCKET, dtype=np.int64)
    busy = (din > 0) & (dout > 0)
    bucket[busy] = 16 * np.minimum(14, _floor_log2(din[busy])) + np.minimum(15, _floor_log2(dout[busy]))
    return din, dout, bucket


def bucket_totals(off: np.ndarray, col: np.ndarray, window_log2: int = 17):
    """Per bucket (256 entries, NO_BUCKET excluded from every sum): vertices,
    sum of d_in, sum of d_out, sum of d_in * d_out, and the bitmap windows of
    2^window_log2 ids that each middle list N+(v) spans, counted from its first
    element rounded down to a multiple of 32 to its last."""
    off = np.asarray(off, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    din, dout, bucket = middle_buckets(off, col)
    busy = np.nonzero(bucket != NO_BUCKET)[0]
    b = bucket[busy]
    lo, hi = col[off[busy]], col[off[busy + 1] - 1]
    win = ((hi - (lo & ~31)) >> window_log2) + 1
    out = {}
    for name, w in (("vertices", np.ones_like(b)), ("in_edges", din[busy]), ("out_edges", dout[busy]),
                    ("work", din[busy] * dout[busy]), ("windows", win)):
        acc = np.zeros(256, dtype=np.int64)
        np.add.at(acc, b, w.astype(np.int64))   # integer sums, no rounding
        out[name] = acc
    return out


def oriented_counts(off: np.ndarray, col: np.ndarray, src: np.ndarray) -> np.ndarray:
    """|N+(u) intersected with N+(v)| for each kept edge u -> v, by Python sets (small graphs)."""
    n = off.shape[0] - 1
    rows = [set(col[off[v]:off[v + 1]].tolist()) for v in range(n)]
    return np.array([len(rows[u] & rows[v]) for u, v in zip(src.tolist(), col.tolist())], dtype=np.int64)
