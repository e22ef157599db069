"""CPU oracle for exact triangle counting. TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The GPU library never imports, links or
calls it, and it imports nothing from the GPU package: the two share no code.

Contents
  * ``tc_oracle.cpp`` (built into ``liboracle.so``): the forward algorithm,
    definition-level per-vertex / per-edge counts, the matrix formulation
    (Algorithm 3, row by row) and the full-list variant; see that file's
    header.
  * ``dense``: brute force over vertex triples, trace(A^3)/6 and the matrix
    formulation (Algorithm 3) on dense matrices, for small graphs.
  * ``stages``: plain numpy definitions of the intermediate products of the
    GPU pipeline (canonical simple graph, degree-rank order, oriented CSR,
    per-edge buckets), for stage-level parity.
  * ``mlp``: float64 numpy forward/backward of the kernel-selector MLP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None

ORDER_DEG_ID = 0     # (degree, id) ascending
ORDER_PAPER = 1      # degree descending, id ascending (the paper's literal filter)
ORDER_ID = 2         # plain id order


def build() -> str:
    """Compile tc_oracle.cpp into liboracle.so (g++ -O3, OpenMP)."""
    src = os.path.join(_HERE, "tc_oracle.cpp")
    tmp = _SO + ".tmp"
    subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    vp = ctypes.c_void_p
    lib.tc_oracle_count.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, vp, ctypes.c_int]
    lib.tc_oracle_count.restype = ctypes.c_uint64
    lib.oracle_graph_build.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(vp)]
    lib.oracle_graph_build.restype = ctypes.c_int
    lib.oracle_graph_build_timed.argtypes = [vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int, ctypes.POINTER(vp), vp]
    lib.oracle_graph_build_timed.restype = ctypes.c_int
    lib.oracle_graph_free.argtypes = [vp]
    lib.oracle_graph_num_edges.argtypes = [vp]
    lib.oracle_graph_num_edges.restype = ctypes.c_int64
    lib.oracle_graph_edges.argtypes = [vp, vp]
    lib.oracle_graph_degrees.argtypes = [vp, vp]
    lib.oracle_count_forward.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    lib.oracle_count_forward.restype = ctypes.c_uint64
    lib.oracle_count_forward_timed.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int, vp]
    lib.oracle_count_forward_timed.restype = ctypes.c_uint64
    lib.oracle_count_forward_rows.argtypes = [vp, ctypes.c_int, ctypes.c_int32, vp, ctypes.c_int, vp, vp]
    lib.oracle_count_forward_rows.restype = ctypes.c_uint64
    lib.oracle_forward_edge_counts.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    lib.oracle_vertex_triangles.argtypes = [vp, vp, ctypes.c_int64, vp, ctypes.c_int]
    lib.oracle_oriented_edge_counts.argtypes = [vp, ctypes.c_int, vp, ctypes.c_int]
    lib.oracle_edge_support.argtypes = [vp, vp, ctypes.c_int]
    lib.oracle_pair_counts.argtypes = [vp, vp, ctypes.c_int64, ctypes.c_int, vp, ctypes.c_int]
    lib.oracle_full_sum.argtypes = [vp, ctypes.c_int]
    lib.oracle_full_sum.restype = ctypes.c_uint64
    lib.oracle_matrix_rows.argtypes = [vp, ctypes.c_int, ctypes.c_int, vp, ctypes.c_int]
    lib.oracle_matrix_rows.restype = ctypes.c_uint64
    _lib = lib
    return lib


class VertexRangeError(ValueError):
    pass


class Graph:
    """The simple undirected graph denoted by an edge list (loops dropped, repeats merged)."""

    def __init__(self, edges: np.ndarray, n: int, threads: int = 0):
        e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
        self.n = int(n)
        self.threads = threads
        lib = _load()
        h = ctypes.c_void_p()
        secs = np.zeros(3, dtype=np.float64)
        st = lib.oracle_graph_build_timed(e.ctypes.data if e.size else None, e.shape[0], self.n, threads,
                                          ctypes.byref(h), secs.ctypes.data)
        if st == 2:
            raise VertexRangeError("vertex id outside [0, n)")
        if st != 0:
            raise ValueError("invalid argument")
        self._h = h
        # wall seconds: canonicalisation (sort + de-duplication), the degrees, and
        # the symmetric adjacency of the definition-level functions
        self.build_seconds = (float(secs[0]), float(secs[1]), float(secs[2]))
        self.count_seconds = None

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            _load().oracle_graph_free(h)
            self._h = None

    @property
    def m(self) -> int:
        return int(_load().oracle_graph_num_edges(self._h))

    def edges(self) -> np.ndarray:
        out = np.empty((self.m, 2), dtype=np.int32)
        if self.m:
            _load().oracle_graph_edges(self._h, out.ctypes.data)
        return out

    def degrees(self) -> np.ndarray:
        out = np.empty(self.n, dtype=np.int32)
        if self.n:
            _load().oracle_graph_degrees(self._h, out.ctypes.data)
        return out

    def count(self, order: int = ORDER_DEG_ID, per_vertex: bool = False):
        """Forward algorithm. Returns T, or (T, t) with per_vertex. Afterwards
        count_seconds = (orientation + out-lists, intersections) wall seconds."""
        t = np.zeros(self.n, dtype=np.uint64) if per_vertex else None
        secs = np.zeros(2, dtype=np.float64)
        T = int(_load().oracle_count_forward_timed(self._h, order, t.ctypes.data if per_vertex and self.n else None,
                                                   self.threads, secs.ctypes.data))
        self.count_seconds = (float(secs[0]), float(secs[1]))
        return (T, t) if per_vertex else T

    def count_rows(self, row_stride: int, order: int = ORDER_DEG_ID):
        """The forward algorithm with the intersections of rows u % row_stride == 0 only
        (a bounded sample for timing). Returns (triangles whose earliest vertex is such a
        row, kept edges of those rows); count_seconds as in count()."""
        if row_stride < 1:
            raise ValueError("row_stride must be >= 1")
        secs = np.zeros(2, dtype=np.float64)
        edges = ctypes.c_int64(0)
        T = int(_load().oracle_count_forward_rows(self._h, order, row_stride, None, self.threads,
                                                  secs.ctypes.data, ctypes.byref(edges)))
        self.count_seconds = (float(secs[0]), float(secs[1]))
        return T, int(edges.value)

    def forward_edge_counts(self, degree: str = "simple") -> np.ndarray:
        """The forward algorithm's per-edge intersection sizes (the list of
        intersection sizes of Algorithm 2) per canonical edge, uint32 [m]: the same values as
        oriented_edge_counts, computed by merging out-lists instead of by definition."""
        out = np.zeros(self.m, dtype=np.uint32)
        if self.m:
            _load().oracle_forward_edge_counts(self._h, {"simple": 0, "input": 1}[degree], out.ctypes.data,
                                               self.threads)
        return out

    def vertex_triangles(self, vs) -> np.ndarray:
        vs = np.ascontiguousarray(vs, dtype=np.int32)
        out = np.zeros(vs.shape[0], dtype=np.uint64)
        if vs.size:
            _load().oracle_vertex_triangles(self._h, vs.ctypes.data, vs.shape[0], out.ctypes.data, self.threads)
        return out

    def oriented_edge_counts(self, degree: str = "simple") -> np.ndarray:
        """Per canonical edge, |N+(x) n N+(y)| for the (degree, id) orientation.

        degree="simple": degree in the simple graph; degree="input": number of
        input pairs at the vertex (self-loops dropped, repeats counted).
        """
        out = np.zeros(self.m, dtype=np.uint32)
        mode = {"simple": 0, "input": 1}[degree]
        if self.m:
            _load().oracle_oriented_edge_counts(self._h, mode, out.ctypes.data, self.threads)
        return out

    def pair_counts(self, pairs, degree: str = "simple") -> np.ndarray:
        """oriented_edge_counts for the given pairs only (0 for a pair that is not an edge)."""
        p = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros(p.shape[0], dtype=np.uint32)
        if p.size:
            _load().oracle_pair_counts(self._h, p.ctypes.data, p.shape[0], {"simple": 0, "input": 1}[degree],
                                       out.ctypes.data, self.threads)
        return out

    def full_sum(self) -> int:
        """Full-list variant: sum over the edges of |N(a) n N(b)| (= 3T)."""
        return int(_load().oracle_full_sum(self._h, self.threads)) if self.m else 0

    def matrix_sum(self, order: int = ORDER_DEG_ID, upper: bool = False, row_sums: bool = False):
        """Algorithm 3 row by row: sum of C = A o (L U) (= 2T; T with upper).

        order: ORDER_DEG_ID (rows by increasing nonzeros, ties by id) or
        ORDER_ID (no permutation). With row_sums, also the per-row sums of C
        (uint64, original ids).
        """
        if order not in (ORDER_DEG_ID, ORDER_ID):
            raise ValueError("order must be ORDER_DEG_ID or ORDER_ID")
        rs = np.zeros(self.n, dtype=np.uint64) if row_sums else None
        s = int(_load().oracle_matrix_rows(self._h, order, 1 if upper else 0,
                                           rs.ctypes.data if row_sums and self.n else None, self.threads))
        return (s, rs) if row_sums else s

    def edge_support(self) -> np.ndarray:
        out = np.zeros(self.m, dtype=np.uint32)
        if self.m:
            _load().oracle_edge_support(self._h, out.ctypes.data, self.threads)
        return out


def tc_oracle_count(edges: np.ndarray, n: int, per_vertex: bool = False, threads: int = 0):
    """The one-call C entry (edge list to T, and t[v] with per_vertex); None for invalid input."""
    e = np.ascontiguousarray(edges, dtype=np.int32).reshape(-1, 2)
    t = np.zeros(max(n, 0), dtype=np.uint64) if per_vertex else None
    T = int(_load().tc_oracle_count(e.ctypes.data if e.size else None, e.shape[0], n,
                                    t.ctypes.data if per_vertex and n > 0 else None, threads))
    if T == (1 << 64) - 1:
        return None
    return (T, t) if per_vertex else T


def count_triangles(edges: np.ndarray, n: int, per_vertex: bool = False, threads: int = 0,
                    order: int = ORDER_DEG_ID):
    """T (and t[v] with per_vertex) of the simple graph denoted by ``edges``."""
    return Graph(edges, n, threads).count(order=order, per_vertex=per_vertex)
