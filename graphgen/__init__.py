"""Seeded synthetic graph inputs shared by the oracle tests, the GPU tests and bench.py.

Nothing here counts triangles or orders vertices: it only draws vertex pairs. The
C part (``graphgen.c``) uses a counter-based generator, so every array is a pure
function of its seed, whatever the thread count.

Workload shapes follow the paper's dataset classes (scale-free and mesh-like,
Table "Dataset Description", Section 5); the graphs themselves are synthetic.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "libgraphgen.so")
_lib = None

RMAT_ABC = (0.57, 0.19, 0.19)   # d = 0.05


def build() -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, OpenMP)."""
    src = os.path.join(_HERE, "graphgen.c")
    tmp = _SO + ".tmp"
    subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gg_permutation.argtypes = [ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int32, i32p]
    lib.gg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_uint64,
                                ctypes.c_void_p, ctypes.c_int32, i32p]
    lib.gg_rgg.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_uint64, i32p, ctypes.c_int64]
    lib.gg_rgg.restype = ctypes.c_int64
    lib.gg_shuffle_edges.argtypes = [i32p, ctypes.c_int64, ctypes.c_uint64]
    lib.gg_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                             ctypes.POINTER(ctypes.c_uint64)]
    _lib = lib
    return lib


def _i32p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _sub_seed(seed: int, k: int) -> int:
    """A distinct 64-bit seed for item k of a family (SplitMix64 of seed + k)."""
    z = (seed * 0x9E3779B97F4A7C15 + (k + 1) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & 0xFFFFFFFFFFFFFFFF
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & 0xFFFFFFFFFFFFFFFF
    return z ^ (z >> 31)


def draws(seed: int, stream: int, count: int) -> np.ndarray:
    """Raw uint64 draws of the counter-based generator (for generator tests)."""
    out = np.empty(count, dtype=np.uint64)
    _load().gg_draws(seed, stream, count, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    return out


def permutation(n: int, seed: int) -> np.ndarray:
    p = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed, _i32p(p))
    return p


def erdos_renyi(n: int, m: int, seed: int = 1804) -> np.ndarray:
    """G(n, m): m distinct unordered pairs, no self-loops, drawn with numpy PCG64(seed).

    Pairs are drawn in rounds and rejected if they are loops or repeats until m
    distinct pairs exist; the result is returned in draw order, random direction.
    """
    if m > n * (n - 1) // 2:
        raise ValueError("m exceeds n choose 2")
    rng = np.random.Generator(np.random.PCG64(seed))
    seen: set = set()
    out = np.empty((m, 2), dtype=np.int32)
    k = 0
    while k < m:
        need = m - k
        cand = rng.integers(0, n, size=(need + need // 4 + 16, 2), dtype=np.int64)
        for a, b in cand:
            if a == b:
                continue
            key = (min(a, b), max(a, b))
            if key in seen:
                continue
            seen.add(key)
            out[k, 0], out[k, 1] = a, b
            k += 1
            if k == m:
                break
    return out


def rmat(scale: int, edge_factor: int = 16, seed: int = 1, abc=RMAT_ABC,
         permute: bool = True, flip: bool = True) -> np.ndarray:
    """R-MAT draws: edge_factor * 2**scale pairs over 2**scale vertices.

    The array is the raw draw list (self-loops and repeats included); the graph it
    denotes is its symmetrised, loop-free, deduplicated version, which is what the
    counter computes on. With permute, vertex ids go through a seeded random
    permutation (so vertex 0 is not the hub).
    """
    n = 1 << scale
    E = edge_factor * n
    out = np.empty((E, 2), dtype=np.int32)
    perm = permutation(n, _sub_seed(seed, 7)) if permute else None
    a, b, c = abc
    _load().gg_rmat(scale, E, a, b, c, seed,
                    perm.ctypes.data if perm is not None else None, int(flip), _i32p(out))
    return out


def chung_lu(n: int, E: int, gamma: float = 2.1, seed: int = 1, permute: bool = True,
             base: int = 0) -> np.ndarray:
    """Chung-Lu draws: E pairs with endpoints drawn proportionally to (i+1)^(-1/(gamma-1))."""
    out = np.empty((E, 2), dtype=np.int32)
    chung_lu_into(out, n, gamma, seed, permute, base)
    return out


def chung_lu_into(out: np.ndarray, n: int, gamma: float, seed: int, permute: bool = True,
                  base: int = 0) -> None:
    assert out.dtype == np.int32 and out.flags.c_contiguous and out.ndim == 2
    perm = permutation(n, _sub_seed(seed, 11)) if permute else None
    _load().gg_chung_lu(n, out.shape[0], gamma, seed,
                        perm.ctypes.data if perm is not None else None, base, _i32p(out))


def chung_lu_batch_sizes(num_graphs: int = 4096, lo: float = 1e3, hi: float = 1e6,
                         seed: int = 2101, avg_degree: float = 16.0):
    """Per-graph (n_g, E_g): E_g log-uniform in [lo, hi] draws, n_g = round(E_g * 2 / avg_degree)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    E = np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=num_graphs))).astype(np.int64)
    n = np.maximum(np.rint(E * 2.0 / avg_degree), 2).astype(np.int32)
    return n, E


def chung_lu_batch(num_graphs: int = 4096, lo: float = 1e3, hi: float = 1e6, gamma: float = 2.1,
                   seed: int = 2101, avg_degree: float = 16.0):
    """A batch of Chung-Lu graphs with graph-local ids.

    Returns (edges int32[sum E_g][2], edge_offsets int64[G+1], num_vertices int32[G]).
    Graph g's pairs are edges[edge_offsets[g]:edge_offsets[g+1]], ids in [0, n_g).
    """
    n, E = chung_lu_batch_sizes(num_graphs, lo, hi, seed, avg_degree)
    off = np.zeros(num_graphs + 1, dtype=np.int64)
    np.cumsum(E, out=off[1:])
    edges = np.empty((int(off[-1]), 2), dtype=np.int32)
    for g in range(num_graphs):
        chung_lu_into(edges[off[g]:off[g + 1]], int(n[g]), gamma, _sub_seed(seed, 1000 + g))
    return edges, off, n


def rgg(n: int, avg_degree: float = 32.0, seed: int = 5, shuffle: bool = True) -> np.ndarray:
    """Random geometric graph on the unit square, radius sqrt(avg_degree / (pi n)).

    Returns the simple graph's pairs (each once), in random order and direction
    when shuffle is set.
    """
    r = math.sqrt(avg_degree / (math.pi * n))
    lib = _load()
    cap = int(n * avg_degree / 2 * 1.05) + 1024
    while True:
        out = np.empty((cap, 2), dtype=np.int32)
        total = lib.gg_rgg(n, r, seed, _i32p(out), cap)
        if total <= cap:
            break
        cap = int(total)
    out = out[:total]
    if shuffle:
        out = np.ascontiguousarray(out)
        lib.gg_shuffle_edges(_i32p(out), out.shape[0], _sub_seed(seed, 3))
    return out


def shuffle_edges(e: np.ndarray, seed: int) -> np.ndarray:
    """Copy of e in a seeded random order, each pair in a random direction."""
    out = np.ascontiguousarray(e, dtype=np.int32).copy()
    _load().gg_shuffle_edges(_i32p(out), out.shape[0], seed)
    return out


# ---- small structured graphs with closed-form triangle counts (used as pins) ----

def complete(n: int) -> np.ndarray:
    i, j = np.triu_indices(n, 1)
    return np.stack([i, j], 1).astype(np.int32)


def complete_bipartite(a: int, b: int) -> np.ndarray:
    i, j = np.meshgrid(np.arange(a), a + np.arange(b), indexing="ij")
    return np.stack([i.ravel(), j.ravel()], 1).astype(np.int32)


def complete_tripartite(a: int, b: int, c: int) -> np.ndarray:
    parts = [np.arange(a), a + np.arange(b), a + b + np.arange(c)]
    out = []
    for x in range(3):
        for y in range(x + 1, 3):
            i, j = np.meshgrid(parts[x], parts[y], indexing="ij")
            out.append(np.stack([i.ravel(), j.ravel()], 1))
    return np.concatenate(out).astype(np.int32)


def grid2d(rows: int, cols: int) -> np.ndarray:
    idx = np.arange(rows * cols).reshape(rows, cols)
    h = np.stack([idx[:, :-1].ravel(), idx[:, 1:].ravel()], 1)
    v = np.stack([idx[:-1, :].ravel(), idx[1:, :].ravel()], 1)
    return np.concatenate([h, v]).astype(np.int32)


def cycle(k: int) -> np.ndarray:
    i = np.arange(k)
    return np.stack([i, (i + 1) % k], 1).astype(np.int32)


def wheel(k: int) -> np.ndarray:
    """Hub 0 joined to a k-cycle on vertices 1..k."""
    rim = cycle(k) + 1
    spokes = np.stack([np.zeros(k, dtype=np.int64), 1 + np.arange(k)], 1)
    return np.concatenate([rim, spokes]).astype(np.int32)


def friendship(k: int) -> np.ndarray:
    """k triangles sharing vertex 0 (windmill graph F_k), 2k+1 vertices."""
    out = []
    for t in range(k):
        a, b = 1 + 2 * t, 2 + 2 * t
        out += [(0, a), (0, b), (a, b)]
    return np.array(out, dtype=np.int32).reshape(-1, 2)


def star(k: int) -> np.ndarray:
    return np.stack([np.zeros(k, dtype=np.int64), 1 + np.arange(k)], 1).astype(np.int32)


def spread_hubs(n: int = 1 << 21, background: int = 2_000_000, hubs: int = 64, pool: int = 8000,
                pool_degree: int = 4000, spread_degree: int = 1000, seed: int = 21) -> np.ndarray:
    """Hubs whose neighbourhoods reach across the whole vertex range.

    A uniform background of ``background`` random pairs over n vertices (low
    degrees, so their degree ranks spread over the range); ``hubs`` vertices
    joined in a clique; each hub joined to ``pool_degree`` vertices of a shared
    pool of ``pool`` vertices (many triangles through hub pairs) and to
    ``spread_degree`` uniform random vertices. numpy PCG64(seed); repeats and
    loops may occur (the counting path drops them). Random order and direction.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    bg = rng.integers(0, n, size=(background, 2), dtype=np.int64)
    ids = rng.choice(n, size=hubs + pool, replace=False)
    H, P = ids[:hubs], ids[hubs:]
    i, j = np.triu_indices(hubs, 1)
    clique = np.stack([H[i], H[j]], 1)
    parts = [bg, clique]
    for h in H:
        nb = rng.choice(P, size=pool_degree, replace=False)
        parts.append(np.stack([np.full(pool_degree, h), nb], 1))
        sp = rng.integers(0, n, size=spread_degree, dtype=np.int64)
        parts.append(np.stack([np.full(spread_degree, h), sp], 1))
    e = np.concatenate(parts)
    e = e[rng.permutation(e.shape[0])]
    flip = rng.random(e.shape[0]) < 0.5
    e[flip] = e[flip][:, ::-1]
    return np.ascontiguousarray(e, dtype=np.int32)
