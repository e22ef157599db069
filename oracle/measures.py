"""Triangle-based graph measures on the CPU. TEST INFRASTRUCTURE ONLY.

Section 1 names the clustering coefficient and the transitivity ratio as the
measures built on triangle counts, and the end of Section 5 notes that the
method extends to them. Definitions (Watts and Strogatz for the local
coefficient; transitivity as the fraction of wedges that close):
  * d(v): degree of v in the simple graph (loops and repeats dropped);
  * wedges(v) = C(d(v), 2), the paths of two edges centred at v;
  * C(v) = t[v] / wedges(v), or 0 when d(v) < 2;
  * transitivity = 3 T / sum_v wedges(v), or 0 without wedges.
Each ratio is one correctly rounded float64 division of exact integers, each
converted to float64 first; the transitivity multiplies 3.0 by T before it
divides.
"""
from __future__ import annotations

import numpy as np

from . import Graph


def clustering(edges: np.ndarray, n: int, threads: int = 0):
    """(coeff float64 [n], T, wedges, transitivity, t uint64 [n])."""
    g = Graph(edges, n, threads)
    T, t = g.count(per_vertex=True)
    d = g.degrees().astype(np.uint64)
    w = np.where(d >= 2, d * (d - np.uint64(1)) // np.uint64(2), np.uint64(0)).astype(np.uint64)
    coeff = np.zeros(n, dtype=np.float64)
    nz = w > 0
    coeff[nz] = t[nz].astype(np.float64) / w[nz].astype(np.float64)
    W = int(w.sum(dtype=np.uint64))
    tr = 3.0 * float(T) / float(W) if W else 0.0
    return coeff, int(T), W, tr, t
