#!/usr/bin/env python
"""Write tests/golden/large_counts.json: the oracle's exact results on the
full-size workloads, for the whole-graph GPU parity tests.

Only the seeded generators (graphgen) and the CPU oracle (oracle/) run here;
nothing comes from the GPU library. Every value is the oracle's forward
algorithm (Section 3.2, Algorithm 2, with the degree filter of Section 4.2):

  rmat24   R-MAT scale 24, edge factor 16, seed 1 (raw draws with loops and
           repeats): T, m, t[v] for every vertex, and the per-edge intersection
           sizes of the forward algorithm for every kept edge (orientation by
           the number of input pairs at a vertex, then id: the order the
           library uses on input with repeats), in canonical pair order.
  rgg23    random geometric graph, 2^23 vertices, average degree 32, seed 5
           (no repeats): the same, orientation by simple degree.
  clbatch  the 4096 Chung-Lu graphs (gamma 2.1, draws log-uniform in
           [1e3, 1e6], n_g = E_g / 8): T of every graph.

Vectors too large to store are kept as the SHA-256 of their little-endian
bytes: t[v] (uint64), the per-edge counts (uint32) and the canonical edge
keys a << 32 | b, a < b, ascending (uint64), with the sums of the counts.
Takes about 10 minutes on 8 cores.

    python tests/golden/make_large_golden.py [--only rmat24,rgg23,clbatch]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(HERE, "large_counts.json")


def sha256(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def whole_graph(name, edges, n, degree):
    t0 = time.time()
    g = oracle.Graph(edges, n)
    T, t = g.count(per_vertex=True)
    c = g.forward_edge_counts(degree)
    assert int(t.sum()) == 3 * T and int(c.astype(np.uint64).sum()) == T
    pe = g.edges().astype(np.uint64)
    keys = (pe[:, 0] << np.uint64(32)) | pe[:, 1]   # canonical pairs a < b, ascending
    del pe
    print(f"[golden] {name}: m={g.m} T={T} ({time.time() - t0:.0f} s)", flush=True)
    return {"n": n, "raw_pairs": int(edges.shape[0]), "m": g.m, "triangles": T,
            "edge_keys_sha256_u64le": sha256(keys.astype("<u8")),
            "t_sha256_u64le": sha256(t.astype("<u8")), "t_sum": int(t.sum()),
            "edge_counts_degree": degree, "edge_counts_sha256_u32le": sha256(c.astype("<u4")),
            "edge_counts_sum": int(c.astype(np.uint64).sum()), "max_edge_count": int(c.max()) if c.size else 0}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--only", default="rmat24,rgg23,clbatch")
    args = ap.parse_args(argv)
    doc = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            doc = json.load(f)
    doc["_about"] = ("Exact results of the CPU oracle (forward algorithm, Section 3.2 / Algorithm 2) on the "
                     "full-size synthetic workloads; written by tests/golden/make_large_golden.py, which "
                     "calls only graphgen and oracle.")
    for name in args.only.split(","):
        if name == "rmat24":
            doc["rmat24"] = {"generator": "rmat", "scale": 24, "edge_factor": 16, "seed": 1,
                             **whole_graph(name, graphgen.rmat(24, 16, seed=1), 1 << 24, "input")}
        elif name == "rgg23":
            doc["rgg23"] = {"generator": "rgg", "avg_degree": 32.0, "seed": 5,
                            **whole_graph(name, graphgen.rgg(1 << 23, 32.0, seed=5), 1 << 23, "simple")}
        elif name == "clbatch":
            t0 = time.time()
            e, off, nv = graphgen.chung_lu_batch(4096)
            counts = [oracle.count_triangles(e[off[g]:off[g + 1]], int(nv[g])) for g in range(nv.size)]
            print(f"[golden] clbatch: {nv.size} graphs, T sum {sum(counts)} ({time.time() - t0:.0f} s)", flush=True)
            doc["clbatch"] = {"generator": "chung_lu_batch", "graphs": int(nv.size), "gamma": 2.1,
                              "raw_pairs": int(e.shape[0]), "counts": [int(c) for c in counts]}
        else:
            raise SystemExit(f"unknown workload {name}")
        with open(OUT, "w") as f:
            json.dump(doc, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
