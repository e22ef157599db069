#!/usr/bin/env python
"""Benchmark: exact triangle counting on one MI355X.

One step = one full pass of the counting path over one resident graph:
validate/canonicalise, degree order, orient, radix sort -> CSR, de-duplicate,
degree-pair buckets, kernel selection, tiles, intersection, reduction, count
read back to the host. The input edge list is in HBM before timing starts.

Default workload: R-MAT scale 20, edge factor 16 (a, b, c, d = 0.57, 0.19, 0.19,
0.05), 16,777,216 raw draws over 1,048,576 vertices (random vertex permutation,
random direction); the counted graph is its symmetrised, loop-free,
de-duplicated version. Metric: Gedges/s = m / step time, m = unique undirected
edges (= oriented edges intersected).

Prints one JSON line (rank 0).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "Gedges/s intersected + HBM GB/s; learned/batched vs plain speedup, exact"

WORKLOADS = {
    "rmat20": dict(kind="rmat", scale=20, edge_factor=16, seed=1),
    "rmat18": dict(kind="rmat", scale=18, edge_factor=16, seed=1),
    "rmat22": dict(kind="rmat", scale=22, edge_factor=16, seed=1),
    "rmat24": dict(kind="rmat", scale=24, edge_factor=16, seed=1),
    "er4096": dict(kind="er", n=4096, m=32768, seed=1804),
    "uniform20": dict(kind="uniform", n=1 << 20, pairs=16 << 20, seed=7),
    "rgg23": dict(kind="rgg", n=1 << 23, avg_degree=32.0, seed=5),
    "clbatch": dict(kind="batch"),
}


def make_graph(name):
    import graphgen
    w = WORKLOADS[name]
    if w["kind"] == "rmat":
        return graphgen.rmat(w["scale"], w["edge_factor"], seed=w["seed"]), 1 << w["scale"], w
    if w["kind"] == "er":
        return graphgen.erdos_renyi(w["n"], w["m"], seed=w["seed"]), w["n"], w
    if w["kind"] == "uniform":
        import numpy as np
        rng = np.random.Generator(np.random.PCG64(w["seed"]))
        return rng.integers(0, w["n"], size=(w["pairs"], 2), dtype=np.int32), w["n"], w
    return graphgen.rgg(w["n"], w["avg_degree"], seed=w["seed"]), w["n"], w


def counted_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE passes scaled by a copy of known size), or None when
    there is none for this workload or the kernel source changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.md")
    src = os.path.join(ROOT, "paper_1804_06926_amd", "csrc", "isect.hip")
    if not os.path.exists(path):
        return None
    fields = {}
    with open(path) as f:
        for line in f:
            if ": " in line and not line.startswith(("|", "#", " ")):
                k, v = line.strip().split(": ", 1)
                fields[k] = v
    with open(src, "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()
    key = f"{kernel}_traffic_bytes"
    if fields.get("isect_source_sha256") != digest or key not in fields:
        return None
    return float(fields[key])


def algorithmic_bytes(tc, d_edges, n, stats):
    """Compulsory global reads of each intersection kernel for this graph.

    Per in-edge e = (u -> v) with a non-empty tail: 8 B (its entry) + 4 B per
    tail element; per tile (v, chunk of in-edges): 16 B of descriptors and
    offsets + 4 B per element of N+(v). The same figure holds for every
    strategy (each must read the tail and N+(v) at least once).
    """
    import numpy as np
    rank, off, col = tc.build_csr(d_edges, n)
    off = off.cpu().numpy().astype(np.int64)
    col = col.cpu().numpy().astype(np.int64)
    m = col.shape[0]
    dplus = np.diff(off)
    src = np.repeat(np.arange(n, dtype=np.int64), dplus)
    tail = off[src + 1] - np.arange(m) - 1
    active = (tail > 0) & (dplus[col] > 0)
    din = np.bincount(col[active], minlength=n)
    li = np.minimum(14, np.floor(np.log2(np.maximum(din, 1)))).astype(np.int64)
    lo = np.minimum(15, np.floor(np.log2(np.maximum(dplus, 1)))).astype(np.int64)
    bucket = np.where((din > 0) & (dplus > 0), 16 * li + lo, 255)
    kern = np.asarray(stats["bucket_kernel"], dtype=np.int64)[bucket]
    chunk = np.asarray(stats["bucket_chunk"], dtype=np.int64)[bucket]
    tiles = np.where(bucket != 255, (din + chunk - 1) // np.maximum(chunk, 1), 0)
    out = {}
    ek = kern[col[active]]
    for k, name in enumerate(("merge", "bsearch", "bitmap")):
        e_bytes = int((8 + 4 * tail[active][ek == k]).sum())
        t_bytes = int((tiles[kern == k] * (16 + 4 * dplus[kern == k])).sum())
        out[name] = e_bytes + t_bytes
    S = int((dplus[col]).sum())
    balg = 4 * (m + S) + 16 * m + 8 * (n + 1)   # merge-formulation minimum
    # list elements each formulation streams over all kept edges (u -> v), before
    # any window clipping: tails; whole rows N(u); rows N+(u)
    deg = dplus + np.bincount(col, minlength=n)
    elems = {"filtered": int(tail[active].sum()), "full": int(deg[src].sum()),
             "matrix": int(dplus[src].sum()), "matrix_upper": int(dplus[src].sum())}
    return out, balg, int(tail[active].sum()), elems


def formulation_compare(tc, d_edges, n, T, steps, elems):
    """The full-list and matrix formulations timed on the same graph; each
    count asserted equal to the filtered one."""
    import torch
    out = {}
    for form in ("full", "matrix", "matrix_upper"):
        tc.count_triangles_formulation(d_edges, n, form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):   # whole steps, without per-stage events
            Tf, total = tc.count_triangles_formulation(d_edges, n, form)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
        assert Tf == T, (form, Tf, T)
        isect = {}
        for _ in range(steps):   # the same steps with events at the stage boundaries
            _, _, st = tc.count_triangles_formulation(d_edges, n, form, timing=True)
            for k, v in st.items():
                if k.startswith("isect_"):
                    isect[k[6:]] = isect.get(k[6:], 0.0) + v / max(steps, 1)
        out[form] = {"ms_per_step": ms,
                     "isect_ms": sum(isect.values()), "isect_ms_by_kernel": isect, "sum": total,
                     "streamed_elements": elems[form]}
    return out


def cpu_baseline(edges, n, m):
    """The CPU oracle (forward algorithm, OpenMP) on the same graph, whole."""
    import oracle
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    t0 = time.perf_counter()
    g = oracle.Graph(edges, n, threads=threads)
    T = g.count()
    dt = time.perf_counter() - t0
    return {"value": m / dt / 1e9, "unit": "Gedges/s", "cores": threads, "kind": "oracle",
            "sample": f"whole graph (canonicalise + CSR + count), {dt:.2f} s", "T": T}


def batch_bench(args, tc, autotune, sel):
    """4096 Chung-Lu graphs (gamma 2.1, draws log-uniform in [1e3, 1e6], n_g = E_g / 8):
    one batched call (captured graph replayed) against 4096 separate calls."""
    import numpy as np
    import torch

    import graphgen
    print("[bench] clbatch generating 4096 graphs", file=sys.stderr, flush=True)
    edges, off, nv = graphgen.chung_lu_batch(4096)
    d = torch.from_numpy(edges).to("cuda:0")
    tuned = autotune.apply_cached(sel, "cuda:0")
    for _ in range(max(args.warmup, 1)):
        counts = tc.count_triangles_batch(d, off, nv, select=sel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts = tc.count_triangles_batch(d, off, nv, select=sel)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / max(args.steps, 1)
    m = tc.last_stats("cuda:0")["m"]
    print(f"[bench] batched: {ms_batch:.2f} ms/step, union m={m}", file=sys.stderr, flush=True)
    # the same graphs through 4096 plain calls (one warm pass, then one timed pass), with the
    # default tile shapes (the tuned ones are for the batch's union graph)
    tc.set_tile_shapes(device="cuda:0")
    sep = np.zeros(nv.size, dtype=np.uint64)
    for rep in range(2):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for g in range(nv.size):
            sep[g] = tc.count_triangles(d[off[g]:off[g + 1]], int(nv[g]), select=sel)
        torch.cuda.synchronize()
        ms_sep = (time.perf_counter() - t1) * 1e3
        print(f"[bench] separate pass {rep}: {ms_sep:.1f} ms", file=sys.stderr, flush=True)
    assert np.array_equal(sep, counts), "batched and separate counts differ"
    # the same 4096 calls queued without host synchronisation (one workspace, one result slot each)
    ws = torch.empty(max(tc.workspace_size(int(off[g + 1] - off[g]), int(nv[g]), sel) for g in range(nv.size)),
                     dtype=torch.uint8, device="cuda:0")
    res = torch.empty((nv.size, 2), dtype=torch.int64, device="cuda:0")
    for rep in range(2):
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for g in range(nv.size):
            tc.count_triangles_async(d[off[g]:off[g + 1]], int(nv[g]), result=res[g], select=sel, workspace=ws)
        torch.cuda.synchronize()
        ms_async = (time.perf_counter() - t1) * 1e3
        print(f"[bench] async-queued pass {rep}: {ms_async:.1f} ms", file=sys.stderr, flush=True)
    r = res.cpu().numpy()
    assert np.all(r[:, 1] == 0) and np.array_equal(r[:, 0].astype(np.uint64), counts), "async counts differ"
    result = {
        "metric": METRIC, "value": m / (ms_batch * 1e-3) / 1e9, "unit": "Gedges/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_batch, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "clbatch", "graphs": int(nv.size), "gamma": 2.1, "draws_loguniform": [1e3, 1e6],
                   "raw_pairs": int(edges.shape[0]), "n": int(nv.astype(np.int64).sum()), "m": m,
                   "triangles": int(counts.astype(np.int64).sum()), "select": args.select,
                   "autotuned_tiles": bool(tuned)},
        "roofline": None,
        "batched_vs_separate": {"ms_batched": ms_batch, "ms_separate_4096_calls": ms_sep,
                                "speedup": ms_sep / ms_batch, "ms_async_queued_4096_calls": ms_async,
                                "speedup_vs_async": ms_async / ms_batch},
    }
    print(json.dumps(result), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat20", choices=sorted(WORKLOADS))
    ap.add_argument("--select", default="heuristic", choices=["heuristic", "learned", "merge", "bsearch", "bitmap"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle equality check")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-selector comparison (profiling runs: one selection mode only)")
    ap.add_argument("--formulations", action="store_true",
                    help="also time the full-list and matrix formulations on the same graph")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (calibrates counter-based traffic)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(the multi-GPU sharding is described in DESIGN.md, not implemented)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import __graft_entry__
    __graft_entry__._ensure_built()
    import paper_1804_06926_amd as tc

    from paper_1804_06926_amd import autotune, selector
    have_weights = selector.load_default("cuda:0")
    if args.select == "learned" and not have_weights:
        print("bench.py: --select learned needs trained selector weights "
              f"({selector.DEFAULT_WEIGHTS})", file=sys.stderr)
        return 2
    sel = {"heuristic": tc.SELECT_HEURISTIC, "learned": tc.SELECT_LEARNED, "merge": tc.FORCE_MERGE,
           "bsearch": tc.FORCE_BSEARCH, "bitmap": tc.FORCE_BITMAP}[args.select]
    if args.copy_probe > 0:
        src = torch.ones(args.copy_probe << 18, dtype=torch.int32, device="cuda:0")   # MiB of int32
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.workload == "clbatch":
        return batch_bench(args, tc, autotune, sel)
    print(f"[bench] workload={args.workload} generating", file=sys.stderr, flush=True)
    edges, n, spec = make_graph(args.workload)
    d_edges = torch.from_numpy(edges).to("cuda:0")
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        T = tc.count_triangles(d_edges, n, select=sel)
    torch.cuda.synchronize()
    print(f"[bench] warmup done T={T}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        T = tc.count_triangles(d_edges, n, select=sel)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = dt * 1e3 / max(args.steps, 1)
    # After the timed region: the same steps again with HIP events recorded on the
    # library's stream at every stage boundary (each record leaves a few
    # microseconds between kernels, so these runs are not the ones timed above).
    # They give the per-stage times and the dominant kernel's launch duration.
    stage_sum = {}
    for _ in range(args.steps):
        T_s, st = tc.count_triangles(d_edges, n, select=sel, timing=True)
        assert T_s == T, (T_s, T)
        for k, v in st.items():
            stage_sum[k] = stage_sum.get(k, 0.0) + v
    stages = {k: v / max(args.steps, 1) for k, v in stage_sum.items()}
    stats = tc.last_stats("cuda:0")
    m = stats["m"]
    print(f"[bench] timed {args.steps} steps: {ms_per_step:.3f} ms/step T={T} m={m}", file=sys.stderr, flush=True)

    kbytes, balg, tail_sum, elems = algorithmic_bytes(tc, d_edges, n, stats)
    isect = {k: stages.get(f"isect_{k}", 0.0) for k in ("merge", "bsearch", "bitmap")}
    dom = max(isect, key=isect.get)
    dom_ms = isect[dom]
    achieved = kbytes[dom] / (dom_ms * 1e-3) / 1e9 if dom_ms > 0 else 0.0
    isect_ms = sum(isect.values())

    result = {
        "metric": METRIC,
        "value": m / (ms_per_step * 1e-3) / 1e9,
        "unit": "Gedges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": args.workload, **{k: v for k, v in spec.items() if k != "kind"},
                   "generator": spec["kind"], "raw_pairs": int(edges.shape[0]), "n": n, "m": m,
                   "triangles": T, "select": args.select},
        "roofline": {"bound": "hbm", "kernel": f"k_isect_{dom}", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counted_traffic(f"k_isect_{dom}", args.workload),
                     "algorithmic_bytes": kbytes[dom], "avg_launch_ms": dom_ms},
        "stages_ms": stages,
        "intersect_gedges_per_s": m / (isect_ms * 1e-3) / 1e9 if isect_ms > 0 else None,
        "tail_elements": tail_sum,
        "effective_gbps_merge_formulation": balg / (isect_ms * 1e-3) / 1e9 if isect_ms > 0 else None,
    }
    if have_weights and args.select == "heuristic" and not args.no_learned:
        # the learned selector against the heuristic on the same graph, counts equal
        for _ in range(2):
            T_l = tc.count_triangles(d_edges, n, select=tc.SELECT_LEARNED)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.steps):
            T_l = tc.count_triangles(d_edges, n, select=tc.SELECT_LEARNED)
        torch.cuda.synchronize()
        ms_l = (time.perf_counter() - t1) * 1e3 / max(args.steps, 1)
        assert T_l == T, (T_l, T)
        result["learned_vs_heuristic"] = {"ms_per_step_learned": ms_l, "ms_per_step_heuristic": ms_per_step,
                                          "speedup": ms_per_step / ms_l}
    if args.formulations and args.select == "heuristic":
        print("[bench] full-list and matrix formulations", file=sys.stderr, flush=True)
        forms = formulation_compare(tc, d_edges, n, T, args.steps, elems)
        forms["filtered"] = {"ms_per_step": ms_per_step, "isect_ms": isect_ms, "sum": T,
                             "streamed_elements": elems["filtered"]}
        result["formulations"] = forms
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        cb = cpu_baseline(edges, n, m)
        if not args.no_check:
            assert cb["T"] == T, f"GPU count {T} != oracle {cb['T']}"
        cb.pop("T")
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
