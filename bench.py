#!/usr/bin/env python
"""Benchmark: exact triangle counting on one MI355X.

One step = one full pass of the counting path over one resident graph:
validate/canonicalise, degree order, orient, radix sort -> CSR, de-duplicate,
degree-pair buckets, kernel selection, tiles, intersection, reduction, count
read back to the host. The input edge list is in HBM before timing starts.

Default workload: R-MAT scale 24, edge factor 16 (a, b, c, d = 0.57, 0.19, 0.19,
0.05), 268,435,456 raw draws over 16,777,216 vertices (random vertex
permutation, random direction); the counted graph is its symmetrised,
loop-free, de-duplicated version. Metric: Gedges/s = m / step time, m = unique
undirected edges (= oriented edges intersected).

Beside the headline the line carries: the learned selector against the fixed
thresholds on the same graph (alternating blocks of steps, so the spread of
the ratio is stated), the latency of one count of an Erdos-Renyi G(4096, 32768)
graph, the batch of 4096 Chung-Lu graphs in one call against 4096 separate
calls (first call with graph capture reported apart from replays), and the
CPU oracle timed on a bounded sample of the same graph at all cores and at one
thread, stage by stage.

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


def _threads():
    return len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()


def cpu_oracle_leg(edges, n, threads, stride):
    """The CPU oracle (forward algorithm, OpenMP) on this graph: canonicalisation,
    degrees, orientation + out-lists whole; the intersections of every `stride`-th
    row (by vertex id), scaled by `stride` for the whole graph's estimate."""
    import oracle
    g = oracle.Graph(edges, n, threads=threads)
    canon_s, degree_s, adjacency_s = g.build_seconds
    T_rows, rows_edges = g.count_rows(stride)
    orient_s, isect_sample_s = g.count_seconds
    m = g.m
    isect_s = isect_sample_s * stride
    total_s = canon_s + degree_s + orient_s + isect_s
    return {"threads": threads, "row_stride": stride, "m": m,
            "seconds": {"canonicalise": canon_s, "degrees": degree_s, "orient_csr": orient_s,
                        "intersect_sample": isect_sample_s, "intersect_estimate": isect_s, "total_estimate": total_s,
                        "symmetric_adjacency_excluded": adjacency_s},
            "sample_rows_edges": rows_edges, "sample_triangles": T_rows,
            "gedges_per_s": m / total_s / 1e9}


def cpu_baseline(edges, n, all_stride, one_stride, one_thread=True):
    """The oracle timed on the host: all cores (the reported value) and one thread."""
    threads = _threads()
    allc = cpu_oracle_leg(edges, n, threads, all_stride)
    def desc(k):
        if k == 1:
            return "oracle forward algorithm on the whole graph (canonicalise + CSR + count), single run"
        return ("oracle forward algorithm on this graph: canonicalise (sort + unique), degrees, "
                f"orientation + out-lists run whole; intersections of every {k}-th row by vertex id "
                f"(ids randomly permuted), time x {k}; single run (the whole-graph run exceeds 60 s)")
    out = {"value": allc["gedges_per_s"], "unit": "Gedges/s", "cores": threads, "kind": "oracle",
           "sample": desc(all_stride), "stages_s": allc["seconds"], "row_stride": all_stride,
           "sample_triangles": allc["sample_triangles"]}
    if one_thread:
        one = cpu_oracle_leg(edges, n, 1, one_stride)
        out["one_thread"] = {"value": one["gedges_per_s"], "unit": "Gedges/s", "cores": 1,
                             "sample": desc(one_stride), "stages_s": one["seconds"],
                             "row_stride": one_stride}
    return out


def er_latency(tc, sel, calls=200):
    """One count of Erdos-Renyi G(4096, 32768) (seed 1804): host-synchronised calls
    back to back; latency-bound (a roofline fraction means nothing at this size)."""
    import numpy as np
    import torch

    import graphgen
    import oracle
    e = graphgen.erdos_renyi(4096, 32768, seed=1804)
    d = torch.from_numpy(e).to("cuda:0")
    for _ in range(20):
        T = tc.count_triangles(d, 4096, select=sel)
    torch.cuda.synchronize()
    times = []
    for _ in range(calls):
        t0 = time.perf_counter()
        T = tc.count_triangles(d, 4096, select=sel)
        times.append(time.perf_counter() - t0)
    us = float(np.median(times) * 1e6)
    cpu = []
    for _ in range(3):
        t0 = time.perf_counter()
        Tc = oracle.count_triangles(e, 4096, threads=1)
        cpu.append(time.perf_counter() - t0)
    assert Tc == T, (Tc, T)
    return {"workload": "er4096", "n": 4096, "m": 32768, "triangles": T, "us_per_count_median": us,
            "us_per_count_min": float(min(times) * 1e6), "us_per_count_max": float(max(times) * 1e6),
            "calls": calls, "gedges_per_s": 32768 / (us * 1e-6) / 1e9, "bound": "latency",
            "roofline": "not meaningful (launch and synchronisation latency)",
            "cpu_oracle_us_one_thread_median_of_3": float(np.median(cpu) * 1e6)}


def learned_compare(tc, d_edges, n, T, steps, blocks=5):
    """Heuristic and learned selection in alternating blocks of `steps` steps on the
    same resident graph, counts asserted equal; the ratio of each block pair gives the
    spread."""
    import numpy as np
    import torch
    for _ in range(2):
        assert tc.count_triangles(d_edges, n, select=tc.SELECT_LEARNED) == T
    ms = {"heuristic": [], "learned": []}
    for _ in range(blocks):
        for name, sel in (("heuristic", tc.SELECT_HEURISTIC), ("learned", tc.SELECT_LEARNED)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                Tx = tc.count_triangles(d_edges, n, select=sel)
            torch.cuda.synchronize()
            ms[name].append((time.perf_counter() - t0) * 1e3 / max(steps, 1))
            assert Tx == T, (name, Tx, T)
    ratios = np.array(ms["heuristic"]) / np.array(ms["learned"])
    return {"ms_per_step_learned": float(np.median(ms["learned"])),
            "ms_per_step_heuristic": float(np.median(ms["heuristic"])),
            "speedup": float(np.median(ms["heuristic"]) / np.median(ms["learned"])),
            "block_ratios": [float(x) for x in ratios], "ratio_min": float(ratios.min()),
            "ratio_max": float(ratios.max()), "blocks": blocks, "steps_per_block": steps,
            "triangles_equal": True}


def batch_compare(tc, autotune, sel, steps, warmup):
    """4096 Chung-Lu graphs (gamma 2.1, draws log-uniform in [1e3, 1e6], n_g = E_g / 8):
    one batched call (captured graph replayed) against 4096 separate calls; per-graph
    counts asserted equal between the two forms."""
    import numpy as np
    import torch

    import graphgen
    print("[bench] clbatch generating 4096 graphs", file=sys.stderr, flush=True)
    edges, off, nv = graphgen.chung_lu_batch(4096)
    d = torch.from_numpy(edges).to("cuda:0")
    tuned = autotune.apply_cached(sel, "cuda:0")
    # one direct (uncaptured) call first: the workspace and pinned buffers are allocated there
    c_direct = tc.count_triangles_batch(d, off, nv, select=sel, graph=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()   # first captured call: capture + instantiate + launch
    counts = tc.count_triangles_batch(d, off, nv, select=sel)
    ms_first = (time.perf_counter() - t0) * 1e3
    assert np.array_equal(c_direct, counts)
    for _ in range(max(warmup, 1)):
        counts = tc.count_triangles_batch(d, off, nv, select=sel)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        counts = tc.count_triangles_batch(d, off, nv, select=sel)
    torch.cuda.synchronize()
    ms_batch = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    t0 = time.perf_counter()   # the same batch without capture (kernels launched directly)
    for _ in range(steps):
        c_direct = tc.count_triangles_batch(d, off, nv, select=sel, graph=False)
    ms_direct = (time.perf_counter() - t0) * 1e3 / max(steps, 1)
    assert np.array_equal(c_direct, counts)
    m = tc.last_stats("cuda:0")["m"]
    print(f"[bench] batched: first {ms_first:.1f} ms, replay {ms_batch:.2f} ms, m={m}", file=sys.stderr, flush=True)
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
    r = res.cpu().numpy()
    assert np.all(r[:, 1] == 0) and np.array_equal(r[:, 0].astype(np.uint64), counts), "async counts differ"
    if tuned:
        tc.set_tile_shapes(device="cuda:0")
    del d, ws
    torch.cuda.synchronize()
    return {"workload": "clbatch", "graphs": int(nv.size), "raw_pairs": int(edges.shape[0]), "m": m,
            "triangles": int(counts.astype(np.int64).sum()), "autotuned_tiles": bool(tuned),
            "ms_batched_replay": ms_batch, "ms_batched_first_call_with_capture": ms_first,
            "ms_batched_without_capture": ms_direct,
            "ms_separate_4096_calls": ms_sep, "ms_async_queued_4096_calls": ms_async,
            "speedup": ms_sep / ms_batch, "speedup_first_call": ms_sep / ms_first,
            "speedup_vs_async": ms_async / ms_batch, "gedges_per_s_batched": m / (ms_batch * 1e-3) / 1e9,
            "counts_equal": True}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24", choices=sorted(WORKLOADS))
    ap.add_argument("--select", default="heuristic", choices=["heuristic", "learned", "merge", "bsearch", "bitmap"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-one-thread", action="store_true", help="CPU baseline at all cores only")
    ap.add_argument("--cpu-stride", type=int, default=0,
                    help="CPU baseline: intersect every k-th row at all cores (0: by graph size)")
    ap.add_argument("--cpu-one-thread-stride", type=int, default=0,
                    help="CPU baseline: intersect every k-th row at one thread (0: by graph size)")
    ap.add_argument("--no-check", action="store_true", help="skip the oracle equality check")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-selector comparison (profiling runs: one selection mode only)")
    ap.add_argument("--no-latency", action="store_true", help="skip the ER G(4096, 32768) latency")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-separate comparison")
    ap.add_argument("--formulations", action="store_true",
                    help="also time the full-list and matrix formulations on the same graph")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="also run one device-to-device copy of MIB MiB (calibrates counter-based traffic)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the counter runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sharding across GPUs is designed, not implemented)", file=sys.stderr)
        return 2

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
        b = batch_compare(tc, autotune, sel, args.steps, args.warmup)
        result = {
            "metric": METRIC, "value": b["gedges_per_s_batched"], "unit": "Gedges/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["ms_batched_replay"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
            "config": {"workload": "clbatch", "graphs": b["graphs"], "gamma": 2.1, "draws_loguniform": [1e3, 1e6],
                       "raw_pairs": b["raw_pairs"], "m": b["m"], "triangles": b["triangles"],
                       "select": args.select},
            "roofline": None, "batched_vs_separate": b}
        print(json.dumps(result), flush=True)
        return 0
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
                     "algorithmic_bytes": kbytes[dom], "avg_launch_ms": dom_ms,
                     "launch_ms_from": "HIP events at the stage boundaries, K steps after the timed region"},
        "stages_ms": stages,
        "intersect_gedges_per_s": m / (isect_ms * 1e-3) / 1e9 if isect_ms > 0 else None,
        "tail_elements": tail_sum,
        # what a per-edge merge of whole out-lists would read (4(m + S) + 16 m + 8(n + 1)
        # bytes); this path reads only the tails and each N+(v) once per tile, so this is
        # a size of work, not a bandwidth
        "merge_formulation_bytes": balg,
    }
    if have_weights and args.select == "heuristic" and not args.no_learned:
        print("[bench] learned vs heuristic", file=sys.stderr, flush=True)
        result["learned_vs_heuristic"] = learned_compare(tc, d_edges, n, T, args.steps)
    if args.formulations and args.select == "heuristic":
        print("[bench] full-list and matrix formulations", file=sys.stderr, flush=True)
        forms = formulation_compare(tc, d_edges, n, T, args.steps, elems)
        forms["filtered"] = {"ms_per_step": ms_per_step, "isect_ms": isect_ms, "sum": T,
                             "streamed_elements": elems["filtered"]}
        result["formulations"] = forms
    del d_edges
    torch.cuda.synchronize()
    if not args.no_latency:
        print("[bench] ER G(4096, 32768) latency", file=sys.stderr, flush=True)
        result["er4096_latency"] = er_latency(tc, sel)
    if not args.no_batch and args.select in ("heuristic", "learned"):
        result["batched_vs_separate"] = batch_compare(tc, autotune, sel, 3, 1)
    if not args.no_cpu_baseline:
        big = m > (1 << 26)
        all_stride = args.cpu_stride or (4 if big else 1)
        one_stride = args.cpu_one_thread_stride or (256 if big else 16)
        print(f"[bench] cpu baseline (oracle), row strides {all_stride} / {one_stride}", file=sys.stderr, flush=True)
        cb = cpu_baseline(edges, n, all_stride, one_stride, one_thread=not args.no_cpu_one_thread)
        if all_stride == 1 and not args.no_check:   # the whole graph was counted: same T
            assert cb["sample_triangles"] == T, f"GPU count {T} != oracle {cb['sample_triangles']}"
        result["cpu_baseline"] = cb
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
