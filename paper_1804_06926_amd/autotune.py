"""Tile-shape autotuner: in-edges per tile, per degree-pair bucket.

For each candidate tile size the library lays out the tiles and times every
busy bucket's tiles alone with the strategy its selection mode picks
(``profile_selected``); each bucket keeps its fastest size. Tile sizes change
the speed only, never the counts. Results are cached as JSON keyed by the GPU
architecture, the HIP runtime version and the selection mode.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tile_shapes.json")
CANDIDATES = (32, 64, 128, 256, 512, 1024, 2048)   # the bitmap kernel caps at 512


def device_key(select: int, device: str = "cuda:0") -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.device(device))
    arch = getattr(p, "gcnArchName", p.name)
    return f"{arch}|hip{torch.version.hip}|select{select}"


def tune(edges, num_vertices: int, select: int = _lib.SELECT_HEURISTIC, candidates=CANDIDATES, repeats: int = 3,
         device: str = "cuda:0", log=None):
    """Per-bucket best tile size [256] (0 = bucket idle) and the timing table [len(candidates), 256]."""
    table = np.full((len(candidates), 256), -1.0)
    for i, K in enumerate(candidates):
        _lib.set_tile_shapes(chunk=np.full(256, K, dtype=np.uint16), device=device)
        table[i] = _lib.profile_selected(edges, num_vertices, select=select, repeats=repeats)
        if log:
            log(f"[autotune] chunk {K}: {np.sum(table[i][table[i] > 0]):.3f} ms over busy buckets")
    _lib.set_tile_shapes(None, None, device=device)
    best = np.zeros(256, dtype=np.uint16)
    for b in range(256):
        col = table[:, b]
        ok = col > 0
        if ok.any():
            best[b] = candidates[int(np.argmin(np.where(ok, col, np.inf)))]
    return best, table


def save(shapes: np.ndarray, key: str, path: str = DEFAULT_CACHE) -> None:
    doc = {}
    if os.path.exists(path):
        with open(path) as f:
            doc = json.load(f)
    doc[key] = {str(b): int(k) for b, k in enumerate(shapes) if k}
    with open(path, "w") as f:
        json.dump(doc, f, indent=1, sort_keys=True)


def load(key: str, path: str = DEFAULT_CACHE):
    if not os.path.exists(path):
        return None
    with open(path) as f:
        doc = json.load(f)
    if key not in doc:
        return None
    out = np.zeros(256, dtype=np.uint16)
    for b, k in doc[key].items():
        out[int(b)] = k
    return out


def apply_cached(select: int = _lib.SELECT_HEURISTIC, device: str = "cuda:0", path: str = DEFAULT_CACHE) -> bool:
    """Install cached tile shapes for this device and mode; False if none are cached."""
    shapes = load(device_key(select, device), path)
    if shapes is None:
        return False
    _lib.set_tile_shapes(chunk=shapes, device=device)
    return True


def main(argv=None):
    """Tune on the disjoint union of the 4096-graph Chung-Lu batch (or an R-MAT graph)."""
    import argparse
    import sys
    import time

    import torch

    root = os.path.dirname(HERE)
    if root not in sys.path:
        sys.path.insert(0, root)
    import graphgen
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="clbatch", choices=["clbatch", "rmat20"])
    ap.add_argument("--select", type=int, default=_lib.SELECT_HEURISTIC)
    ap.add_argument("--out", default=DEFAULT_CACHE)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args(argv)

    def log(msg):
        print(msg, flush=True)

    t0 = time.time()
    if args.workload == "clbatch":
        e, off, nv = graphgen.chung_lu_batch(4096)
        base = np.zeros(nv.size, dtype=np.int64)
        np.cumsum(nv[:-1].astype(np.int64), out=base[1:])
        e = e + np.repeat(base, np.diff(off)).astype(np.int32)[:, None]
        n = int(nv.astype(np.int64).sum())
    else:
        e, n = graphgen.rmat(20, 16, seed=1), 1 << 20
    d = torch.from_numpy(np.ascontiguousarray(e, dtype=np.int32)).cuda()
    log(f"[autotune] {args.workload}: E={e.shape[0]} n={n}")
    if args.select == _lib.SELECT_LEARNED:
        from . import selector
        selector.load_default()
    best, table = tune(d, n, select=args.select, repeats=args.repeats, log=log)
    key = device_key(args.select)
    save(best, key, args.out)
    tot = {K: float(np.sum(table[i][table[i] > 0])) for i, K in enumerate(CANDIDATES)}
    picked = float(sum(table[CANDIDATES.index(int(best[b])), b] for b in range(256) if best[b]))
    log(f"[autotune] per-size totals (ms) {tot}; per-bucket best total {picked:.3f} ms; "
        f"saved under {key} in {args.out} ({time.time() - t0:.0f} s)")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
