"""Learned kernel selection: timing collection, labels, training, persistence.

The counting path groups the middle vertices of the oriented graph into
degree-pair buckets and runs one of three intersection strategies per bucket
(merge path, binary search, LDS bitmap). This module trains the small
network that picks the strategy:

1. ``collect``: for each training graph, the library times every strategy on
   every bucket's tiles alone (``profile_buckets``) and reports the bucket
   features.
2. ``make_labels``: the fastest strategy per bucket by median time; within
   ``tie`` (relative) or ``abs_tie`` (ms) of it the heuristic's choice is kept.
3. ``train``: full-batch Adam on the GPU with the library's own forward and
   backward kernels (``selector_train_step``); samples are weighted by how
   much time the choice can save.
4. ``save`` / ``load``: float32 master parameters as JSON.

The fixed-threshold heuristic (``heuristic_choice``) is the fallback and the
baseline the learned choice is compared with.
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import _lib

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "selector_weights.json")
KERNELS = ("merge", "bsearch", "bitmap")


def heuristic_choice(bucket: int) -> int:
    """The library's fixed thresholds (same rule as the device code)."""
    li, lo = bucket >> 4, bucket & 15
    if li >= 6 or (li >= 4 and lo >= 6):
        return 2
    if lo >= 4:
        return 1
    return 0


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights, zero biases (float32, 1379 entries)."""
    rng = np.random.default_rng(seed)
    shapes = [(32, 6), (32,), (32, 32), (32,), (3, 32), (3,)]
    parts = []
    for s in shapes:
        if len(s) == 2:
            parts.append(rng.normal(0.0, np.sqrt(2.0 / s[1]), size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts).astype(np.float32)


def collect(graphs, repeats: int = 5, device: str = "cuda:0", log=None):
    """Time every strategy on every busy bucket of each graph.

    graphs: iterable of (name, edges int32 [E, 2] numpy, num_vertices).
    Returns a dict of arrays: features [N, 6], times [N, 3] (ms), bucket [N],
    graph [N] (index into names), and names.
    """
    import torch
    feats, times, buckets, gids, names = [], [], [], [], []
    for gi, (name, edges, n) in enumerate(graphs):
        d = torch.from_numpy(np.ascontiguousarray(edges, dtype=np.int32)).to(device)
        ms, feat = _lib.profile_buckets(d, n, repeats=repeats)
        for b in range(255):
            if np.all(ms[:, b] > 0):
                feats.append(feat[b])
                times.append(ms[:, b])
                buckets.append(b)
                gids.append(gi)
        names.append(name)
        if log:
            log(f"[selector] collected {name}: {sum(1 for g in gids if g == gi)} buckets")
        del d
    return {"features": np.array(feats, dtype=np.float32).reshape(-1, 6),
            "times": np.array(times, dtype=np.float64).reshape(-1, 3),
            "bucket": np.array(buckets, dtype=np.int64), "graph": np.array(gids, dtype=np.int64),
            "names": names}


def collect_in_launch(graphs, repeats: int = 7, device: str = "cuda:0", log=None, min_tie_ms: float = 0.004):
    """Time each strategy for each busy bucket inside the combined launch.

    For each graph the whole intersection stage (three kernels over their tile
    ranges, as a counting call launches them) is timed with the fixed thresholds'
    choice everywhere, then once per (busy bucket, other strategy) with only that
    bucket changed. times[i, k] = stage time with bucket i on strategy k (the others
    on the heuristic's), so times[i, k] - times[i].min() is the time that choice
    costs in the combined launch. The baseline is re-timed between the changes; the
    spread of those repeats (noise_ms) sets how large a difference must be to count.
    graphs: iterable of (name, edges int32 [E, 2] numpy, num_vertices). Returns the
    dict of collect() plus noise_ms [N] (per bucket, its graph's baseline spread).
    """
    import torch
    feats, times, buckets, gids, names, noise = [], [], [], [], [], []
    for gi, (name, edges, n) in enumerate(graphs):
        d = torch.from_numpy(np.ascontiguousarray(edges, dtype=np.int32)).to(device)
        T = _lib.count_triangles(d, n)
        st = _lib.last_stats(device)
        feat = _lib.bucket_features(device)
        heur = st["bucket_kernel"].astype(int)
        busy = [b for b in range(255) if st["bucket_vertices"][b] > 0]
        base = np.full(256, 255, dtype=np.uint8)
        bases = []

        def stage(choice):
            ms, _, Tx = _lib.profile_choices(d, n, choice, repeats=repeats)
            assert Tx == T, (name, Tx, T)
            return ms

        bases.append(stage(base))
        rows = []
        for j, b in enumerate(busy):
            t = np.zeros(3)
            for k in range(3):
                if k == heur[b]:
                    continue
                c = base.copy()
                c[b] = k
                t[k] = stage(c)
            rows.append(t)
            if j % 8 == 7:
                bases.append(stage(base))
        bases.append(stage(base))
        t_base = float(np.median(bases))
        spread = float(np.max(bases) - np.min(bases))
        for b, t in zip(busy, rows):
            t[heur[b]] = t_base
            feats.append(feat[b])
            times.append(t)
            buckets.append(b)
            gids.append(gi)
            noise.append(max(spread, min_tie_ms))
        names.append(name)
        if log:
            log(f"[selector] collected {name}: {len(busy)} buckets, stage {t_base:.3f} ms "
                f"(baseline spread {spread * 1e3:.1f} us over {len(bases)} repeats)")
        del d
    return {"features": np.array(feats, dtype=np.float32).reshape(-1, 6),
            "times": np.array(times, dtype=np.float64).reshape(-1, 3),
            "bucket": np.array(buckets, dtype=np.int64), "graph": np.array(gids, dtype=np.int64),
            "names": names, "noise_ms": np.array(noise, dtype=np.float64)}


def make_labels_in_launch(times: np.ndarray, buckets: np.ndarray, noise_ms: np.ndarray) -> np.ndarray:
    """Fastest strategy per bucket in the combined launch; the heuristic's unless
    another is faster by more than the baseline's repeat spread."""
    best = np.argmin(times, axis=1)
    heur = np.array([heuristic_choice(int(b)) for b in buckets])
    idx = np.arange(len(best))
    keep = times[idx, heur] - times[idx, best] <= noise_ms
    return np.where(keep, heur, best).astype(np.int32)


def make_labels(times: np.ndarray, buckets: np.ndarray, tie: float = 0.02, abs_tie: float = 0.005) -> np.ndarray:
    """Fastest strategy per bucket; the heuristic's when its time is within `tie`
    (relative) or `abs_tie` ms of the best. A bucket timed alone costs at least one
    launch's fixed time (~13 us), and differences of a few microseconds there do not
    carry over to the bucket's share of the combined launch of its strategy."""
    best = np.argmin(times, axis=1)
    heur = np.array([heuristic_choice(int(b)) for b in buckets])
    t_best = times[np.arange(len(best)), best]
    keep = times[np.arange(len(best)), heur] <= np.maximum((1.0 + tie) * t_best, t_best + abs_tie)
    return np.where(keep, heur, best).astype(np.int32)


def sample_weights(times: np.ndarray) -> np.ndarray:
    """Weight each bucket by the time at stake (slowest minus fastest), mean 1."""
    stake = times.max(axis=1) - times.min(axis=1)
    w = np.sqrt(stake + 1e-6)
    return (w / w.mean()).astype(np.float32)


def train(features, labels, weights=None, steps: int = 3000, lr: float = 3e-3, seed: int = 0,
          device: str = "cuda:0", log=None):
    """Full-batch Adam on the GPU. Returns (params, losses)."""
    import torch
    _lib.selector_set_params(init_params(seed), device)
    x = torch.from_numpy(np.ascontiguousarray(features, dtype=np.float32)).to(device)
    y = torch.from_numpy(np.ascontiguousarray(labels, dtype=np.int32)).to(device)
    w = None if weights is None else torch.from_numpy(np.ascontiguousarray(weights, dtype=np.float32)).to(device)
    losses = []
    for step in range(steps):
        losses.append(_lib.selector_train_step(x, y, w, lr=lr))
        if log and (step % 500 == 0 or step == steps - 1):
            log(f"[selector] step {step} loss {losses[-1]:.4f}")
    return _lib.selector_get_params(device), losses


def predict(features, device: str = "cuda:0") -> np.ndarray:
    import torch
    x = torch.from_numpy(np.ascontiguousarray(features, dtype=np.float32)).to(device)
    return _lib.selector_forward(x).argmax(dim=1).cpu().numpy()


def regret(times: np.ndarray, choices: np.ndarray) -> float:
    """Sum over buckets of (time of the chosen strategy - best time), ms."""
    idx = np.arange(times.shape[0])
    return float(np.sum(times[idx, choices] - times.min(axis=1)))


def save(path: str, params: np.ndarray, meta: dict | None = None) -> None:
    doc = {"format": "tc-selector-v1", "num_params": int(params.size),
           "params": [float(x) for x in np.asarray(params, dtype=np.float32)], "meta": meta or {}}
    with open(path, "w") as f:
        json.dump(doc, f)


def load(path: str) -> np.ndarray:
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != "tc-selector-v1" or doc.get("num_params") != _lib.SELECTOR_NUM_PARAMS:
        raise ValueError(f"{path}: not a selector parameter file")
    return np.asarray(doc["params"], dtype=np.float32)


def load_default(device: str = "cuda:0") -> bool:
    """Load the packaged trained parameters into the device's context, if present."""
    if not os.path.exists(DEFAULT_WEIGHTS):
        return False
    _lib.selector_set_params(load(DEFAULT_WEIGHTS), device)
    return True
