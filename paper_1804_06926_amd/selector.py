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


SCALES = (0.5, 1.0, 2.0)   # the tile network's classes: the rule's tile size times these


def collect_in_launch(graphs, repeats: int = 7, device: str = "cuda:0", log=None, min_tie_ms: float = 0.004,
                      tiles: bool = True):
    """Time each (strategy, tile size) for each busy bucket inside the combined launch.

    For each graph the whole intersection stage (three kernels over their tile
    ranges, as a counting call launches them) is timed with the fixed thresholds'
    choice everywhere, then once per (busy bucket, strategy, tile scale) with only
    that bucket changed: the strategy, and its tiles at the rule's size for that
    strategy times 1/2, 1 or 2 (sizes the clamp leaves unchanged are not re-timed).
    times[i, k, s] = stage time with bucket i on strategy k at scale SCALES[s], the
    other buckets as the heuristic leaves them, so times[i] - times[i].min() is what
    each choice costs in the combined launch. The baseline is re-timed between the
    changes; the spread of those repeats (noise_ms) sets how large a difference must
    be to count. graphs: iterable of (name, edges int32 [E, 2] numpy, num_vertices).
    Returns features [N, 6], times [N, 3, 3] (ms; inf where a scale is not
    available), bucket [N], graph [N], names, noise_ms [N].
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

        def stage(choice, chunk=None):
            ms, _, Tx = _lib.profile_choices(d, n, choice, chunk, repeats=repeats)
            assert Tx == T, (name, Tx, T)
            return ms

        bases.append(stage(base))
        rows = []
        for j, b in enumerate(busy):
            t = np.full((3, 3), np.inf)
            for k in range(3):
                c = base.copy()
                c[b] = k
                if k != heur[b]:
                    t[k, 1] = stage(c)
                rule = int(_lib.last_stats(device)["bucket_chunk"][b]) if k != heur[b] else \
                    int(st["bucket_chunk"][b])
                if not tiles:
                    continue
                cap = 512 if k == 2 else 2048
                for si, f in ((0, 0.5), (2, 2.0)):
                    size = min(cap, max(16, int(rule * f)))
                    if size == rule:
                        continue
                    ch = np.zeros(256, dtype=np.uint16)
                    ch[b] = size
                    t[k, si] = stage(c, ch)
            rows.append(t)
            if j % 4 == 3:
                bases.append(stage(base))
        bases.append(stage(base))
        t_base = float(np.median(bases))
        spread = float(np.max(bases) - np.min(bases))
        for b, t in zip(busy, rows):
            t[heur[b], 1] = t_base
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
            "times": np.array(times, dtype=np.float64).reshape(-1, 3, 3),
            "bucket": np.array(buckets, dtype=np.int64), "graph": np.array(gids, dtype=np.int64),
            "names": names, "noise_ms": np.array(noise, dtype=np.float64)}


def make_labels_in_launch(times: np.ndarray, buckets: np.ndarray, noise_ms: np.ndarray):
    """Fastest (strategy, tile scale) per bucket in the combined launch; the fixed
    thresholds' (strategy, rule size) unless another is faster by more than the
    baseline's repeat spread. Returns (strategy labels, scale labels), int32 [N]."""
    N = times.shape[0]
    flat = times.reshape(N, 9)
    best = np.argmin(flat, axis=1)
    heur = np.array([heuristic_choice(int(b)) for b in buckets])
    idx = np.arange(N)
    keep = flat[idx, heur * 3 + 1] - flat[idx, best] <= noise_ms
    pick = np.where(keep, heur * 3 + 1, best)
    return (pick // 3).astype(np.int32), (pick % 3).astype(np.int32)


def in_launch_regret(times: np.ndarray, kernels: np.ndarray, scales: np.ndarray) -> float:
    """Sum over buckets of (stage time with the chosen strategy and scale - the best), ms.
    A scale that is not available for the chosen strategy counts as the rule's size."""
    idx = np.arange(times.shape[0])
    t = times[idx, kernels, scales]
    t = np.where(np.isfinite(t), t, times[idx, kernels, 1])
    return float(np.sum(t - times.reshape(times.shape[0], 9).min(axis=1)))


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
    """Weight each bucket by the time at stake (slowest minus fastest available), mean 1."""
    t = times.reshape(times.shape[0], -1)
    fin = np.where(np.isfinite(t), t, np.nan)
    stake = np.nanmax(fin, axis=1) - np.nanmin(fin, axis=1)
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


def save(path: str, params: np.ndarray, meta: dict | None = None, tile_params: np.ndarray | None = None) -> None:
    doc = {"format": "tc-selector-v1", "num_params": int(params.size),
           "params": [float(x) for x in np.asarray(params, dtype=np.float32)], "meta": meta or {}}
    if tile_params is not None:
        doc["tile_params"] = [float(x) for x in np.asarray(tile_params, dtype=np.float32)]
    with open(path, "w") as f:
        json.dump(doc, f)


def load(path: str) -> np.ndarray:
    """The strategy network's parameters."""
    with open(path) as f:
        doc = json.load(f)
    if doc.get("format") != "tc-selector-v1" or doc.get("num_params") != _lib.SELECTOR_NUM_PARAMS:
        raise ValueError(f"{path}: not a selector parameter file")
    return np.asarray(doc["params"], dtype=np.float32)


def load_tile(path: str):
    """The tile network's parameters, or None when the file has none."""
    with open(path) as f:
        doc = json.load(f)
    if "tile_params" not in doc:
        return None
    p = np.asarray(doc["tile_params"], dtype=np.float32)
    if p.size != _lib.SELECTOR_NUM_PARAMS:
        raise ValueError(f"{path}: bad tile network parameters")
    return p


def load_default(device: str = "cuda:0") -> bool:
    """Load the packaged trained networks into the device's context, if present."""
    if not os.path.exists(DEFAULT_WEIGHTS):
        return False
    _lib.selector_set_params(load(DEFAULT_WEIGHTS), device)
    _lib.selector_set_tile_params(load_tile(DEFAULT_WEIGHTS), device)
    return True
