"""Train the kernel-selector network on the GPU and evaluate it on held-out graphs.

Training graphs: R-MAT scales 18-22 (edge factor 16) and Chung-Lu graphs
(power-law exponent 2.1), all seeded apart from the benchmark and test graphs;
with --with-rgg also random geometric graphs of 2^17-2^21 vertices.
Held-out graphs: R-MAT scale 24 and a random geometric graph on 2^23 vertices
(average degree 32).

Labels come from the combined launch (selector.collect_in_launch): the whole
intersection stage is timed with one bucket's strategy changed at a time, so a
bucket's label reflects what it costs among the others, not alone (--labels
isolated takes the older per-bucket launches instead).

Writes the float32 parameters (JSON, see selector.save) and a report with the
per-graph regret of the learned choice, of the heuristic and of every single
strategy, and the end-to-end step time of the learned and heuristic modes
(alternating blocks, with the spread of the per-block ratio).

    python -m paper_1804_06926_amd.train_selector --out selector_weights.json --report report.json
    python -m paper_1804_06926_amd.train_selector --evaluate selector_weights.json --report report.json
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def log(msg):
    print(msg, flush=True)


def training_graphs(quick: bool, with_rgg: bool = False):
    import graphgen
    scales = (16, 17, 18) if quick else (18, 19, 20, 21, 22)
    for i, s in enumerate(scales):
        yield f"rmat{s}_seed{101 + i}", graphgen.rmat(s, 16, seed=101 + i), 1 << s
    sizes = ((1 << 16, 8 << 16), (1 << 17, 16 << 17)) if quick else \
        ((1 << 17, 8 << 17), (1 << 18, 16 << 18), (1 << 19, 8 << 19), (1 << 20, 16 << 20), (1 << 21, 8 << 21))
    for i, (n, E) in enumerate(sizes):
        yield f"chunglu_n{n}_seed{201 + i}", graphgen.chung_lu(n, E, 2.1, seed=201 + i), n
    if not with_rgg:
        return
    # mesh-like graphs: without them the network never sees buckets where merge
    # path beats binary search by a wide margin (sizes and seeds distinct from
    # the held-out random geometric graphs); one large size, since the edge
    # kernels' tile size, and with it their relative speed, grows with a
    # bucket's in-edges
    rsizes = (1 << 15, 1 << 16) if quick else (1 << 17, 1 << 18, 1 << 19, 1 << 21)
    for i, n in enumerate(rsizes):
        for j, deg in enumerate((16.0, 32.0)):
            yield f"rgg_n{n}_d{int(deg)}_seed{301 + 2 * i + j}", graphgen.rgg(n, deg, seed=301 + 2 * i + j), n


def heldout_graphs(quick: bool):
    import graphgen
    if quick:
        yield "rmat19_seed1", graphgen.rmat(19, 16, seed=1), 1 << 19
        yield "rgg_2^18", graphgen.rgg(1 << 18, 32.0, seed=5), 1 << 18
    else:
        yield "rmat24_seed1", graphgen.rmat(24, 16, seed=1), 1 << 24
        yield "rgg_2^23", graphgen.rgg(1 << 23, 32.0, seed=5), 1 << 23


def step_times(tc, d, n, steps=5, blocks=5):
    """Learned and heuristic steps in alternating blocks: (median ms learned, median ms
    heuristic, per-block heuristic/learned ratios, T)."""
    import torch
    T = tc.count_triangles(d, n, select=tc.SELECT_HEURISTIC)
    assert tc.count_triangles(d, n, select=tc.SELECT_LEARNED) == T
    ms = {tc.SELECT_LEARNED: [], tc.SELECT_HEURISTIC: []}
    for _ in range(blocks):
        for sel in (tc.SELECT_HEURISTIC, tc.SELECT_LEARNED):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                Tx = tc.count_triangles(d, n, select=sel)
            torch.cuda.synchronize()
            ms[sel].append((time.perf_counter() - t0) * 1e3 / steps)
            assert Tx == T, (sel, Tx, T)
    ratios = np.array(ms[tc.SELECT_HEURISTIC]) / np.array(ms[tc.SELECT_LEARNED])
    return float(np.median(ms[tc.SELECT_LEARNED])), float(np.median(ms[tc.SELECT_HEURISTIC])), ratios, T


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", help="where the trained weights go (required unless --evaluate)")
    ap.add_argument("--report", required=True)
    ap.add_argument("--repeats", type=int, default=5)
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--quick", action="store_true", help="small graphs (for a smoke run)")
    ap.add_argument("--with-rgg", action="store_true", help="random geometric graphs in the training set too")
    ap.add_argument("--labels", choices=["in-launch", "isolated"], default="in-launch")
    ap.add_argument("--no-heldout-profile", action="store_true",
                    help="held-out graphs: step times only (no per-bucket in-launch regret)")
    ap.add_argument("--evaluate", metavar="WEIGHTS",
                    help="skip training: evaluate these saved weights on the held-out graphs")
    args = ap.parse_args(argv)
    if not args.evaluate and not args.out:
        ap.error("--out is required when training")

    import torch

    import paper_1804_06926_amd as tc
    from paper_1804_06926_amd import selector

    t0 = time.time()
    if args.evaluate:
        params = (selector.load(args.evaluate), selector.load_tile(args.evaluate))
        report = {"train": {"weights": args.evaluate}}
    else:
        params, report = _train(args, tc, selector)
    _evaluate(args, tc, selector, params, report)
    report["wall_s"] = time.time() - t0
    with open(args.report, "w") as f:
        json.dump(report, f, indent=1)
    log(f"[selector] report written to {args.report}")
    return 0


def _train(args, tc, selector):
    graphs = training_graphs(args.quick, args.with_rgg)
    tile_params = None
    if args.labels == "in-launch":
        data = selector.collect_in_launch(graphs, repeats=args.repeats, log=log)
        y, ys = selector.make_labels_in_launch(data["times"], data["bucket"], data["noise_ms"])
    else:
        data = selector.collect(graphs, repeats=args.repeats, log=log)
        y, ys = selector.make_labels(data["times"], data["bucket"]), None
    w = selector.sample_weights(data["times"])
    log(f"[selector] {len(y)} training buckets; strategy labels {np.bincount(y, minlength=3).tolist()}"
        + (f", tile-scale labels {np.bincount(ys, minlength=3).tolist()}" if ys is not None else ""))
    report = {"train": {"buckets": int(len(y)), "graphs": data["names"]}}
    if ys is not None:   # the tile network first (the trainer's kernels work on one parameter set at a time)
        tile_params, tl = selector.train(data["features"], ys, w, steps=args.steps, lr=args.lr, seed=1, log=log)
        ps = selector.predict(data["features"])
        report["train"].update({"tile_accuracy": float(np.mean(ps == ys)), "tile_loss_last": tl[-1]})
    params, losses = selector.train(data["features"], y, w, steps=args.steps, lr=args.lr, log=log)
    pred = selector.predict(data["features"])
    heur = np.array([selector.heuristic_choice(int(b)) for b in data["bucket"]])
    report["train"].update({"accuracy": float(np.mean(pred == y)), "loss_first": losses[0], "loss_last": losses[-1]})
    if ys is not None:
        report["train"].update({
            "regret_learned_ms": selector.in_launch_regret(data["times"], pred, ps),
            "regret_learned_strategy_only_ms": selector.in_launch_regret(data["times"], pred, np.ones_like(pred)),
            "regret_heuristic_ms": selector.in_launch_regret(data["times"], heur, np.ones_like(heur))})
    else:
        report["train"].update({"regret_learned_ms": selector.regret(data["times"], pred),
                                "regret_heuristic_ms": selector.regret(data["times"], heur)})
    selector.save(args.out, params, {"trained_on": data["names"], "steps": args.steps, "lr": args.lr,
                                     "repeats": args.repeats, "labels": args.labels}, tile_params=tile_params)
    log(f"[selector] saved {args.out}; train report {report['train']}")
    return (params, tile_params), report


def _install(tc, params):
    tc.selector_set_params(params[0])
    tc.selector_set_tile_params(params[1])


def _evaluate(args, tc, selector, params, report):
    import torch
    _install(tc, params)   # predict() and the learned mode use the library's parameters
    report["heldout"] = []
    for name, edges, n in heldout_graphs(args.quick):
        log(f"[selector] held-out {name}")
        d = torch.from_numpy(edges).cuda()
        entry = {"graph": name}
        if not args.no_heldout_profile:
            data = selector.collect_in_launch([(name, edges, n)], repeats=args.repeats, log=log)
            times, busy = data["times"], data["bucket"]
            scales = np.ones(len(busy), dtype=int)
            if params[1] is not None:   # predict() runs the library's strategy network: load the tile one there
                tc.selector_set_params(params[1])
                scales = selector.predict(data["features"])
            tc.selector_set_params(params[0])
            kernels = selector.predict(data["features"])
            heur = np.array([selector.heuristic_choice(int(b)) for b in busy])
            one = np.ones(len(busy), dtype=int)
            entry.update({"buckets": int(len(busy)),
                          "stage_ms_heuristic": float(times[0, heur[0], 1]) if len(busy) else 0.0,
                          "noise_ms": float(data["noise_ms"][0]) if len(busy) else 0.0,
                          "regret_learned_ms": selector.in_launch_regret(times, kernels, scales),
                          "regret_learned_strategy_only_ms": selector.in_launch_regret(times, kernels, one),
                          "regret_heuristic_ms": selector.in_launch_regret(times, heur, one)})
            for k, kn in enumerate(selector.KERNELS):
                entry[f"regret_all_{kn}_ms"] = selector.in_launch_regret(times, np.full(len(busy), k), one)
            # the buckets where either choice misses the fastest (strategy, tile scale)
            flat = times.reshape(len(busy), 9)
            entry["misses"] = [{"bucket": int(b), "best": [int(flat[i].argmin() // 3), int(flat[i].argmin() % 3)],
                                "learned": [int(kernels[i]), int(scales[i])], "heuristic": int(heur[i]),
                                "gain_best_ms": round(float(times[i, heur[i], 1] - flat[i].min()), 4)}
                               for i, b in enumerate(busy)
                               if (kernels[i] * 3 + scales[i]) != flat[i].argmin() or heur[i] * 3 + 1 != flat[i].argmin()]
        _install(tc, params)
        t_l, t_h, ratios, T = step_times(tc, d, n)
        entry.update({"step_ms_learned": t_l, "step_ms_heuristic": t_h, "speedup": t_h / t_l,
                      "block_ratios": [float(x) for x in ratios], "triangles": T})
        report["heldout"].append(entry)
        log(f"[selector] {entry}")
        del d


if __name__ == "__main__":
    sys.exit(main())
