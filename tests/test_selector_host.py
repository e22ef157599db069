"""Host-side logic of the selector and the autotuner (no GPU)."""
import json

import numpy as np

from paper_1804_06926_amd import autotune, selector


def test_heuristic_thresholds():
    assert selector.heuristic_choice(16 * 6 + 0) == 2     # >= 64 in-edges: bitmap
    assert selector.heuristic_choice(16 * 4 + 6) == 2     # >= 16 in-edges and >= 64 out-neighbours: bitmap
    assert selector.heuristic_choice(16 * 4 + 5) == 1     # fewer, long lists: binary search
    assert selector.heuristic_choice(16 * 3 + 9) == 1
    assert selector.heuristic_choice(16 * 2 + 2) == 0     # short lists: merge path


def test_labels_keep_heuristic_within_tie():
    times = np.array([[1.00, 1.01, 2.0],     # heuristic (bucket 0 -> merge) within 2%: keep merge
                      [2.00, 1.00, 3.0],     # clearly faster binary search
                      [5.00, 4.00, 1.0]])
    buckets = np.array([0, 0, 0])
    y = selector.make_labels(times, buckets, tie=0.02)
    assert y.tolist() == [0, 1, 2]


def test_labels_keep_heuristic_within_absolute_tie():
    # small buckets, timed alone: 4 us apart is a tie (5 us tolerance), 6 us is not
    times = np.array([[0.019, 0.015, 0.12],
                      [0.025, 0.019, 0.13]])
    buckets = np.array([0, 0])   # the heuristic's choice: merge path
    y = selector.make_labels(times, buckets)
    assert y.tolist() == [0, 1]
    assert selector.make_labels(times, buckets, abs_tie=0.0).tolist() == [1, 1]


def test_sample_weights_and_regret():
    times = np.array([[1.0, 1.0, 1.0], [1.0, 5.0, 9.0]])
    w = selector.sample_weights(times)
    assert abs(w.mean() - 1.0) < 1e-6 and w[1] > w[0]
    assert selector.regret(times, np.array([0, 2])) == 8.0
    assert selector.regret(times, np.array([1, 0])) == 0.0


def test_init_params_shape_and_scale():
    p = selector.init_params(3)
    assert p.dtype == np.float32 and p.size == 1379
    W1 = p[:192]
    assert abs(W1.std() - np.sqrt(2 / 6)) < 0.1
    assert np.all(p[192:224] == 0)


def test_weights_roundtrip(tmp_path):
    p = selector.init_params(1)
    f = tmp_path / "w.json"
    selector.save(str(f), p, {"note": "x"})
    np.testing.assert_array_equal(selector.load(str(f)), p)
    doc = json.loads(f.read_text())
    assert doc["format"] == "tc-selector-v1"


def test_autotune_cache_roundtrip(tmp_path):
    f = tmp_path / "t.json"
    shapes = np.zeros(256, dtype=np.uint16)
    shapes[[3, 100, 254]] = [64, 256, 512]
    autotune.save(shapes, "gfx950|hipX|select0", str(f))
    autotune.save(shapes * 0 + 0, "other", str(f))
    got = autotune.load("gfx950|hipX|select0", str(f))
    np.testing.assert_array_equal(got, shapes)
    assert autotune.load("missing", str(f)) is None


def test_in_launch_labels_joint_strategy_and_tile_scale():
    # times[i, strategy, scale]: stage time with bucket i changed alone (inf: scale unavailable)
    inf = np.inf
    t = np.full((3, 3, 3), 10.0)
    # bucket 0 (heuristic: merge path): binary search at double tiles is 0.5 ms faster
    t[0, 1, 2] = 9.5
    # bucket 1: the better choice is within the baseline spread: keep the heuristic's
    t[1, 2, 0] = 9.995
    # bucket 2 (heuristic: bitmap, bucket 16*6): halving its tiles wins; doubling unavailable
    t[2, 2, 2] = inf
    t[2, 2, 0] = 9.0
    buckets = np.array([0, 0, 16 * 6])
    noise = np.array([0.01, 0.01, 0.01])
    k, s = selector.make_labels_in_launch(t, buckets, noise)
    assert k.tolist() == [1, 0, 2] and s.tolist() == [2, 1, 0]
    # regret: the chosen cell minus the bucket's best; an unavailable scale counts as the rule's size
    assert abs(selector.in_launch_regret(t, k, s) - 0.005) < 1e-12   # bucket 1's tie kept
    heur = np.array([0, 0, 2])
    assert abs(selector.in_launch_regret(t, heur, np.ones(3, int)) - (0.5 + 0.005 + 1.0)) < 1e-12
    assert abs(selector.in_launch_regret(t, np.array([2, 2, 2]), np.array([2, 2, 2])) - (0.5 + 0.005 + 1.0)) < 1e-12
    w = selector.sample_weights(t)
    assert np.all(np.isfinite(w)) and abs(w.mean() - 1.0) < 1e-6


def test_selector_file_holds_both_networks(tmp_path):
    p = np.arange(1379, dtype=np.float32) / 1379.0
    q = -p
    path = str(tmp_path / "w.json")
    selector.save(path, p, {"note": "test"}, tile_params=q)
    np.testing.assert_array_equal(selector.load(path), p)
    np.testing.assert_array_equal(selector.load_tile(path), q)
    selector.save(path, p)
    assert selector.load_tile(path) is None
    shipped = selector.load_tile(selector.DEFAULT_WEIGHTS)
    assert shipped is not None and shipped.size == 1379
