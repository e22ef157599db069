"""GPU parity of the selector network's kernels against the float64 oracle, and
the learned selection mode's exactness. Inputs are seeded synthetic features."""
import os

import numpy as np
import pytest

import graphgen
import oracle
from oracle import mlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tc():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_1804_06926_amd import _lib
    if not os.path.exists(_lib.library_path()):
        import __graft_entry__
        __graft_entry__.build()
    import paper_1804_06926_amd
    return paper_1804_06926_amd


def _batch(B, seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, size=(B, 6)).astype(np.float32)
    y = rng.integers(0, 3, size=B).astype(np.int32)
    w = rng.uniform(0.2, 3.0, size=B).astype(np.float32)
    return X, y, w


def _params(seed):
    theta = mlp.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    theta[mlp.N_PARAMS - 3:] = rng.normal(0, 0.3, 3)
    theta[192:224] = rng.normal(0, 0.1, 32)     # b1
    theta[1248:1280] = rng.normal(0, 0.1, 32)   # b2
    return theta.astype(np.float32)


@pytest.mark.parametrize("B", [1, 255, 256, 1000])
def test_forward_matches_oracle_within_error_bound(tc, B):
    import torch
    theta = _params(B)
    X, _, _ = _batch(B, B)
    tc.selector_set_params(theta)
    z = tc.selector_forward(torch.from_numpy(X).cuda()).cpu().numpy().astype(np.float64)
    z64, _, _ = mlp.forward(theta, X)
    bound = mlp.forward_error_bound(theta, X)
    assert np.all(np.abs(z - z64) <= bound), np.max(np.abs(z - z64) - bound)
    np.testing.assert_array_equal(tc.selector_get_params(), theta)


@pytest.mark.parametrize("B,weighted", [(1, False), (300, True), (4096, True)])
def test_gradient_matches_oracle(tc, B, weighted):
    """Tolerance: each gradient entry is a sum of B products formed from float32
    activations; float32 rounding of the layer outputs and of the sum bounds the
    error by about (B + 70) * 2^-24 times the sum of absolute terms. That sum is
    at most B * max|term| <= B times the largest gradient entry here, so the
    slack 1e-4 * (|g| + max|g|) + 1e-7 covers B up to about 4096 with margin."""
    import torch
    theta = _params(7 + B)
    X, y, w = _batch(B, 11 + B)
    tc.selector_set_params(theta)
    g, loss = tc.selector_gradient(torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(),
                                   torch.from_numpy(w).cuda() if weighted else None)
    g = g.cpu().numpy().astype(np.float64)
    loss64, g64 = mlp.loss_and_grad(theta, X, y, w if weighted else None)
    assert abs(loss - loss64) <= 1e-5 * max(1.0, abs(loss64))
    tol = 1e-4 * np.abs(g64) + 1e-4 * np.max(np.abs(g64)) + 1e-7
    assert np.all(np.abs(g - g64) <= tol), np.max(np.abs(g - g64) - tol)


def test_training_steps_match_oracle_adam_and_lower_the_loss(tc):
    import torch
    theta = _params(3)
    X, y, w = _batch(512, 5)
    tc.selector_set_params(theta)
    dx, dy, dw = torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda(), torch.from_numpy(w).cuda()
    th = theta.astype(np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    losses = []
    for t in range(1, 6):
        losses.append(tc.selector_train_step(dx, dy, dw, lr=1e-2))
        _, g = mlp.loss_and_grad(th.astype(np.float32), X, y, w)
        th, m, v = mlp.adam_step(th, g, m, v, t, lr=1e-2)
    got = tc.selector_get_params().astype(np.float64)
    # Adam moves each parameter by at most about lr per step; float32 gradients may
    # flip the sign of tiny components, so compare with a step-sized tolerance
    assert np.max(np.abs(got - th)) < 5 * 1e-2
    assert np.mean(np.abs(got - th)) < 1e-3
    for _ in range(200):
        last = tc.selector_train_step(dx, dy, dw, lr=1e-2)
    assert last < losses[0] * 0.9


def test_learned_selection_gives_exact_counts(tc):
    import torch
    rng = np.random.default_rng(0)
    theta = mlp.init_params(5)
    tc.selector_set_params(theta)
    for scale, seed in ((12, 1), (15, 2)):
        n = 1 << scale
        e = graphgen.rmat(scale, 16, seed=seed)
        ref = oracle.count_triangles(e, n)
        d = torch.from_numpy(e).cuda()
        assert tc.count_triangles(d, n, select=tc.SELECT_LEARNED) == ref
        # bucket features are those of the graph, computed on the device
        feat = tc.bucket_features()
        assert feat.shape == (256, 6) and np.all(np.isfinite(feat))
    _ = rng


def test_profile_buckets_shapes(tc):
    import torch
    n = 1 << 14
    e = graphgen.rmat(14, 16, seed=3)
    ms, feat = tc.profile_buckets(torch.from_numpy(e).cuda(), n, repeats=3)
    st = tc.last_stats()
    busy = np.nonzero(st["bucket_vertices"][:255])[0]
    assert busy.size > 0
    for b in busy:
        assert np.all(ms[:, b] > 0), b
    assert np.all(ms[:, 255] < 0)


def test_device_heuristic_matches_host_rule(tc):
    import torch
    from paper_1804_06926_amd import selector
    n = 1 << 16
    e = graphgen.rmat(16, 16, seed=4)
    tc.count_triangles(torch.from_numpy(e).cuda(), n, select=tc.SELECT_HEURISTIC)
    st = tc.last_stats()
    for b in range(255):
        assert st["bucket_kernel"][b] == selector.heuristic_choice(b), b


def test_trained_selector_gains_over_heuristic(tc):
    """Held-out graphs (R-MAT scale 22 seed 77, and a random geometric graph of 2^20
    vertices; neither in the training set): every (strategy, tile size) alternative of
    every busy bucket is timed inside the combined launch, and the time the learned
    choice leaves on the table (its regret against the per-bucket best) must be below
    the fixed thresholds' by more than the spread of repeated baseline timings, summed
    over the graphs; counts are identical in both modes."""
    import torch
    from paper_1804_06926_amd import selector
    if not os.path.exists(selector.DEFAULT_WEIGHTS):
        pytest.skip("no trained selector weights in the package yet")
    params, tile = selector.load(selector.DEFAULT_WEIGHTS), selector.load_tile(selector.DEFAULT_WEIGHTS)
    r_l = r_h = noise = 0.0
    for name, e, n in (("rmat22", graphgen.rmat(22, 16, seed=77), 1 << 22),
                       ("rgg20", graphgen.rgg(1 << 20, 32.0, seed=78), 1 << 20)):
        data = selector.collect_in_launch([(name, e, n)], repeats=5)
        busy = data["bucket"]
        scales = np.ones(len(busy), dtype=int)
        if tile is not None:   # predict() runs the library's strategy network: load the tile one there
            tc.selector_set_params(tile)
            scales = selector.predict(data["features"])
        tc.selector_set_params(params)
        kernels = selector.predict(data["features"])
        heur = np.array([selector.heuristic_choice(int(b)) for b in busy])
        gl = selector.in_launch_regret(data["times"], kernels, scales)
        gh = selector.in_launch_regret(data["times"], heur, np.ones_like(heur))
        print(f"{name}: in-launch regret learned {gl:.3f} ms, heuristic {gh:.3f} ms, "
              f"baseline spread {data['noise_ms'][0]:.3f} ms")
        r_l, r_h, noise = r_l + gl, r_h + gh, noise + float(data["noise_ms"][0])
        selector.load_default()
        d = torch.from_numpy(e).cuda()
        assert tc.count_triangles(d, n, select=tc.SELECT_LEARNED) == tc.count_triangles(d, n)
    assert r_l + noise < r_h, (r_l, r_h, noise)


def test_window_feature_matches_host_count(tc):
    """Feature 2 is log2(1 + the LDS-bitmap windows the bucket's middle lists span) / 32,
    recomputed here from the exported degree-ordered CSR."""
    import torch
    n = 1 << 19   # ranks span four 2^17-id windows
    e = graphgen.rmat(19, 16, seed=9)
    d = torch.from_numpy(e).cuda()
    tc.count_triangles(d, n, select=tc.SELECT_HEURISTIC)
    feat = tc.bucket_features()
    _, off, col = tc.build_csr(d, n)
    off = off.cpu().numpy().astype(np.int64)
    col = col.cpu().numpy().astype(np.int64)
    dplus = np.diff(off)
    src = np.repeat(np.arange(n), dplus)
    tail = off[src + 1] - np.arange(col.size) - 1
    din = np.bincount(col[tail > 0], minlength=n)
    v = np.nonzero((din > 0) & (dplus > 0))[0]
    b = 16 * np.minimum(14, np.floor(np.log2(din[v]))).astype(np.int64) + \
        np.minimum(15, np.floor(np.log2(dplus[v]))).astype(np.int64)
    lo, hi = col[off[v]], col[off[v + 1] - 1]
    win = ((hi - (lo & ~31)) >> 17) + 1
    assert win.max() > 1
    tot = np.bincount(b, weights=win, minlength=256)
    busy = np.nonzero(np.bincount(b, minlength=256))[0]
    np.testing.assert_allclose(feat[busy, 2], np.log2(1.0 + tot[busy]).astype(np.float32) / 32.0, rtol=1e-5)


def test_learned_choices_match_forward_argmax(tc):
    """The selection kernel (eight lanes per bucket) picks, for every bucket, the argmax of
    the logits the plain forward kernel gives for the same features (same arithmetic order)."""
    import torch
    from paper_1804_06926_amd import selector
    for seed in (5, 11):
        tc.selector_set_params(mlp.init_params(seed))
        n = 1 << 16
        e = graphgen.rmat(16, 16, seed=seed)
        tc.count_triangles(torch.from_numpy(e).cuda(), n, select=tc.SELECT_LEARNED)
        st = tc.last_stats()
        feat = tc.bucket_features()
        want = selector.predict(feat[:255])
        np.testing.assert_array_equal(st["bucket_kernel"][:255], want)
    # the shipped network as well
    assert selector.load_default()
    tc.count_triangles(torch.from_numpy(graphgen.rmat(16, 16, seed=4)).cuda(), 1 << 16, select=tc.SELECT_LEARNED)
    st = tc.last_stats()
    np.testing.assert_array_equal(st["bucket_kernel"][:255], selector.predict(tc.bucket_features()[:255]))


def test_profile_choices_applies_the_given_strategies(tc):
    """tc_profile_choices lays out the tiles with the caller's strategy per bucket
    (values 3..255 keep the fixed thresholds' choice), times the whole intersection
    stage, and counts the same T whatever the choice."""
    import torch
    from paper_1804_06926_amd import selector
    n = 1 << 15
    e = graphgen.rmat(15, 16, seed=21)
    d = torch.from_numpy(e).cuda()
    T = oracle.count_triangles(e, n)
    ms, per, Tx = tc.profile_choices(d, n, np.full(256, 255, np.uint8), repeats=3)
    # medians of the stage and of each kernel over the repeats: close, not equal
    assert Tx == T and ms > 0 and np.all(per >= 0) and abs(per.sum() - ms) <= 0.25 * ms
    st = tc.last_stats()
    busy = np.nonzero(st["bucket_vertices"][:255])[0]
    for b in range(255):
        assert st["bucket_kernel"][b] == selector.heuristic_choice(b)
    rng = np.random.default_rng(5)
    for trial in range(3):
        choice = np.full(256, 255, np.uint8)
        choice[busy] = rng.integers(0, 3, size=busy.size)
        chunk = np.zeros(256, np.uint16)
        chunk[busy] = rng.choice([64, 128, 512], size=busy.size)
        ms, per, Tx = tc.profile_choices(d, n, choice, chunk, repeats=2)
        assert Tx == T, trial
        st = tc.last_stats()
        np.testing.assert_array_equal(st["bucket_kernel"][busy], choice[busy])
        np.testing.assert_array_equal(st["bucket_chunk"][busy], chunk[busy])
    # the context's own selection is untouched afterwards
    assert tc.count_triangles(d, n) == T
    st = tc.last_stats()
    for b in range(255):
        assert st["bucket_kernel"][b] == selector.heuristic_choice(b)


def test_selector_file_load_and_save(tc, tmp_path):
    """tc_selector_load reads the shipped parameter file into exactly the float32 parameters the
    Python reader gives, for both networks; tc_selector_save writes a file that reads back the
    same; a file with the wrong number of parameters is rejected."""
    from paper_1804_06926_amd import selector
    path = selector.DEFAULT_WEIGHTS
    tc.selector_load(path)
    np.testing.assert_array_equal(tc.selector_get_params(), selector.load(path))
    np.testing.assert_array_equal(tc.selector_get_tile_params(), selector.load_tile(path))
    out = tmp_path / "saved.json"
    tc.selector_save(str(out))
    np.testing.assert_array_equal(selector.load(str(out)), selector.load(path))
    np.testing.assert_array_equal(selector.load_tile(str(out)), selector.load_tile(path))
    bad = tmp_path / "bad.json"
    bad.write_text('{"format": "tc-selector-v1", "num_params": 1379, "params": [1.0, 2.0]}')
    with pytest.raises(tc.TCError):
        tc.selector_load(str(bad))
    with pytest.raises(tc.TCError):
        tc.selector_load(str(tmp_path / "missing.json"))
    tc.selector_load(path)   # leave the shipped networks installed
