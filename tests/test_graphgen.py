"""Seeded input generators: determinism and the statistics each one promises."""
import math
import os
import subprocess
import sys

import numpy as np

import graphgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_deterministic_and_seed_sensitive():
    a = graphgen.rmat(12, 16, seed=3)
    b = graphgen.rmat(12, 16, seed=3)
    c = graphgen.rmat(12, 16, seed=4)
    np.testing.assert_array_equal(a, b)
    assert not np.array_equal(a, c)


def test_independent_of_thread_count():
    code = ("import sys; sys.path.insert(0, %r); import graphgen, hashlib; "
            "e = graphgen.rmat(14, 16, seed=5); r = graphgen.rgg(1 << 14, seed=2); "
            "print(hashlib.sha256(e.tobytes() + r.tobytes()).hexdigest())" % ROOT)
    out = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t)
        out.append(subprocess.check_output([sys.executable, "-c", code], env=env).strip())
    assert out[0] == out[1]


def test_rmat_quadrant_frequencies():
    scale = 10
    e = graphgen.rmat(scale, 64, seed=1, permute=False, flip=False).astype(np.int64)
    # top bit of each endpoint = the first quadrant choice
    ru, rv = e[:, 0] >> (scale - 1), e[:, 1] >> (scale - 1)
    freq = np.array([np.mean((ru == i) & (rv == j)) for i, j in ((0, 0), (0, 1), (1, 0), (1, 1))])
    np.testing.assert_allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.005)


def test_rmat_permutation_is_bijective():
    p = graphgen.permutation(1 << 16, 9)
    assert np.array_equal(np.sort(p), np.arange(1 << 16))


def test_erdos_renyi_distinct_pairs():
    e = graphgen.erdos_renyi(4096, 32768, seed=1804).astype(np.int64)
    assert e.shape == (32768, 2)
    assert np.all(e[:, 0] != e[:, 1])
    k = np.minimum(e[:, 0], e[:, 1]) * 4096 + np.maximum(e[:, 0], e[:, 1])
    assert np.unique(k).size == 32768


def test_rgg_pairs_within_radius_and_complete():
    n = 3000
    e = graphgen.rgg(n, avg_degree=12, seed=4, shuffle=False).astype(np.int64)
    d = graphgen.draws(4, 5, 2 * n)
    xy = ((d >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)).reshape(n, 2)
    r = math.sqrt(12 / (math.pi * n))
    dist2 = ((xy[e[:, 0]] - xy[e[:, 1]]) ** 2).sum(1)
    assert np.all(dist2 <= r * r)
    # brute force: all pairs within r
    diff = xy[:, None, :] - xy[None, :, :]
    close = np.triu((diff ** 2).sum(-1) <= r * r, 1)
    assert close.sum() == e.shape[0]


def test_chung_lu_batch_shapes():
    e, off, n = graphgen.chung_lu_batch(16, 1e3, 1e4, seed=3)
    assert off[0] == 0 and off[-1] == e.shape[0] and off.shape == (17,)
    for g in range(16):
        part = e[off[g]:off[g + 1]]
        assert part.min() >= 0 and part.max() < n[g]
    n2, E2 = graphgen.chung_lu_batch_sizes(4096)
    assert E2.min() >= 1000 and E2.max() <= 1_000_000
