"""Pins for the selector-network oracle (oracle/mlp.py): each function is checked
against an independent computation (torch on the CPU in float64, central
differences, known bfloat16 encodings)."""
import numpy as np
import pytest

from oracle import mlp

torch = pytest.importorskip("torch")


def _data(B=64, seed=0):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, size=(B, 6)).astype(np.float32)
    y = rng.integers(0, 3, size=B)
    w = rng.uniform(0.5, 2.0, size=B)
    return X, y, w


def test_bf16_round_known_values_and_torch():
    vals = np.array([1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 3.14159265, 1e-30, 6.5e4, 0.0],
                    dtype=np.float32)
    r = mlp.bf16_round(vals)
    # exact halves go to the even neighbour: 1 + 2^-8 -> 1.0, 1 + 3*2^-8 -> 1 + 2^-6
    assert r[0] == 1.0 and r[1] == 1.0 and r[2] == np.float32(1.0 + 2.0 ** -6)
    ref = torch.from_numpy(vals).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(r, ref)
    rng = np.random.default_rng(3)
    big = (rng.standard_normal(100000) * 10 ** rng.uniform(-8, 8, 100000)).astype(np.float32)
    np.testing.assert_array_equal(mlp.bf16_round(big), torch.from_numpy(big).to(torch.bfloat16).float().numpy())


def _torch_model(theta):
    p = mlp.unpack(theta)
    t = {k: torch.tensor(mlp.bf16_round(v).astype(np.float64) if k.startswith("W") else v.astype(np.float64),
                         requires_grad=True) for k, v in p.items()}
    return t


def test_forward_and_loss_match_torch_float64():
    theta = mlp.init_params(1)
    theta[mlp.N_PARAMS - 3:] = [0.1, -0.2, 0.05]
    X, y, w = _data()
    z, _, _ = mlp.forward(theta, X)
    t = _torch_model(theta)
    x = torch.tensor(X.astype(np.float64))
    h1 = torch.relu(x @ t["W1"].T + t["b1"])
    h2 = torch.relu(h1 @ t["W2"].T + t["b2"])
    zt = h2 @ t["W3"].T + t["b3"]
    np.testing.assert_allclose(z, zt.detach().numpy(), rtol=1e-12, atol=1e-12)
    ce = torch.nn.functional.cross_entropy(zt, torch.tensor(y), reduction="none")
    lt = (ce * torch.tensor(w)).sum() / len(y)
    lt.backward()
    loss, g = mlp.loss_and_grad(theta, X, y, w)
    assert abs(loss - lt.item()) < 1e-12
    gt = mlp.pack({k: v.grad.numpy() for k, v in t.items()})
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_gradient_matches_central_differences():
    theta = mlp.init_params(2)
    X, y, w = _data(16, 5)
    _, g = mlp.loss_and_grad(theta, X, y, w)
    p = mlp.unpack(theta.astype(np.float64))
    base = mlp.pack({k: (mlp.bf16_round(v).astype(np.float64) if k.startswith("W") else v) for k, v in p.items()})
    rng = np.random.default_rng(0)
    idx = rng.choice(mlp.N_PARAMS, 120, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(mlp.N_PARAMS)
        e[i] = h
        num = (mlp.loss_only(base + e, X, y, w) - mlp.loss_only(base - e, X, y, w)) / (2 * h)
        assert abs(num - g[i]) <= 1e-6 + 1e-4 * abs(g[i]), (i, num, g[i])


def test_adam_matches_torch():
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    tp = torch.tensor(theta.copy(), requires_grad=True)
    opt = torch.optim.Adam([tp], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.standard_normal(50)
        theta, m, v = mlp.adam_step(theta, g, m, v, t, lr=1e-2)
        opt.zero_grad()
        tp.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, tp.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_error_bound_covers_float32_evaluation():
    theta = mlp.init_params(7)
    X, _, _ = _data(256, 9)
    z64, _, _ = mlp.forward(theta, X)
    p = mlp.unpack(theta)
    f = np.float32
    W = {k: mlp.bf16_round(v) if k.startswith("W") else v.astype(f) for k, v in p.items()}
    h1 = np.maximum(X @ W["W1"].T + W["b1"], f(0))
    h2 = np.maximum(h1 @ W["W2"].T + W["b2"], f(0))
    z32 = h2 @ W["W3"].T + W["b3"]
    bound = mlp.forward_error_bound(theta, X)
    assert np.all(np.abs(z32 - z64) <= bound)
