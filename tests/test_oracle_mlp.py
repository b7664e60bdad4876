"""Pins of the seed-proposer oracle (oracle/mlp_oracle.py) against library
routines, closed forms, brute force and finite differences -- no GPU."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import mlp_oracle as MO


def _layers(rng, dims):
    return [(rng.uniform(-1, 1, (o, i)) / math.sqrt(i), rng.uniform(-0.1, 0.1, o)) for i, o in dims]


def test_bf16_round_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-6, 6, 20000),
                        [1 + 2 ** -8, 1 + 3 * 2 ** -8, -(1 + 2 ** -8), 0.0, -0.0, 65504.0]])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    got = MO.bf16_round(x32)
    np.testing.assert_array_equal(got, ref)
    # halfway cases: 1 + 2^-8 lies midway between 1 and 1 + 2^-7 -> even (1);
    # 1 + 3*2^-8 lies midway between 1 + 2^-7 and 1 + 2^-6 -> even (1 + 2^-6)
    assert MO.bf16_round(1 + 2 ** -8) == 1.0
    assert MO.bf16_round(1 + 3 * 2 ** -8) == 1 + 2 ** -6
    # relative error bound of an 8-bit significand (unit roundoff 2^-8), idempotence
    nz = np.abs(x32) > 1e-30
    assert np.all(np.abs(got[nz] - x32[nz]) <= 2.0 ** -8 * np.abs(x32[nz]) * (1 + 1e-12))
    np.testing.assert_array_equal(MO.bf16_round(got), got)


def test_gelu_and_its_derivative_match_torch():
    x = torch.linspace(-8, 8, 4001, dtype=torch.float64, requires_grad=True)
    y = torch.nn.functional.gelu(x, approximate="none")
    (g,) = torch.autograd.grad(y.sum(), x)
    xn = x.detach().numpy()
    np.testing.assert_allclose(MO.gelu(xn), y.detach().numpy(), rtol=0, atol=1e-15)
    np.testing.assert_allclose(MO.gelu_grad(xn), g.numpy(), rtol=0, atol=1e-14)
    # x Phi(x) - (-x) Phi(-x) = x Phi(x) + x (1 - Phi(x)) = x
    np.testing.assert_allclose(MO.gelu(xn) - MO.gelu(-xn), xn, atol=1e-14)


def test_forward_float64_matches_torch_sequential():
    rng = np.random.default_rng(1)
    dims = MO.layer_dims(12, 16, 3, 5)
    layers = _layers(rng, dims)
    X = rng.standard_normal((33, 12))
    Y, _ = MO.forward(layers, X, bf16=False)
    mods = []
    for li, (W, b) in enumerate(layers):
        lin = torch.nn.Linear(W.shape[1], W.shape[0]).double()
        with torch.no_grad():
            lin.weight.copy_(torch.from_numpy(W))
            lin.bias.copy_(torch.from_numpy(b))
        mods.append(lin)
        if li + 1 < len(layers):
            mods.append(torch.nn.GELU())
    ref = torch.nn.Sequential(*mods)(torch.from_numpy(X)).detach().numpy()
    np.testing.assert_allclose(Y, ref, rtol=1e-13, atol=1e-13)


def test_forward_bf16_rounding_points():
    """With BF16 on, each layer equals float64 torch products of operands that
    torch itself rounded to bfloat16."""
    rng = np.random.default_rng(2)
    dims = MO.layer_dims(8, 16, 2, 4)
    layers = _layers(rng, dims)
    X = rng.standard_normal((9, 8))
    Y, (hs, zs) = MO.forward(layers, X, bf16=True)

    def tb(a):
        return torch.from_numpy(np.asarray(a, np.float32)).to(torch.bfloat16).double()

    h = tb(X)
    for li, (W, b) in enumerate(layers):
        z = h @ tb(W).T + torch.from_numpy(b)
        if li + 1 < len(layers):
            np.testing.assert_allclose(zs[li], z.numpy(), rtol=1e-12, atol=1e-12)
            h = tb(torch.nn.functional.gelu(z).numpy())
            np.testing.assert_array_equal(hs[li + 1], h.numpy())
        else:
            np.testing.assert_allclose(Y, z.numpy(), rtol=1e-12, atol=1e-12)


def test_backward_float64_matches_autograd_and_differences():
    rng = np.random.default_rng(3)
    dims = MO.layer_dims(6, 10, 3, 4)
    layers = _layers(rng, dims)
    p = MO.flatten(layers)
    X = rng.standard_normal((7, 6))
    dY = rng.standard_normal((7, 4))
    Y, cache = MO.forward(layers, X, bf16=False)
    g = MO.backward(layers, cache, dY, bf16=False)

    pt = torch.from_numpy(p.copy()).requires_grad_(True)
    off, h = 0, torch.from_numpy(X)
    for li, (i, o) in enumerate(dims):
        W = pt[off:off + i * o].reshape(o, i)
        off += i * o
        b = pt[off:off + o]
        off += o
        h = h @ W.T + b
        if li + 1 < len(dims):
            h = torch.nn.functional.gelu(h)
    (gt,) = torch.autograd.grad((h * torch.from_numpy(dY)).sum(), pt)
    np.testing.assert_allclose(g, gt.numpy(), rtol=1e-11, atol=1e-12)

    def f(pp):
        yy, _ = MO.forward(MO.unflatten(pp, dims), X, bf16=False)
        return float((yy * dY).sum())

    for j in rng.choice(p.size, 25, replace=False):
        e = np.zeros_like(p)
        e[j] = 1e-6
        fd = (f(p + e) - f(p - e)) / 2e-6
        assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])), (j, fd, g[j])


def test_backward_bf16_within_rounding_bound_of_exact_gradient():
    rng = np.random.default_rng(4)
    dims = MO.layer_dims(24, 64, 3, 12)
    layers = [(MO.bf16_round(W), b) for W, b in _layers(rng, dims)]
    X = MO.bf16_round(rng.standard_normal((64, 24)))
    dY = rng.standard_normal((64, 12))
    _, c64 = MO.forward(layers, X, bf16=False)
    g64 = MO.backward(layers, c64, dY, bf16=False)
    _, c16 = MO.forward(layers, X, bf16=True)
    g16 = MO.backward(layers, c16, dY, bf16=True)
    rel = np.linalg.norm(g16 - g64) / np.linalg.norm(g64)
    # a few BF16 roundings (unit roundoff 2^-8) on the way: well under 2 %
    assert 1e-5 < rel < 2e-2, rel


def test_imle_select_brute_force_and_ties():
    rng = np.random.default_rng(5)
    Y = rng.standard_normal((6, 5, 3))
    T = rng.standard_normal((6, 3))
    got = MO.imle_select(Y, T)
    for b in range(6):
        best, bi = None, None
        for s in range(5):
            d = sum((Y[b, s, k] - T[b, k]) ** 2 for k in range(3))
            if best is None or d < best:
                best, bi = d, s
        assert got[b] == bi
    Y2 = np.zeros((1, 4, 2))
    Y2[0, 1] = Y2[0, 3] = [1.0, 0.0]
    Y2[0, 0] = Y2[0, 2] = [3.0, 0.0]
    assert MO.imle_select(Y2, np.array([[1.0, 0.0]]))[0] == 1
    # weights: only the second coordinate counts
    Y3 = np.array([[[0.0, 5.0], [9.0, 1.0]]])
    assert MO.imle_select(Y3, np.array([[0.0, 0.0]]))[0] == 0
    assert MO.imle_select(Y3, np.array([[0.0, 0.0]]), np.array([[0.0, 1.0]]))[0] == 1
    W = rng.integers(0, 2, (6, 3)).astype(float)
    got = MO.imle_select(Y, T, W)
    for b in range(6):
        d = [sum(W[b, k] * (Y[b, s, k] - T[b, k]) ** 2 for k in range(3)) for s in range(5)]
        assert got[b] == int(np.argmin(d))


def test_weighted_mse_brute_force():
    rng = np.random.default_rng(8)
    Y, T = rng.standard_normal((2, 4, 3))
    W = rng.integers(0, 2, (4, 3)).astype(float)
    loss, g = MO.mse(Y, T, W)
    assert loss == pytest.approx(sum(W[i, j] * (Y[i, j] - T[i, j]) ** 2 for i in range(4) for j in range(3)) / 12)
    for i in range(4):
        for j in range(3):
            e = np.zeros_like(Y)
            e[i, j] = 1e-6
            fd = (MO.mse(Y + e, T, W)[0] - MO.mse(Y - e, T, W)[0]) / 2e-6
            assert abs(fd - g[i, j]) < 1e-8
    assert MO.mse(Y, T)[0] == pytest.approx(((Y - T) ** 2).mean())


def test_normal_noise_is_standard_normal_and_counter_based():
    rows = 8192
    z = MO.normal_noise(7, np.arange(rows), np.zeros(rows), 32)
    assert z.shape == (rows, 32)
    flat = z.reshape(-1)
    assert stats.kstest(flat, "norm").pvalue > 1e-3
    assert abs(flat.mean()) < 0.01 and abs(flat.var() - 1) < 0.01
    # the cos and sin halves of one Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(z[:, 0], z[:, 1])[0, 1]) < 0.05
    # each row depends only on its own counter words
    z2 = MO.normal_noise(7, np.array([5, 3]), np.array([0, 0]), 32)
    np.testing.assert_array_equal(z2, z[[5, 3]])
    # other draws and other seeds give other numbers
    assert not np.allclose(MO.normal_noise(7, [5], [1], 32), z[5])
    assert not np.allclose(MO.normal_noise(8, [5], [0], 32), z[5])


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(6)
    p, g1, g2 = rng.standard_normal((3, 50))
    pt = torch.from_numpy(p.copy()).requires_grad_(True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    m = v = np.zeros(50)
    q = p.copy()
    for t, g in enumerate((g1, g2), 1):
        pt.grad = torch.from_numpy(g.copy())
        opt.step()
        q, m, v = MO.adam(q, m, v, g, t, 1e-3)
    np.testing.assert_allclose(q, pt.detach().numpy(), rtol=0, atol=1e-15)


def test_imle_step_lowers_the_loss():
    rng = np.random.default_rng(7)
    dims = MO.layer_dims(4 + 8, 32, 2, 3)
    p = MO.flatten(_layers(rng, dims))
    feats = rng.standard_normal((2, 4))
    fr = rng.integers(0, 2, 64)
    T = rng.standard_normal((64, 3)) * 0.5 + feats[fr, :3]
    m = v = np.zeros_like(p)
    losses = []
    for t in range(1, 61):
        p, m, v, loss, chosen, _ = MO.imle_step(p, m, v, t, dims, feats, fr, T, 4, 100 + t, 8, 3e-3)
        losses.append(loss)
        assert chosen.min() >= 0 and chosen.max() < 4
    assert np.mean(losses[-10:]) < 0.7 * np.mean(losses[:5])


def test_destandardize_wraps_and_clamps():
    Y = np.array([[0.0, 10.0, -10.0, 0.5]])
    mean = np.array([0.1, 0.0, 0.0, 3.0])
    std = np.array([1.0, 1.0, 1.0, 1.0])
    lo = np.array([-1.0, -2.0, -math.pi, -math.pi])
    hi = np.array([1.0, 2.0, math.pi, math.pi])
    wrap = np.array([0, 0, 1, 1])
    x = MO.destandardize(Y, mean, std, lo, hi, wrap)
    assert x[0, 0] == pytest.approx(0.1)
    assert x[0, 1] == 2.0                      # clamped
    assert x[0, 2] == pytest.approx(-10.0 + 4 * math.pi)   # wrapped, not clamped
    assert x[0, 3] == pytest.approx(3.5 - 2 * math.pi)
    assert np.all((x >= lo) & (x <= hi))
