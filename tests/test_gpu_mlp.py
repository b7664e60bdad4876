"""GPU parity of the seed proposer's matrix-core kernels with the FP64 oracle
(oracle/mlp_oracle.py, BF16 rounding emulated at the same points), through
the C ABI.

Tolerances (no published bound exists for this network; derived from the
number format): the GPU accumulates in FP32 where the oracle sums in FP64, and
a BF16 rounding whose FP32 input sits within an FP32 ulp of a rounding tie may
go the other way (one BF16 ulp, 2^-8 relative, on that element).  Hence
norm-wise relative errors: outputs <= 2e-3, weight gradients <= 5e-3 per layer,
and element-wise within one BF16 ulp (2^-8) of the element's own magnitude
plus one BF16 ulp of the tensor's RMS (a flipped rounding of an input moves
an element by about one ulp of the typical magnitude, not of that element,
which cancellation can make arbitrarily small).  For the outputs of the
forward pass that band is a typical bound, not a worst case: a flip of one
activation h of the last hidden layer moves every output y_n of its row by
w_n h 2^-8 to 2^-7, the largest weight-activation products of a 512-wide
layer reach about the RMS of the row's outputs, and a row can hold several
flips (FP32 accumulation of the same network with the exact GELU leaves the
band on the 4100-row case).  So at most 1e-4 of the outputs may leave the
one-ulp band, and none may exceed four times it;
noise (FP32 log / sin / cos vs FP64) <= 2e-5 absolute; nearest-draw choices
identical wherever the oracle's best and second-best distances differ by more
than 1e-3 relative.
"""
import math

import numpy as np
import pytest

from oracle import mlp_oracle as MO
from paper_2411_11833_amd import inputs as I

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = {
    # d_feat, d_noise, hidden, depth, d_out
    "small": (8, 8, 64, 2, 5),
    "proposer": (120, 32, 512, 3, 84),
    "narrow": (64, 32, 512, 1, 21),
    "deep": (8, 8, 512, 8, 7),
}


def _mlp(shape, max_rows=4096):
    from paper_2411_11833_amd.seeds import GpuMlp
    d_feat, d_noise, hidden, depth, d_out = shape
    return GpuMlp(d_feat, d_noise, hidden, depth, d_out, max_rows)


def _dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda().contiguous()


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


ULP_BF16 = 2.0 ** -8


def _elementwise(got, want, axis=None):
    """Largest |got - want| / (ulp |want| + ulp rms(want)), rms over `axis`
    (None: the whole tensor); <= 1 passes."""
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    rms = np.sqrt(np.mean(want * want, axis=axis, keepdims=axis is not None))
    return float(np.max(np.abs(got - want) / (ULP_BF16 * (np.abs(want) + rms) + 1e-30)))


def _setup(name, rows, seed=0, noise_gain=1.0, draws=1):
    shape = SHAPES[name]
    d_feat, d_noise, hidden, depth, d_out = shape
    m = _mlp(shape, max_rows=max(4096, ((rows * draws + 63) // 64) * 64))
    dims = MO.layer_dims(d_feat + d_noise, hidden, depth, d_out)
    p = I.mlp_init(dims, seed)
    i, o = dims[0]
    p[:i * o].reshape(o, i)[:, d_feat:] *= noise_gain   # first-layer weights of the noise inputs
    m.set_params(_dev(p))
    rng = np.random.default_rng(seed)
    feats = rng.standard_normal((5, d_feat)).astype(np.float32)
    fr = rng.integers(0, 5, rows).astype(np.int32)
    draw = rng.integers(0, 8, rows).astype(np.int32)
    return m, dims, p.astype(np.float64), feats, fr, draw


def test_noise_matches_oracle():
    m = _mlp(SHAPES["proposer"])
    rows = 1000
    draw = np.arange(rows, dtype=np.int32) % 7
    z = m.noise(123456789012, rows, _dev(draw, torch.int32)).cpu().numpy()
    want = MO.normal_noise(123456789012, np.arange(rows), draw, 32)
    assert np.max(np.abs(z - want)) <= 2e-5
    m.close()


# keep=True runs the training forward, layer by layer (Z, H and H^T kept):
# 16384 and more rows take the 256 x 256 hidden and 128 x 128 output tiles
# of the pipelined kernel, fewer rows its 32 x 32 tiles of four waves.
# keep=False runs inference: from 8192 rows width-512 networks run in one
# launch for all layers, in 32-row blocks below 16384 rows, 64-row blocks
# up to 32767, 128-row blocks from there (narrow: one hidden layer, 21
# outputs; deep: the most hidden layers, 7 outputs); fewer rows and the
# width-64 network run layer by layer with the inference epilogues.  200,
# 4100, 5000, 8200, 16400, 32800 and 33000 rows leave ragged last tiles.
@pytest.mark.parametrize("keep", [True, False])
@pytest.mark.parametrize("name,rows", [("small", 100), ("small", 64), ("proposer", 4096), ("proposer", 200),
                                       ("proposer", 4100), ("small", 5000), ("proposer", 16400),
                                       ("small", 16384), ("proposer", 8200), ("proposer", 32800),
                                       ("narrow", 300), ("narrow", 33000), ("deep", 8200)])
def test_forward_matches_oracle(name, rows, keep):
    m, dims, p, feats, fr, draw = _setup(name, rows)
    Y = m.forward(_dev(feats), rows, 77, _dev(fr, torch.int32), _dev(draw, torch.int32), keep=keep).cpu().numpy()
    X = MO.input_rows(feats, fr, 77, np.arange(rows), draw, m.d_noise)
    want, _ = MO.forward(MO.unflatten(p, dims), X, bf16=True)
    err = _rel(Y, want)
    ew = _elementwise(Y, want, axis=1)
    rms = np.sqrt(np.mean(want * want, axis=1, keepdims=True))
    outside = float(np.mean(np.abs(Y - want) > ULP_BF16 * (np.abs(want) + rms)))
    print(f"{name} rows={rows} keep={keep}: forward rel err {err:.2e}, element-wise {ew:.3f} of the one-ulp "
          f"band ({outside:.1e} of outputs outside it)")
    assert err <= 2e-3
    assert outside <= 1e-4
    assert ew <= 4.0
    # and well away from the unrounded network, so the rounding points are real
    plain, _ = MO.forward(MO.unflatten(p, dims), X, bf16=False)
    assert _rel(want, plain) > 1e-4
    m.close()


@pytest.mark.parametrize("name,rows", [("small", 128), ("proposer", 4096), ("proposer", 4160)])
def test_backward_matches_oracle(name, rows):
    m, dims, p, feats, fr, draw = _setup(name, rows, seed=1)
    rng = np.random.default_rng(11)
    dY = rng.standard_normal((rows, m.d_out)).astype(np.float32)
    m.forward(_dev(feats), rows, 5, _dev(fr, torch.int32), _dev(draw, torch.int32))
    m.backward(_dev(dY), rows)
    g = m.grads().cpu().numpy().astype(np.float64)
    X = MO.input_rows(feats, fr, 5, np.arange(rows), draw, m.d_noise)
    layers = MO.unflatten(p, dims)
    _, cache = MO.forward(layers, X, bf16=True)
    want = MO.backward(layers, cache, dY.astype(np.float64), bf16=True)
    off = 0
    for li, (i, o) in enumerate(dims):
        for part, cnt in (("W", i * o), ("b", o)):
            e = _rel(g[off:off + cnt], want[off:off + cnt])
            ew = _elementwise(g[off:off + cnt], want[off:off + cnt])
            print(f"{name} layer {li} {part}: rel err {e:.2e}, element-wise {ew:.3f} of the one-ulp bound")
            assert e <= 5e-3, (li, part, e)
            assert ew <= 1.0, (li, part, ew)
            off += cnt
    m.close()


def test_backward_rejects_rows_other_than_forward():
    from paper_2411_11833_amd.binding import CtError
    m, dims, p, feats, fr, draw = _setup("small", 128)
    m.forward(_dev(feats), 128, 5, _dev(fr, torch.int32), _dev(draw, torch.int32))
    with pytest.raises(CtError):
        m.backward(torch.zeros(64, m.d_out, device="cuda"), 64)
    m.close()


# the proposer's selection forward: 2,048 draws layer by layer, the
# training step's 1,024 targets x 32 draws in the one-launch inference
# kernel (128-row blocks)
@pytest.mark.parametrize("weighted", [False, True])
@pytest.mark.parametrize("name,rows,S", [("small", 128, 4), ("proposer", 256, 8), ("proposer", 1024, 32)])
def test_imle_step_matches_oracle(weighted, name, rows, S):
    # at the default initialization the wide network's draws differ too
    # little for most nearest-draw choices to be clear; larger noise weights
    # spread them
    m, dims, p, feats, fr, _ = _setup(name, rows, seed=2, noise_gain=16.0 if name == "proposer" else 1.0,
                                       draws=S)
    rng = np.random.default_rng(12)
    T = rng.standard_normal((rows, m.d_out)).astype(np.float32)
    W = rng.integers(0, 2, (rows, m.d_out)).astype(np.float32) if weighted else None
    chosen = torch.zeros(rows, dtype=torch.int32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    m.imle_step(_dev(feats), _dev(fr, torch.int32), _dev(T), S, 99, lr=1e-3, chosen=chosen, loss=loss,
                weights=None if W is None else _dev(W))
    p1 = m.params().cpu().numpy().astype(np.float64)
    g = m.grads().cpu().numpy().astype(np.float64)
    zero = np.zeros_like(p)
    w1, _, _, wl, wc, wg = MO.imle_step(p, zero, zero, 1, dims, feats, fr, T, S, 99, m.d_noise, 1e-3, weights=W)
    # choices: identical wherever the choice is clear
    bb = np.repeat(np.arange(rows), S)
    ss = np.tile(np.arange(S), rows)
    Yall, _ = MO.forward(MO.unflatten(p, dims), MO.input_rows(feats, fr[bb], 99, bb, ss, m.d_noise))
    Wb = 1.0 if W is None else W[:, None, :]
    d2 = np.sort((Wb * (Yall.reshape(rows, S, -1) - T[:, None, :]) ** 2).sum(-1), axis=1)
    clear = (d2[:, 1] - d2[:, 0]) > 1e-3 * d2[:, 1]
    got_c = chosen.cpu().numpy()
    assert clear.mean() > 0.9
    np.testing.assert_array_equal(got_c[clear], wc[clear])
    # where two draws are equally near within rounding either is a valid
    # choice: every choice must be a nearest draw to that precision, and the
    # rest of the step is compared from the GPU's choices
    d2all = (Wb * (Yall.reshape(rows, S, -1) - T[:, None, :]) ** 2).sum(-1)
    assert np.all(d2all[np.arange(rows), got_c] <= d2all.min(axis=1) * (1 + 1e-3))
    if not np.all(got_c == wc):
        layers = MO.unflatten(p, dims)
        Xc = MO.input_rows(feats, fr, 99, np.arange(rows), got_c, m.d_noise)
        Yc, cache = MO.forward(layers, Xc, bf16=True)
        wl, dYc = MO.mse(Yc, T, W)
        wg = MO.backward(layers, cache, dYc, bf16=True)
        w1, _, _ = MO.adam(p, zero, zero, wg, 1, 1e-3)
    assert abs(loss.item() - wl) <= 1e-3 * wl
    assert _rel(g, wg) <= 5e-3
    # first Adam step moves each parameter by about lr * sign(g): compare
    # where the gradient is not tiny
    big = np.abs(wg) > 1e-3 * np.abs(wg).max()
    assert np.max(np.abs(p1 - w1)[big]) <= 2e-5
    assert np.max(np.abs(p1 - w1)) <= 2.1e-3
    m.close()


def test_adam_matches_oracle_over_two_steps():
    m, dims, p, feats, fr, draw = _setup("small", 128, seed=3)
    rng = np.random.default_rng(13)
    dY = rng.standard_normal((128, m.d_out)).astype(np.float32)
    X = MO.input_rows(feats, fr, 5, np.arange(128), draw, m.d_noise)
    q, mo, vo = p.copy(), np.zeros_like(p), np.zeros_like(p)
    for t in (1, 2):
        m.forward(_dev(feats), 128, 5, _dev(fr, torch.int32), _dev(draw, torch.int32))
        m.backward(_dev(dY), 128)
        m.adam(lr=1e-3)
        layers = MO.unflatten(q, dims)
        _, cache = MO.forward(layers, X, bf16=True)
        g = MO.backward(layers, cache, dY.astype(np.float64), bf16=True)
        q, mo, vo = MO.adam(q, mo, vo, g, t, 1e-3)
    got = m.params().cpu().numpy()
    big = np.abs(g) > 1e-2 * np.abs(g).max()
    assert np.max(np.abs(got - q)[big]) <= 5e-5
    assert np.max(np.abs(got - q)) <= 4.1e-3
    m.close()


def test_sample_matches_oracle_and_respects_bounds():
    prob = I.packing(0, 7)
    D = prob.dim
    m, dims, p, feats, fr, _ = _setup("proposer", 4096, seed=4)
    n, ld = 1000, 1024
    rng = np.random.default_rng(14)
    f = rng.standard_normal(120).astype(np.float32)
    mean = rng.standard_normal(D).astype(np.float32)
    std = (0.2 + rng.random(D)).astype(np.float32)
    lo, hi = prob.bounds()
    wrap = I.angle_dims(prob)
    X = torch.full((D, ld), 7.0, device="cuda")
    M = torch.full((D, ld), 7.0, device="cuda")
    V = torch.full((D, ld), 7.0, device="cuda")
    m.sample(_dev(f), 31, _dev(mean), _dev(std), _dev(lo), _dev(hi), _dev(wrap, torch.uint8), X, M, V, n)
    Xh = X.cpu().numpy()
    assert np.all(M[:, :n].cpu().numpy() == 0) and np.all(V[:, :n].cpu().numpy() == 0)
    assert np.all(Xh[:, n:] == 7.0)
    x = Xh[:, :n].T.astype(np.float64)
    assert np.all(x >= lo.astype(np.float32) - 1e-7) and np.all(x <= hi.astype(np.float32) + 1e-7)
    Y, _ = MO.forward(MO.unflatten(p, dims), MO.input_rows(f[None], np.zeros(n, int), 31, np.arange(n),
                                                             np.zeros(n, int), 32))
    want = MO.destandardize(Y, mean, std, lo, hi, wrap)
    diff = np.abs(x - want)
    # a wrapped angle near +-pi may land on the other end
    w = wrap.astype(bool)
    diff[:, w] = np.minimum(diff[:, w], np.abs(diff[:, w] - 2 * math.pi))
    scale = np.linalg.norm(Y) / math.sqrt(Y.size)
    assert np.max(diff / std) <= 2e-2 * max(1.0, scale), np.max(diff / std)
    m.close()


def test_training_lowers_the_loss():
    from paper_2411_11833_amd.seeds import GpuMlp
    m = GpuMlp(8, 8, 64, 2, 3, max_rows=8 * 1024)
    dims = m.dims
    m.set_params(_dev(I.mlp_init(dims, 5)))
    rng = np.random.default_rng(15)
    feats = rng.standard_normal((16, 8)).astype(np.float32)
    fr = rng.integers(0, 16, 1024).astype(np.int32)
    # two modes per scene: the network must use the noise to cover both
    T = (feats[fr, :3] + np.where(rng.random((1024, 1)) < 0.5, 1.0, -1.0)).astype(np.float32)
    Fd, Rd, Td = _dev(feats), _dev(fr, torch.int32), _dev(T)
    losses = []
    for k in range(300):
        losses.append(m.imle_step(Fd, Rd, Td, 8, 1000 + k, lr=3e-3).item())
    print("loss", losses[0], losses[-1])
    assert np.mean(losses[-20:]) < 0.3 * np.mean(losses[:5])
    m.close()
