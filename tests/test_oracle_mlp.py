"""Pins of the network oracle: finite differences and torch autograd (FP64, no
quantisation), closed forms of GELU and of the BF16 rounding."""
import math

import numpy as np
import pytest


def test_bf16_rounding_closed_form():
    from oracle.mlp import bf16_round
    # exactly representable values stay; halfway cases round to even
    assert bf16_round(1.0) == 1.0 and bf16_round(-2.5) == -2.5
    one_ulp = 2.0 ** -7
    assert bf16_round(1.0 + one_ulp / 2) == 1.0                 # tie -> even mantissa (…0)
    assert bf16_round(1.0 + 3 * one_ulp / 2) == 1.0 + 2 * one_ulp  # tie -> even mantissa
    assert bf16_round(1.0 + 0.51 * one_ulp) == 1.0 + one_ulp
    x = np.random.default_rng(0).normal(size=10000)
    r = bf16_round(x)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8 * 1.0001)


def test_gelu_closed_forms():
    from oracle.mlp import gelu, gelu_grad
    assert gelu(np.array([0.0]))[0] == 0.0
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    assert np.allclose(gelu_grad(z), (gelu(z + h) - gelu(z - h)) / (2 * h), atol=1e-8)
    assert abs(gelu(np.array([1.0]))[0] - 0.5 * (1 + math.erf(1 / math.sqrt(2)))) < 1e-15


def _tiny(seed=0, B=5):
    from oracle.mlp import Net
    net = Net(in_dim=10, hidden=7, layers=3, out_dim=2 + 720)
    rng = np.random.default_rng(seed)
    flat = net.init(seed) + 0.01 * rng.normal(size=net.n_params)
    X = rng.normal(size=(B, 10))
    yf = (rng.random(B) < 0.5).astype(float)
    yc = rng.random(B)
    yt = rng.normal(size=(B, 720))
    mask = (rng.random((B, 720)) < 0.3).astype(float)
    return net, flat, X, yf, yc, yt, mask


def _loss(net, flat, X, yf, yc, yt, mask):
    Y, _ = net.forward(flat, X, quantize=False)
    return net.loss_grad(Y, yf, yc, yt, mask)[0].sum()


def test_gradient_matches_finite_differences():
    net, flat, X, yf, yc, yt, mask = _tiny()
    Y, cache = net.forward(flat, X, quantize=False)
    _, dY = net.loss_grad(Y, yf, yc, yt, mask)
    g = net.backward(flat, cache, dY, quantize=False)
    idx = np.random.default_rng(1).choice(net.n_params, 300, replace=False)
    for i in idx:
        h = 1e-6
        fp, fm = flat.copy(), flat.copy()
        fp[i] += h
        fm[i] -= h
        fd = (_loss(net, fp, X, yf, yc, yt, mask) - _loss(net, fm, X, yf, yc, yt, mask)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, g[i])


def test_gradient_matches_torch_autograd_fp64():
    import torch
    net, flat, X, yf, yc, yt, mask = _tiny(seed=3, B=9)
    Y, cache = net.forward(flat, X, quantize=False)
    _, dY = net.loss_grad(Y, yf, yc, yt, mask)
    g = net.backward(flat, cache, dY, quantize=False)
    p = torch.tensor(flat, dtype=torch.float64, requires_grad=True)
    parts, o = [], 0
    for n, k in net.shapes:
        W = p[o:o + n * k].reshape(n, k)
        o += n * k
        b = p[o:o + n]
        o += n
        parts.append((W, b))
    h = torch.tensor(X)
    for l, (W, b) in enumerate(parts):
        z = h @ W.T + b
        h = torch.nn.functional.gelu(z) if l < len(parts) - 1 else z
    x = h[:, 0]
    t = lambda a: torch.tensor(a)
    bce = torch.nn.functional.binary_cross_entropy_with_logits(x, t(yf), reduction="mean")
    nf = max(yf.sum(), 1.0)
    nm = max(mask.sum(), 1.0)
    lc = (t(yf) * (h[:, 1] - t(yc)) ** 2).sum() / nf
    lw = (t(mask) * (h[:, 2:] - t(yt)) ** 2).sum() / nm
    (bce + lc + lw).backward()
    assert np.allclose(p.grad.numpy(), g, rtol=1e-9, atol=1e-12)


def test_adamw_first_step_closed_form():
    """First AdamW step moves every parameter by lr * (sign(g) + wd * w) (bias-corrected
    moments equal g and g^2), up to eps."""
    from oracle.mlp import Net
    rng = np.random.default_rng(2)
    w = rng.normal(size=100)
    g = rng.normal(size=100)
    w1, m, v = Net.adamw(w, g, np.zeros(100), np.zeros(100), 1, 1e-3, 1e-4)
    assert np.allclose(w1, w - 1e-3 * (np.sign(g) + 1e-4 * w), atol=1e-9)
