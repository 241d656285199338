"""GPU parity of the learned network's BF16 matrix-core kernels against the NumPy oracle.

Bars: every forward output within its element-wise bound derived from the arithmetic
(float32 accumulation of exact BF16 products, float32 GELU, BF16 rounding of the hidden
activations); each parameter tensor's gradient within 1e-2 relative Frobenius error and
cosine >= 0.9999 of the oracle computed in FP64 with BF16 rounding at the same tensors;
one AdamW step within 1e-5 relative; the input encoding identical except single-ulp
differences of the trigonometric entries.
"""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def _net_and_data(B=300, seed=4):
    import torch
    from oracle.mlp import Net, bf16_bits
    from paper_2609_21803_amd import native
    net = Net(416, 512, 4, 736)
    flat = net.init(seed)
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, 416)) * (rng.random((B, 416)) < 0.3)
    yf = (rng.random(B) < 0.4).astype(float)
    yc = rng.random(B)
    yt = rng.normal(size=(B, 720)) * 0.1
    mask = (rng.random((B, 720)) < 0.5).astype(float) * yf[:, None]
    m = native.MLP(max_batch=1024, seed=seed)
    m.set_params(torch.as_tensor(flat, dtype=torch.float32).cuda())
    xb = torch.as_tensor(bf16_bits(X).view(np.int16)).cuda()
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    return net, np.asarray(flat, np.float32).astype(np.float64), X, yf, yc, yt, mask, m, xb, t


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


U32 = 2.0 ** -24          # float32 unit roundoff


def _gamma(n):
    return n * U32 / (1.0 - n * U32)


def _bf16_spacing(x):
    """Spacing of the BF16 numbers at |x| (8 significant bits), taken at the binade above."""
    e = np.floor(np.log2(np.maximum(np.abs(x), 1e-38)))
    return np.exp2(e - 7.0)


def _forward_error_bound(net, flat, X):
    """Element-wise bound of |device - oracle| for every network output, from the
    arithmetic: both sides multiply the same BF16 operands exactly; the device adds K
    products and the bias in float32 in some order (|error| <= gamma_{K+1} sum |a w| +
    |b|), evaluates GELU in float32 (a few roundings, |GELU'| <= 1.13) and rounds the hidden
    activations to BF16 -- where the two float values lie on either side of a BF16 rounding
    midpoint (within the error bound of it), the BF16 values differ by one spacing."""
    from oracle.mlp import bf16_round, gelu
    Yo, (H, Z) = net.forward(flat, X)
    P = net.unpack(flat)
    e = np.zeros_like(H[0])
    for l, (W, b) in enumerate(P):
        Wq = np.abs(bf16_round(W))
        K = W.shape[1]
        Ez = e @ Wq.T + _gamma(K + 1) * (np.abs(H[l]) @ Wq.T + np.abs(b))
        if l == net.nl - 1:
            return Yo, Ez
        z = Z[l]
        g = gelu(z)
        Eg = 1.13 * Ez + 16.0 * U32 * (np.abs(g) + 0.5 * np.abs(z))
        sp = _bf16_spacing(np.abs(g) + Eg)
        mant = np.abs(g) / (128.0 * _bf16_spacing(np.abs(g)))             # in [1, 2)
        frac = (mant - 1.0) * 128.0
        dist = np.abs(frac - np.floor(frac) - 0.5) * _bf16_spacing(np.abs(g))
        near_pow2 = np.abs(np.abs(g) - np.exp2(np.round(np.log2(np.maximum(np.abs(g), 1e-38))))) <= Eg
        e = Eg + np.where((dist <= Eg) | near_pow2, sp, 0.0)


@pytest.mark.parametrize("B", [300, 512])
def test_forward_within_the_elementwise_accumulation_bound(B):
    """A network of the production widths with one hidden layer (416 -> 512 -> 736, the same
    matrix-core products as every layer of the full network): every output lies within its
    own element-wise bound derived from the arithmetic.  (Through four hidden layers a
    worst-case bound compounds the possible BF16 flips of every layer and says nothing; the
    full network is compared by relative error in the next test.)"""
    import torch
    from oracle.mlp import Net, bf16_bits
    from paper_2609_21803_amd import native
    net = Net(416, 512, 1, 736)
    flat = np.asarray(net.init(11), np.float32).astype(np.float64)
    rng = np.random.default_rng(11)
    X = rng.normal(size=(B, 416)) * (rng.random((B, 416)) < 0.3)
    m = native.MLP(max_batch=1024, seed=11, layers=1)
    m.set_params(torch.as_tensor(flat, dtype=torch.float32).cuda())
    Y = m.forward(torch.as_tensor(bf16_bits(X).view(np.int16)).cuda()).cpu().numpy().astype(np.float64)
    Yo, bound = _forward_error_bound(net, flat, X)
    err = np.abs(Y - Yo)
    ratio = err / np.maximum(bound, 1e-300)
    print(f"forward, one hidden layer: max |err| {err.max():.3e}, max err/bound {ratio.max():.3f}, "
          f"median bound {np.median(bound):.2e}, median |y| {np.median(np.abs(Yo)):.2e}")
    assert np.all(err <= bound), np.unravel_index(np.argmax(ratio), ratio.shape)


def test_forward_matches_oracle():
    """The full network (four hidden layers): relative error per output block."""
    net, flat, X, *_, m, xb, t = _net_and_data()
    Y = m.forward(xb).cpu().numpy().astype(np.float64)
    Yo, _ = net.forward(flat, X)
    for cols in (slice(0, 1), slice(1, 2), slice(2, 722)):
        assert _rel(Y[:, cols], Yo[:, cols]) <= 1e-2
    assert _rel(Y, Yo) <= 3e-3, _rel(Y, Yo)


@pytest.mark.parametrize("B", [512, 300])
def test_gradients_and_adamw_step_match_oracle(B):
    """B = 512 takes the weight-gradient products over transposed batch-contiguous copies,
    B = 300 (not a multiple of 8) the row-major operands."""
    from oracle.mlp import Net
    net, flat, X, yf, yc, yt, mask, m, xb, t = _net_and_data(B=B, seed=7)
    loss = m.train_step(xb, t(yf), t(yc), t(yt), t(mask), lr=1e-3, weight_decay=1e-4).cpu().numpy()
    g = m.grads().cpu().numpy().astype(np.float64)
    p1 = m.get_params().cpu().numpy().astype(np.float64)
    Yo, cache = net.forward(flat, X)
    lo, dY = net.loss_grad(Yo, yf, yc, yt, mask)
    go = net.backward(flat, cache, dY)
    assert np.allclose(loss, lo, rtol=1e-2), (loss, lo)
    o = 0
    for n, k in net.shapes:
        for size in (n * k, n):
            a, b = g[o:o + size], go[o:o + size]
            cos = a @ b / max(np.linalg.norm(a) * np.linalg.norm(b), 1e-30)
            assert _rel(a, b) <= 1e-2 and cos >= 0.9999, (n, k, size, _rel(a, b), cos)
            o += size
    # one AdamW step from the GPU's own gradients reproduces the GPU's parameters
    w1, _, _ = Net.adamw(flat, g, np.zeros_like(flat), np.zeros_like(flat), 1, 1e-3, 1e-4)
    assert _rel(p1, w1) <= 1e-5


def test_encoder_matches_oracle():
    import torch
    from oracle.mlp import bf16_bits, encode_push
    from paper_2609_21803_amd import native
    b = I.push_hetero(B=777, seed=9)
    d = native.to_device(b)
    x = native.mlp_encode(d).cpu().numpy().view(np.uint16)
    ref = bf16_bits(encode_push(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"]))
    diff = x.astype(np.int32) - ref.astype(np.int32)
    assert np.all(np.abs(diff) <= 1)
    assert np.all(diff[:, [0, 1, 4, 5, 8, 9, 10, 11]] == 0) and np.all(diff[:, 16:] == 0)


def test_targets_and_warm_decode():
    import torch
    from oracle.mlp import targets
    from paper_2609_21803_amd import native
    b = I.push_hetero(B=200, seed=12, kmax=4)
    d = native.to_device(b)
    ctx = native.Context(max_batch=200, max_intervals=75)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()
    yf, yc, yt, mk = [a.cpu().numpy() for a in native.mlp_targets(d, out, 75)]
    tr = out["traj"].cpu().numpy().astype(np.float64)
    fe = out["feasible"].cpu().numpy()
    co = out["cost"].cpu().numpy().astype(np.float64)
    ryf, ryc, ryt, rmk = targets(tr, b["nseg"], b["knots"], fe, co)
    assert np.array_equal(yf, ryf) and np.array_equal(mk, rmk)
    assert np.allclose(yc, ryc, atol=1e-6) and np.allclose(yt, ryt, atol=1e-5)
    # decoding the targets as if they were network outputs reproduces the trajectory at the
    # sample knots of each segment (intervals 14 -> every knot is a sample)
    Y = torch.zeros((200, 736), device="cuda")
    Y[:, 2:722] = torch.as_tensor(yt).cuda()
    w = native.mlp_decode_warm(Y, d, 75).cpu().numpy()
    N = I.n_intervals(b)
    for i in np.where((fe == 1) & np.all((b["knots"] == 14) | (b["knots"] == 0), axis=1))[0][:20]:
        assert np.allclose(w[i, 1:N[i], :4], tr[i, 1:N[i], :4], atol=1e-5)


def test_targets_and_decode_treat_invalid_counts_as_empty():
    """Knot counts that are non-positive or whose int32 sum would wrap make a sequence
    empty for the target and warm-start hooks: zero targets and mask, zero warm rows with
    x0 in row 0; valid rows of the same batch are unaffected."""
    import torch
    from paper_2609_21803_amd import native
    b = I.push_hetero(B=8, seed=21, kmax=3)
    b["nseg"][1], b["modes"][1, :4], b["knots"][1, :4] = 4, 2, 2 ** 30     # sum wraps to 0
    b["knots"][3, :2] = (5, 2 ** 31 - 1)                                  # sum wraps negative
    b["nseg"][3] = max(int(b["nseg"][3]), 2)
    b["knots"][5, 0] = -4                                                 # negative count
    d = native.to_device(b)
    nmax = 75
    traj = torch.rand((8, nmax + 1, 7), device="cuda")
    out = dict(traj=traj, feasible=torch.ones(8, dtype=torch.uint8, device="cuda"),
               cost=torch.ones(8, device="cuda"))
    yf, yc, yt, mk = [a.cpu().numpy() for a in native.mlp_targets(d, out, nmax)]
    bad = np.array([1, 3, 5])
    good = np.setdiff1d(np.arange(8), bad)
    assert np.all(yt[bad] == 0) and np.all(mk[bad] == 0)
    assert np.all(mk[good].sum(1) > 0)
    Y = torch.rand((8, 736), device="cuda")
    w = native.mlp_decode_warm(Y, d, nmax).cpu().numpy()
    assert np.all(w[bad, 1:] == 0) and np.all(w[bad, 0, 4:] == 0)
    assert np.array_equal(w[bad, 0, :4], b["x0"][bad].astype(np.float32))
    assert np.all(np.abs(w[good, 1]).sum(1) > 0)


def test_training_reduces_the_loss():
    from oracle.mlp import Net
    net, flat, X, yf, yc, yt, mask, m, xb, t = _net_and_data(B=1024, seed=3)
    first = None
    for it in range(60):
        loss = m.train_step(xb, t(yf), t(yc), t(yt), t(mask), lr=1e-3).cpu().numpy()
        if first is None:
            first = loss.copy()
    assert loss.sum() < 0.5 * first.sum(), (first, loss)
