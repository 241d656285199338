"""GPU parity of the network's flipping hooks against the oracle: the input encoding (BF16
bits), the training targets built from evaluator trajectories, and the warm-start decode
of network outputs."""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def test_flip_encoder_matches_oracle():
    from oracle.mlp import bf16_bits, encode_flip
    from paper_2609_21803_amd import native
    b = I.flip_batch(31, 1000, n_pairs=16, kmin=1, kmax=6, knots=10)
    b["knots"] = np.where(b["knots"] > 0, np.random.default_rng(2).integers(1, 16, b["knots"].shape), 0)
    d = native.to_device(b)
    x = native.mlp_encode(d, task=native.TASK_FLIP).cpu().numpy().view(np.uint16)
    ref = bf16_bits(encode_flip(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"]))
    diff = x.astype(np.int32) - ref.astype(np.int32)
    assert np.all(np.abs(diff) <= 1)                       # device cos / sin within one BF16 ulp
    assert np.all(diff[:, [0, 1, 4, 5, 8, 9, 10, 11]] == 0) and np.all(diff[:, 16:] == 0)


def test_flip_targets_and_warm_decode_match_oracle():
    import torch
    from oracle.mlp import decode_warm_flip, targets
    from paper_2609_21803_amd import native
    b = I.flip_tiny(seed=3300, B=300)
    d = native.to_device(b)
    nmax = 15
    ctx = native.Context(max_batch=300, max_intervals=nmax, task=native.TASK_FLIP)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()
    yf, yc, yt, mk = [a.cpu().numpy() for a in native.mlp_targets(d, out, nmax, task=native.TASK_FLIP)]
    tr = out["traj"].cpu().numpy().astype(np.float64)
    fe = out["feasible"].cpu().numpy()
    co = out["cost"].cpu().numpy().astype(np.float64)
    ryf, ryc, ryt, rmk = targets(tr, b["nseg"], b["knots"], fe, co, nch=8)
    assert np.array_equal(yf, ryf) and np.array_equal(mk, rmk)
    fin = np.isfinite(ryc)
    assert np.allclose(yc[fin], ryc[fin], atol=1e-6, rtol=1e-6)
    assert np.allclose(yt, ryt, atol=1e-5, rtol=1e-6)
    # decode of arbitrary network outputs
    Y = np.random.default_rng(4).normal(size=(300, 736)).astype(np.float32)
    w = native.mlp_decode_warm(torch.as_tensor(Y).cuda(), d, nmax, task=native.TASK_FLIP).cpu().numpy()
    ref = decode_warm_flip(Y.astype(np.float64), np.asarray(b["x0"], np.float32).astype(np.float64), b["nseg"],
                           b["modes"], b["knots"], nmax)
    assert w.shape == ref.shape
    assert np.allclose(w, ref, atol=1e-4, rtol=1e-5), np.abs(w - ref).max()
