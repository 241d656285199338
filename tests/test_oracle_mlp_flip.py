"""Pins of the network's flipping input encoding, training targets and warm-start decode
(oracle side): the encoding decodes back to every mode id, the targets of a trajectory
that is linear in time are the closed-form samples, and a decoded warm start satisfies
the flipping dynamics rows for the twist and the finger coordinates exactly (forward
differences), with the contact forces the mode prescribes."""
import math

import numpy as np

from paper_2609_21803_amd import instances as I


def test_flip_encoding_decodes_back_to_every_mode_id():
    from oracle.mlp import encode_flip, POSE_DIMS, SEG_SLOT
    ids = np.arange(845)
    B = len(ids)
    nseg = np.ones(B, np.int32)
    modes = np.zeros((B, 6), np.int32)
    modes[:, 0] = ids
    knots = np.zeros((B, 6), np.int32)
    knots[:, 0] = 1 + ids % 15
    x0 = np.tile(I.FLIP_X0, (B, 1))
    goal = np.tile([0.1, np.pi / 2], (B, 1))
    X = encode_flip(x0, goal, np.full((B, 1), 0.7), nseg, modes, knots)
    s = X[:, POSE_DIMS:POSE_DIMS + SEG_SLOT]
    f1, f2, g = s[:, :13].argmax(1), s[:, 13:26].argmax(1), s[:, 26:31].argmax(1)
    assert np.array_equal((f1 * 13 + f2) * 5 + g, ids)
    assert np.all(s[:, :31].sum(1) == 3)                          # one bit per factor
    assert np.allclose(s[:, 31], knots[:, 0] / 15) and np.all(s[:, 32] == 1)
    assert np.all(X[:, POSE_DIMS + SEG_SLOT:] == 0)               # absent segments are zero
    # pose block: at rest at the origin, goal a quarter turn
    assert np.allclose(X[0, :12], [0, 0.05, 1, 0, 0.1, 0, 0, 1, 0.1, 0, np.pi / 2, 0.7], atol=1e-7)


def _linear_traj(B, nmax, rng):
    """rows r_k = a + b k (per order and channel)"""
    a = rng.normal(size=(B, 1, 17))
    b = rng.normal(size=(B, 1, 17))
    k = np.arange(nmax + 1)[None, :, None]
    return a + b * k, a, b


def test_flip_targets_of_a_linear_trajectory_are_the_closed_form_samples():
    from oracle.mlp import targets, WS_SLOTS, WS_CH
    rng = np.random.default_rng(5)
    B, nmax = 16, 60
    b = I.flip_batch(11, B, n_pairs=4, kmin=1, kmax=6, knots=10)
    b["knots"] = np.where(b["knots"] > 0, rng.integers(1, 11, (B, 6)), 0).astype(np.int32)
    tr, a, s = _linear_traj(B, nmax, rng)
    feas = (np.arange(B) % 3 != 0).astype(np.uint8)
    cost = rng.uniform(0, 5, B)
    yf, yc, yt, mk = targets(tr, b["nseg"], b["knots"], feas, cost, nch=8)
    yt = yt.reshape(B, 6, WS_SLOTS, WS_CH)
    mk = mk.reshape(B, 6, WS_SLOTS, WS_CH)
    for i in range(B):
        k0 = 0
        for j in range(int(b["nseg"][i])):
            n = int(b["knots"][i, j])
            t = k0 + np.arange(WS_SLOTS) / (WS_SLOTS - 1) * n
            assert np.allclose(yt[i, j, :, :8], a[i, 0, :8] + s[i, 0, :8] * t[:, None], atol=1e-12)
            k0 += n
        assert mk[i].sum() == feas[i] * 8 * WS_SLOTS * b["nseg"][i]
    assert np.all(yt[..., 8:] == 0) and np.all(mk[..., 8:] == 0)
    assert np.array_equal(yf, feas) and np.allclose(yc, np.where(feas, np.log1p(cost), 0))


def test_decoded_flip_warm_start_follows_the_dynamics_and_the_mode_forces():
    from oracle import flip as F
    from oracle.mlp import decode_warm_flip, targets, FLIP_MG, FLIP_MU
    rng = np.random.default_rng(8)
    B = 12
    b = I.flip_batch(21, B, n_pairs=4, kmin=1, kmax=4, knots=14)   # 14 intervals: every knot is a sample
    nmax = 56
    tr, _, _ = _linear_traj(B, nmax, rng)
    _, _, yt, _ = targets(tr, b["nseg"], b["knots"], np.ones(B, np.uint8), np.zeros(B), nch=8)
    Y = np.zeros((B, 736))
    Y[:, 2:722] = yt
    W = decode_warm_flip(Y, b["x0"], b["nseg"], b["modes"], b["knots"], nmax)
    N = (b["knots"] * (np.arange(6)[None, :] < b["nseg"][:, None])).sum(1)
    for i in range(B):
        n = int(N[i])
        assert np.allclose(W[i, 0, :8], b["x0"][i])
        assert np.allclose(W[i, 1:n + 1, :8], tr[i, 1:n + 1, :8], atol=1e-12)
        assert np.all(W[i, n:, 8:] == 0)                             # last knot's controls, padding
        K = int(b["nseg"][i])
        seq = F.Seq(b["modes"][i, :K], b["knots"][i, :K], goal=b["goal"][i], mu_g=float(b["inst"][i, 0]),
                    x0=b["x0"][i])
        z = W[i, :n + 1].copy()
        z = np.concatenate([np.concatenate([z[k, 8:], z[k + 1, :8]]) for k in range(n)])
        k = 0
        for j in range(K):
            m = int(b["modes"][i, j])
            for _ in range(int(b["knots"][i, j])):
                c, _ = seq.rows(k, seq.args(z, k), complex_step=False)
                assert np.allclose(c[3:8], 0, atol=1e-9), (i, k, c[:8])   # twist and finger-coordinate defects
                u = W[i, k, 8:]
                for f, code in enumerate((m // 65, (m // 5) % 13)):
                    fn, ft = u[3 + 3 * f], u[4 + 3 * f]
                    if code == 0:
                        assert fn == 0 and ft == 0
                    else:
                        slip = (code - 1) % 3
                        assert math.isclose(fn, FLIP_MG / 2)
                        assert math.isclose(ft, (0.0, FLIP_MU * fn, -FLIP_MU * fn)[slip], abs_tol=1e-15)
                k += 1
