"""Pins of the network's free-motion input encoding, training targets and warm-start decode
(oracle side): hand-written encoding vectors and a round trip of every id in every one of
the eight slots; the targets of a trajectory that is linear in time are the closed-form
samples, with the duration taken from its own column under optimised timing; a decoded
warm start reproduces the trajectory at the sample knots and satisfies the pusher's
defect rows of the free-motion oracle model exactly, with the durations clamped to the
model's bounds."""
import numpy as np
import pytest


def test_encode_free_hand_written_vectors():
    """Layout: 16 pose entries (start x, y, cos, sin; goal x, y, cos, sin; goal - start
    x, y, angle; friction; pusher start p_x, p_y; two zeros), then eight slots of 64:
    one-hot id (16), intervals / 15, presence flag, zeros; absent segments all zero."""
    from oracle.mlp import encode_free
    x0 = np.array([[0.0, 0.0, 0.0, 0.08, 0.0], [0.1, -0.2, np.pi, 0.0, -0.08]])
    goal = np.array([[0.25, -0.125, 0.0], [0.5, 0.0, 0.0]])
    inst = np.array([[0.375], [0.5]])
    nseg = np.array([8, 1], np.int32)
    modes = np.array([[12, 0, 13, 4, 14, 6, 15, 9], [15, 0, 0, 0, 0, 0, 0, 0]], np.int32)
    knots = np.array([[8, 5, 15, 1, 2, 3, 4, 12], [3, 0, 0, 0, 0, 0, 0, 0]], np.int32)
    X = encode_free(x0, goal, inst, nseg, modes, knots)
    E = np.zeros((2, 528))
    E[0, [2, 6]] = 1.0
    E[0, 4], E[0, 5] = 0.25, -0.125
    E[0, 8], E[0, 9] = 0.25, -0.125
    E[0, 11], E[0, 12] = 0.375, 0.08
    for j, (m, n) in enumerate(zip(modes[0], knots[0])):
        E[0, 16 + 64 * j + m], E[0, 16 + 64 * j + 16], E[0, 16 + 64 * j + 17] = 1.0, n / 15, 1.0
    E[1, 0], E[1, 1], E[1, 2], E[1, 3] = 0.1, -0.2, -1.0, 0.0
    E[1, 4], E[1, 5], E[1, 6], E[1, 7] = 0.5, 0.0, 1.0, 0.0
    E[1, 8], E[1, 9], E[1, 10] = 0.4, 0.2, -np.pi
    E[1, 11], E[1, 13] = 0.5, -0.08
    E[1, 16 + 15], E[1, 16 + 16], E[1, 16 + 17] = 1.0, 3 / 15, 1.0
    assert X.shape == (2, 528)
    assert np.allclose(X, E, rtol=0, atol=2e-7), np.argwhere(~np.isclose(X, E, rtol=0, atol=2e-7))


def test_free_encoding_decodes_back_to_every_id_in_every_slot():
    from oracle.mlp import encode_free, POSE_DIMS, SEG_SLOT
    B = 16 * 8
    ids = np.arange(B) % 16
    slot = np.arange(B) // 16
    nseg = (slot + 1).astype(np.int32)
    modes = np.zeros((B, 8), np.int32)
    modes[np.arange(B), slot] = ids
    knots = np.where(np.arange(8)[None, :] <= slot[:, None], 1 + np.arange(B)[:, None] % 15, 0).astype(np.int32)
    x0 = np.tile([0.0, 0.0, 0.0, -0.08, 0.0], (B, 1))
    X = encode_free(x0, np.tile([0.1, 0.1, 0.5], (B, 1)), np.full((B, 1), 0.4), nseg, modes, knots)
    s = X[np.arange(B)[:, None], POSE_DIMS + SEG_SLOT * slot[:, None] + np.arange(SEG_SLOT)[None, :]]
    assert np.array_equal(s[:, :16].argmax(1), ids) and np.all(s[:, :16].sum(1) == 1)
    assert np.allclose(s[:, 16], knots[np.arange(B), slot] / 15) and np.all(s[:, 17] == 1)
    assert np.all(s[:, 18:] == 0)
    for b in range(B):                     # slots past the order's last segment are zero
        assert np.all(X[b, POSE_DIMS + SEG_SLOT * nseg[b]:] == 0)


def _linear_traj(B, nmax, width, rng):
    a = rng.normal(size=(B, 1, width))
    b = rng.normal(size=(B, 1, width))
    k = np.arange(nmax + 1)[None, :, None]
    return a + b * k, a, b


def _free_batch(rng, B, kmax, knots_of):
    from oracle import free as F
    keys = F.seed(kmax)
    pick = rng.choice(len(keys), B, replace=False)
    nseg = np.zeros(B, np.int32)
    modes = np.zeros((B, 8), np.int32)
    knots = np.zeros((B, 8), np.int32)
    for i, p in enumerate(pick):
        m = F.key_modes(int(keys[p]))
        nseg[i] = len(m)
        modes[i, :len(m)] = m
        knots[i, :len(m)] = knots_of(len(m))
    return nseg, modes, knots


@pytest.mark.parametrize("timed", [False, True])
def test_free_targets_of_a_linear_trajectory_are_the_closed_form_samples(timed):
    from oracle.mlp import targets, WS_SLOTS, WS_CH
    rng = np.random.default_rng(6 + timed)
    B, width = 24, (10 if timed else 9)
    nseg, modes, knots = _free_batch(rng, B, 8, lambda K: rng.integers(1, 11, K))
    nmax = int(knots.sum(1).max())
    tr, a, s = _linear_traj(B, nmax, width, rng)
    feas = (np.arange(B) % 3 != 0).astype(np.uint8)
    cost = rng.uniform(0, 5, B)
    cols = [0, 1, 2, 3, 4, 5, 6] + ([9] if timed else [])
    yf, yc, yt, mk = targets(tr, nseg, knots, feas, cost, nch=len(cols), n_seg=8, cols=cols)
    assert yt.shape == (B, 960)
    yt = yt.reshape(B, 8, WS_SLOTS, WS_CH)
    mk = mk.reshape(B, 8, WS_SLOTS, WS_CH)
    for i in range(B):
        k0 = 0
        for j in range(int(nseg[i])):
            n = int(knots[i, j])
            t = k0 + np.arange(WS_SLOTS) / (WS_SLOTS - 1) * n
            assert np.allclose(yt[i, j, :, :len(cols)], a[i, 0, cols] + s[i, 0, cols] * t[:, None], atol=1e-12)
            k0 += n
        assert mk[i].sum() == feas[i] * len(cols) * WS_SLOTS * nseg[i]
        assert np.all(yt[i, int(nseg[i]):] == 0)
    assert np.all(yt[..., len(cols):] == 0) and np.all(mk[..., len(cols):] == 0)
    assert np.array_equal(yf, feas) and np.allclose(yc, np.where(feas, np.log1p(cost), 0))


@pytest.mark.parametrize("timed", [False, True])
def test_decoded_free_warm_start_reproduces_the_knots_and_the_pusher_defects(timed):
    """Segments of 14 intervals (every knot a sample): the decoded states and forces are the
    trajectory's, the durations its clamped ones; the free-motion oracle model's pusher
    defect rows (p_{k+1} - p_k - h v_k, two rows) vanish on every interval; the last knot's
    controls are zero; the start state is x0."""
    from oracle import free as F
    from oracle.mlp import decode_warm_free, targets
    rng = np.random.default_rng(11 + timed)
    B, width = 12, (10 if timed else 9)
    nseg, modes, knots = _free_batch(rng, B, 4, lambda K: np.full(K, 14))
    nmax = 56
    tr, _, _ = _linear_traj(B, nmax, width, rng)
    if timed:                          # durations spread inside and outside the bounds
        tr[:, :, 9] = rng.uniform(-0.1, 0.4, (B, nmax + 1))
    cols = [0, 1, 2, 3, 4, 5, 6] + ([9] if timed else [])
    _, _, yt, _ = targets(tr, nseg, knots, np.ones(B, np.uint8), np.zeros(B), nch=len(cols), n_seg=8, cols=cols)
    Y = np.zeros((B, 968))
    Y[:, 2:962] = yt
    x0 = np.tile([0.0, 0.0, 0.0, -0.08, 0.0], (B, 1))
    W = decode_warm_free(Y, x0, nseg, knots, nmax, timed=timed)
    assert W.shape == (B, nmax + 1, width)
    N = knots.sum(1)
    for i in range(B):
        n = int(N[i])
        assert np.allclose(W[i, 0, :5], x0[i])
        assert np.allclose(W[i, 1:n + 1, :5], tr[i, 1:n + 1, :5], atol=1e-12)
        assert np.allclose(W[i, 1:n, 5:7], tr[i, 1:n, 5:7], atol=1e-12)
        if timed:
            assert np.allclose(W[i, :n, 9], np.clip(tr[i, :n, 9], F.H_MIN, F.H_MAX), atol=1e-12)
        assert np.all(W[i, n, 5:] == 0) and np.all(W[i, n + 1:] == 0)
        for k in range(n):
            mode = int(np.repeat(modes[i, :nseg[i]], knots[i, :nseg[i]])[k])
            v = np.concatenate([W[i, k, :5], W[i, k, 5:], W[i, k + 1, :5]])
            c, _, _, _ = F.rows(mode, 0.4, v, timed=timed)
            assert np.allclose(c[3:5], 0, atol=1e-12), (i, k, c[3:5])
