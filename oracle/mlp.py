"""NumPy FP64 oracle of the learned proposal / warm-start network.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Written from the network's
definition: in_dim -> `layers` hidden layers (exact-erf GELU) -> out_dim; heads
[0] feasibility logit, [1] log(1 + J), [2:] warm start (6 segments, or 8 for free motion,
x 15 samples x 8 channels); loss = mean BCE + MSE of the cost head over feasible samples + MSE of the warm
start over its mask; AdamW.

With quantize=True the tensors that the matrix-core kernels take as BF16 operands are
rounded to BF16 (round to nearest even) at the same places -- inputs, weights, hidden
activations, back-propagated gradients -- and everything else is FP64.  With
quantize=False the network is plain FP64 (used by the finite-difference and autograd pins).
"""
from __future__ import annotations

import math

import numpy as np

WS_SLOTS, WS_CH, N_SEG = 15, 8, 6
POSE_DIMS, SEG_SLOT, N_MODES = 16, 64, 12


def bf16_round(x) -> np.ndarray:
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    f = np.atleast_1d(np.asarray(x, np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    nan = np.isnan(f)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    u = (u << 16).astype(np.uint32)
    out = u.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out.reshape(np.shape(x)) if np.ndim(x) else out[0]


def bf16_bits(x) -> np.ndarray:
    f = np.asarray(bf16_round(x), np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16)


def _erf(x):
    return np.vectorize(math.erf, otypes=[float])(x)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + _erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


class Net:
    def __init__(self, in_dim, hidden, layers, out_dim):
        self.dims = [in_dim] + [hidden] * layers + [out_dim]
        self.nl = layers + 1
        self.shapes = [(self.dims[l + 1], self.dims[l]) for l in range(self.nl)]
        self.n_params = sum(n * k + n for n, k in self.shapes)

    def unpack(self, flat):
        out, o = [], 0
        for n, k in self.shapes:
            W = flat[o:o + n * k].reshape(n, k)
            o += n * k
            b = flat[o:o + n]
            o += n
            out.append((W, b))
        return out

    def pack(self, parts):
        return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in parts])

    def init(self, seed):
        rng = np.random.default_rng(seed)
        parts = [(rng.uniform(-1, 1, (n, k)) / math.sqrt(k), np.zeros(n)) for n, k in self.shapes]
        return self.pack(parts)

    def forward(self, flat, X, quantize=True):
        q = bf16_round if quantize else (lambda a: np.asarray(a, np.float64))
        H = [q(X)]
        Z = []
        P = self.unpack(flat)
        for l, (W, b) in enumerate(P):
            z = H[-1] @ q(W).T + b
            if l < self.nl - 1:
                Z.append(z)
                H.append(q(gelu(z)))
            else:
                Y = z
        return Y, (H, Z)

    def loss_grad(self, Y, y_feas, y_cost, y_traj, mask):
        """Losses (3,) and dL/dY of the combined objective."""
        B = Y.shape[0]
        x = Y[:, 0]
        bce = np.maximum(x, 0) - x * y_feas + np.log1p(np.exp(-np.abs(x)))
        nf = max(y_feas.sum(), 1.0)
        nm = max(mask.sum(), 1.0)
        dc = Y[:, 1] - y_cost
        dw = Y[:, 2:2 + mask.shape[1]] - y_traj
        losses = np.array([bce.mean(), (y_feas * dc * dc).sum() / nf, (mask * dw * dw).sum() / nm])
        dY = np.zeros_like(Y)
        dY[:, 0] = (1.0 / (1.0 + np.exp(-x)) - y_feas) / B
        dY[:, 1] = 2.0 * y_feas * dc / nf
        dY[:, 2:2 + mask.shape[1]] = 2.0 * mask * dw / nm
        return losses, dY

    def backward(self, flat, cache, dY, quantize=True):
        q = bf16_round if quantize else (lambda a: np.asarray(a, np.float64))
        H, Z = cache
        P = self.unpack(flat)
        grads = [None] * self.nl
        g32 = dY
        g = q(dY)
        for l in range(self.nl - 1, -1, -1):
            W, _ = P[l]
            dW = g.T @ H[l]
            db = g32.sum(0)
            grads[l] = (dW, db)
            if l > 0:
                dX = g @ q(W)
                dz = dX * gelu_grad(Z[l - 1])
                g32 = dz
                g = q(dz)
        return self.pack(grads)

    @staticmethod
    def adamw(flat, grad, m, v, step, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
        m = b1 * m + (1 - b1) * grad
        v = b2 * v + (1 - b2) * grad * grad
        mh = m / (1 - b1 ** step)
        vh = v / (1 - b2 ** step)
        return flat - lr * (mh / (np.sqrt(vh) + eps) + wd * flat), m, v


def encode_push(x0, goal, inst, nseg, modes, knots, in_dim=416):
    """Input encoding of planar-pushing orders, computed in float32 then rounded to BF16."""
    B = len(nseg)
    X = np.zeros((B, in_dim), np.float32)
    x0 = np.asarray(x0, np.float32)
    goal = np.asarray(goal, np.float32)
    inst = np.asarray(inst, np.float32).reshape(B, -1)
    X[:, 0] = x0[:, 0]
    X[:, 1] = x0[:, 1]
    X[:, 2] = np.cos(x0[:, 2])
    X[:, 3] = np.sin(x0[:, 2])
    X[:, 4] = goal[:, 0]
    X[:, 5] = goal[:, 1]
    X[:, 6] = np.cos(goal[:, 2])
    X[:, 7] = np.sin(goal[:, 2])
    X[:, 8] = goal[:, 0] - x0[:, 0]
    X[:, 9] = goal[:, 1] - x0[:, 1]
    X[:, 10] = goal[:, 2] - x0[:, 2]
    X[:, 11] = inst[:, 0]
    for b in range(B):
        for j in range(int(nseg[b])):
            base = POSE_DIMS + SEG_SLOT * j
            X[b, base + int(modes[b, j])] = 1.0
            X[b, base + N_MODES] = np.float32(knots[b, j]) / np.float32(15.0)
            X[b, base + N_MODES + 1] = 1.0
    return X


def encode_flip(x0, goal, inst, nseg, modes, knots, in_dim=416):
    """Input encoding of flipping orders (float32, then BF16): pose block (start px, py,
    cos, sin; goal px, 0, cos, sin; goal - start px, 0, angle; table friction); per segment
    the finger-1 code, finger-2 code and table mode as separate one-hots (13 + 13 + 5), the
    interval count / 15 and a presence flag."""
    B = len(nseg)
    X = np.zeros((B, in_dim), np.float32)
    x0 = np.asarray(x0, np.float32)
    goal = np.asarray(goal, np.float32)
    inst = np.asarray(inst, np.float32).reshape(B, -1)
    X[:, 0] = x0[:, 0]
    X[:, 1] = x0[:, 1]
    X[:, 2] = np.cos(x0[:, 2])
    X[:, 3] = np.sin(x0[:, 2])
    X[:, 4] = goal[:, 0]
    X[:, 6] = np.cos(goal[:, 1])
    X[:, 7] = np.sin(goal[:, 1])
    X[:, 8] = goal[:, 0] - x0[:, 0]
    X[:, 10] = goal[:, 1] - x0[:, 2]
    X[:, 11] = inst[:, 0]
    for b in range(B):
        for j in range(int(nseg[b])):
            base = POSE_DIMS + SEG_SLOT * j
            m = int(modes[b, j])
            f1, f2, g = m // 65, (m // 5) % 13, m % 5
            X[b, base + f1] = 1.0
            X[b, base + 13 + f2] = 1.0
            X[b, base + 26 + g] = 1.0
            X[b, base + 31] = np.float32(knots[b, j]) / np.float32(15.0)
            X[b, base + 32] = 1.0
    return X


FREE_SEGS, FREE_MODES = 8, 16


def encode_free(x0, goal, inst, nseg, modes, knots, in_dim=528):
    """Input encoding of free-motion pushing orders (float32, then BF16): the pushing pose
    block (x0 holds the slider pose and then the pusher position), the pusher's start
    position at 12 and 13; per segment (up to eight) a one-hot of the 16 ids, the interval
    count / 15 at 16 and a presence flag at 17."""
    B = len(nseg)
    X = np.zeros((B, in_dim), np.float32)
    x0 = np.asarray(x0, np.float32)
    goal = np.asarray(goal, np.float32)
    inst = np.asarray(inst, np.float32).reshape(B, -1)
    X[:, 0], X[:, 1] = x0[:, 0], x0[:, 1]
    X[:, 2], X[:, 3] = np.cos(x0[:, 2]), np.sin(x0[:, 2])
    X[:, 4], X[:, 5] = goal[:, 0], goal[:, 1]
    X[:, 6], X[:, 7] = np.cos(goal[:, 2]), np.sin(goal[:, 2])
    X[:, 8] = goal[:, 0] - x0[:, 0]
    X[:, 9] = goal[:, 1] - x0[:, 1]
    X[:, 10] = goal[:, 2] - x0[:, 2]
    X[:, 11] = inst[:, 0]
    X[:, 12], X[:, 13] = x0[:, 3], x0[:, 4]
    for b in range(B):
        for j in range(int(nseg[b])):
            base = POSE_DIMS + SEG_SLOT * j
            X[b, base + int(modes[b, j])] = 1.0
            X[b, base + FREE_MODES] = np.float32(knots[b, j]) / np.float32(15.0)
            X[b, base + FREE_MODES + 1] = 1.0
    return X


def targets(traj, nseg, knots, feas, cost, nch=7, n_seg=N_SEG, cols=None):
    """Warm-start targets: per segment (n_seg slots), 15 samples at normalised times i/14
    by linear interpolation between trajectory rows of `nch` channels, channel c taken from
    row column cols[c] (default c; pushing: the 7 row entries; flipping: the 8 states;
    free motion: the 5 states and 2 forces, with optimised timing the duration, column 9,
    as channel 7); mask on those channels of present segments of feasible orders."""
    cols = list(range(nch)) if cols is None else list(cols)
    B = len(nseg)
    y_traj = np.zeros((B, n_seg * WS_SLOTS * WS_CH))
    mask = np.zeros_like(y_traj)
    for b in range(B):
        k0 = 0
        for j in range(int(nseg[b])):
            nj = int(knots[b, j])
            for i in range(WS_SLOTS):
                p = i / (WS_SLOTS - 1) * nj
                k = min(int(math.floor(p)), max(nj - 1, 0))
                fr = p - k
                for c in range(nch):
                    a0 = traj[b, k0 + k, cols[c]]
                    a1 = traj[b, k0 + min(k + 1, nj), cols[c]]
                    e = (j * WS_SLOTS + i) * WS_CH + c
                    y_traj[b, e] = a0 + fr * (a1 - a0)
                    mask[b, e] = 1.0 if feas[b] else 0.0
            k0 += nj
    y_feas = np.asarray(feas, np.float64)
    y_cost = np.where(feas, np.log1p(np.maximum(cost, 0.0)), 0.0)
    return y_feas, y_cost, y_traj, mask


FLIP_MG, FLIP_MU, FLIP_DT = 0.5 * 9.81, 0.5, 0.1


def decode_warm_flip(Y, x0, nseg, modes, knots, nmax):
    """Flipping warm start from network outputs Y [B, >= 722]: the 8 states of every knot
    interpolated linearly from the segment's 15 samples (knot k of n at sample position
    14 k / n), knot 0 replaced by the start state; controls of interval k: accelerations
    (twist rate) and face-coordinate rates as forward differences of the states over dt,
    each finger in contact pushing with mg/2 normal force and tangential force 0 (stick) or
    +-mu mg/2 (slide+/-), a free finger zero; the last knot's controls zero."""
    B = len(nseg)
    W = np.zeros((B, nmax + 1, 17))
    for b in range(B):
        y = np.asarray(Y[b, 2:2 + N_SEG * WS_SLOTS * WS_CH], np.float64).reshape(N_SEG, WS_SLOTS, WS_CH)
        k0 = 0
        for j in range(int(nseg[b])):
            nj = int(knots[b, j])
            for k in range(nj + 1):
                if k0 + k > nmax:
                    break
                p = k / nj * (WS_SLOTS - 1) if nj > 0 else 0.0
                i = min(int(math.floor(p)), WS_SLOTS - 2)
                fr = p - i
                W[b, k0 + k, :8] = y[j, i, :8] + fr * (y[j, i + 1, :8] - y[j, i, :8])
            k0 += nj
        N = min(k0, nmax)
        W[b, 0, :8] = x0[b]
        kk = 0
        for j in range(int(nseg[b])):
            m, nj = int(modes[b, j]), int(knots[b, j])
            codes = (m // 65, (m // 5) % 13)
            for _ in range(nj):
                if kk >= N:
                    break
                xa, xb = W[b, kk, :8], W[b, kk + 1, :8]
                u = W[b, kk, 8:]
                u[0:3] = (xb[3:6] - xa[3:6]) / FLIP_DT
                for f in range(2):
                    fn = ft = 0.0
                    if codes[f] != 0:
                        slip = (codes[f] - 1) % 3
                        fn = 0.5 * FLIP_MG
                        ft = (0.0, FLIP_MU * fn, -FLIP_MU * fn)[slip]
                    u[3 + 3 * f], u[4 + 3 * f] = fn, ft
                    u[5 + 3 * f] = (xb[6 + f] - xa[6 + f]) / FLIP_DT
                kk += 1
    return W


FREE_DT, FREE_H_MIN, FREE_H_MAX = 0.1, 0.02, 0.2


def decode_warm_free(Y, x0, nseg, knots, nmax, timed=False):
    """Free-motion warm start from network outputs Y [B, >= 962]: the states (x, y, theta,
    p_x, p_y) and forces (F_n, F_t) of every knot interpolated linearly from the segment's
    15 samples (knot k of n at sample position 14 k / n), with optimised timing also the
    duration (channel 7) clamped to [h_min, h_max]; knot 0 takes the start state; the pusher
    velocity of interval k is the difference of the decoded pusher positions over the
    interval's duration (dt with the fixed step), which is what the pusher's defect rows
    ask; the last knot's controls are zero.  Rows (x_k, u_k) of width 9, or 10 with h."""
    width = 10 if timed else 9
    B = len(nseg)
    W = np.zeros((B, nmax + 1, width))
    for b in range(B):
        y = np.asarray(Y[b, 2:2 + FREE_SEGS * WS_SLOTS * WS_CH], np.float64).reshape(FREE_SEGS, WS_SLOTS, WS_CH)
        k0 = 0
        for j in range(int(nseg[b])):
            nj = int(knots[b, j])
            for k in range(nj + 1):
                if k0 + k > nmax:
                    break
                p = k / nj * (WS_SLOTS - 1) if nj > 0 else 0.0
                i = min(int(math.floor(p)), WS_SLOTS - 2)
                fr = p - i
                v = y[j, i] + fr * (y[j, i + 1] - y[j, i])
                W[b, k0 + k, :7] = v[:7]
                if timed:
                    W[b, k0 + k, 9] = min(max(v[7], FREE_H_MIN), FREE_H_MAX)
            k0 += nj
        N = min(k0, nmax)
        W[b, 0, :5] = x0[b][:5]
        for k in range(N):
            h = W[b, k, 9] if timed else FREE_DT
            W[b, k, 7:9] = (W[b, k + 1, 3:5] - W[b, k, 3:5]) / h
        W[b, N, 5:] = 0.0
    return W
