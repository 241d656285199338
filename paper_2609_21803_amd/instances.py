"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and lays out arrays; it holds none of the method's
arithmetic.  Every array is produced with ``numpy.random.default_rng(seed)`` (PCG64),
so the CPU oracle and the HIP library read identical bytes.

Workloads (planar pushing, square slider of side 0.1 m, one point pusher):
  * ``push_tiny``      -- 8 start/goal pairs x all 144 two-segment orders, 5+5 intervals;
  * ``push_plain``     -- 64 pairs x all 1,728 three-segment orders, 8+8+8 intervals
                          (110,592 TOs);
  * ``push_hetero``    -- 131,072 i.i.d. orders, K ~ U{1..5} segments, ids ~ U{0..11},
                          intervals per segment ~ U{5..15}, on 64 pairs.
Start at rest at the origin with the pusher at the face centre; goal x, y ~ U[-0.3, 0.3] m,
theta ~ U[-pi, pi]; pusher friction mu ~ U[0.3, 0.5].
Free-motion pushing (``push_free_pairs``): the same slider at rest at the origin with the
pusher 3 cm in front of a face drawn uniformly; goal x, y ~ U[-0.15, 0.15] m, theta ~
U[-pi/2, pi/2]; ``orders_batch`` lays out orders given one by one.  Flipping: see the
``flip_*`` generators below.
"""
from __future__ import annotations

import itertools

import numpy as np

MAXSEG = 6
PUSH_MODES = 12          # id = 3 * face + slip, face 0..3, slip 0 stick / 1 slide+ / 2 slide-


def push_pairs(seed: int, n: int):
    """n start/goal pairs: x0 [n,4], goal [n,3], inst [n,1] (pusher friction)."""
    rng = np.random.default_rng(seed)
    goal = np.empty((n, 3))
    goal[:, 0] = rng.uniform(-0.3, 0.3, n)
    goal[:, 1] = rng.uniform(-0.3, 0.3, n)
    goal[:, 2] = rng.uniform(-np.pi, np.pi, n)
    mu = rng.uniform(0.3, 0.5, n)
    x0 = np.zeros((n, 4))
    return x0, goal, mu.reshape(n, 1)


def all_orders(K: int, n_modes: int = PUSH_MODES) -> np.ndarray:
    """Every order of exactly K segments, lexicographic: [n_modes**K, K] int32."""
    return np.array(list(itertools.product(range(n_modes), repeat=K)), dtype=np.int32).reshape(-1, K)


def _batch(x0, goal, inst, orders, knots_per_seg):
    n_pairs = x0.shape[0]
    n_ord, K = orders.shape
    B = n_pairs * n_ord
    modes = np.zeros((B, MAXSEG), np.int32)
    knots = np.zeros((B, MAXSEG), np.int32)
    modes[:, :K] = np.tile(orders, (n_pairs, 1))
    knots[:, :K] = np.asarray(knots_per_seg, np.int32)[None, :]
    nseg = np.full(B, K, np.int32)
    rep = np.repeat(np.arange(n_pairs), n_ord)
    return dict(x0=x0[rep].copy(), goal=goal[rep].copy(), inst=inst[rep].copy(), nseg=nseg, modes=modes,
                knots=knots, pair=rep)


def push_tiny(seed: int = 0, n_pairs: int = 8):
    """8 pairs x 144 two-segment orders, 5+5 intervals (1,152 TOs)."""
    x0, goal, inst = push_pairs(seed, n_pairs)
    return _batch(x0, goal, inst, all_orders(2), (5, 5))


def push_plain(seed: int = 1000, n_pairs: int = 64):
    """64 pairs x 1,728 three-segment orders, 8+8+8 intervals (110,592 TOs)."""
    x0, goal, inst = push_pairs(seed, n_pairs)
    return _batch(x0, goal, inst, all_orders(3), (8, 8, 8))


def push_hetero(seed: int = 2100, B: int = 131072, n_pairs: int = 64, kmin: int = 1, kmax: int = 5,
                nmin: int = 5, nmax: int = 15):
    """B i.i.d. orders of uneven segment and interval counts on n_pairs pairs."""
    rng = np.random.default_rng(seed)
    x0, goal, inst = push_pairs(seed + 1, n_pairs)
    nseg = rng.integers(kmin, kmax + 1, B).astype(np.int32)
    modes = rng.integers(0, PUSH_MODES, (B, MAXSEG)).astype(np.int32)
    knots = rng.integers(nmin, nmax + 1, (B, MAXSEG)).astype(np.int32)
    live = np.arange(MAXSEG)[None, :] < nseg[:, None]
    modes[~live] = 0
    knots[~live] = 0
    pair = rng.integers(0, n_pairs, B)
    return dict(x0=x0[pair].copy(), goal=goal[pair].copy(), inst=inst[pair].copy(), nseg=nseg, modes=modes,
                knots=knots, pair=pair)


def subset(batch: dict, idx) -> dict:
    return {k: v[idx] for k, v in batch.items()}


def n_intervals(batch: dict) -> np.ndarray:
    live = np.arange(MAXSEG)[None, :] < batch["nseg"][:, None]
    return (batch["knots"] * live).sum(1)


# ---------------------------------------------------------------------------------
# Bimanual flipping (box 0.2 x 0.1 m at rest on its long face at the origin)
# ---------------------------------------------------------------------------------
FLIP_MODES = 845         # id = (f1 * 13 + f2) * 5 + g
FLIP_X0 = (0.0, 0.05, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0)


def flip_pairs(seed: int, n: int):
    """n start/goal pairs: x0 [n,8] at rest, goal [n,2] = (px ~ U[-0.2, 0.2] m,
    th ~ U[pi/2, pi]), inst [n,1] = table friction ~ U[0.62, 0.78]."""
    rng = np.random.default_rng(seed)
    goal = np.empty((n, 2))
    goal[:, 0] = rng.uniform(-0.2, 0.2, n)
    goal[:, 1] = rng.uniform(np.pi / 2, np.pi, n)
    mu = rng.uniform(0.62, 0.78, n)
    x0 = np.tile(np.array(FLIP_X0), (n, 1))
    return x0, goal, mu.reshape(n, 1)


def flip_pivot_pairs(seed: int, n: int, th_lo: float = 0.9, th_hi: float = 1.5):
    """n start/goal pairs whose goal a pivot about the bottom-left corner of the resting box
    reaches: th ~ U[th_lo, th_hi], px the centre's displacement under that rotation, table
    friction ~ U[0.62, 0.78]."""
    rng = np.random.default_rng(seed)
    th = rng.uniform(th_lo, th_hi, n)
    cx, cy = -0.1, -0.05                     # corner relative to the centre (box 0.2 x 0.1 m)
    px = -0.1 - (np.cos(th) * cx - np.sin(th) * cy)
    mu = rng.uniform(0.62, 0.78, n)
    return np.tile(np.array(FLIP_X0), (n, 1)), np.stack([px, th], 1), mu.reshape(n, 1)


def flip_orders(rng, B: int, kmin: int, kmax: int):
    """B i.i.d. flip orders: K ~ U{kmin..kmax}, finger codes ~ U{0..12}, table mode ~
    U{0..4}, except that a pivot directly after a pivot keeps its direction (an order
    whose pivot run changes corner is not a valid problem)."""
    K = rng.integers(kmin, kmax + 1, B)
    f1 = rng.integers(0, 13, (B, MAXSEG))
    f2 = rng.integers(0, 13, (B, MAXSEG))
    g = rng.integers(0, 5, (B, MAXSEG))
    for j in range(1, MAXSEG):
        run = (g[:, j] >= 3) & (g[:, j - 1] >= 3)
        g[run, j] = g[run, j - 1]
    modes = ((f1 * 13 + f2) * 5 + g).astype(np.int32)
    modes[np.arange(MAXSEG)[None, :] >= K[:, None]] = 0
    return K.astype(np.int32), modes


def flip_batch(seed: int, B: int, n_pairs: int = 32, kmin: int = 1, kmax: int = 6, knots: int = 10) -> dict:
    """Ragged flipping batch: B orders spread over n_pairs start/goal pairs, `knots`
    intervals per segment."""
    rng = np.random.default_rng(seed)
    x0, goal, inst = flip_pairs(seed + 1, n_pairs)
    pair = rng.integers(0, n_pairs, B)
    nseg, modes = flip_orders(rng, B, kmin, kmax)
    kn = np.where(np.arange(MAXSEG)[None, :] < nseg[:, None], knots, 0).astype(np.int32)
    return dict(x0=x0[pair], goal=goal[pair], inst=inst[pair], nseg=nseg, modes=modes, knots=kn)


# free-motion pushing: pusher start positions 3 cm in front of face j (slider frame)
_FREE_START = 0.08 * np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])


def push_free_pairs(seed: int, n: int):
    """n start/goal pairs of free-motion pushing: x0 [n, 5] (slider at rest at the origin,
    pusher 3 cm in front of a face drawn uniformly), goal [n, 3] (x, y ~ U[-0.15, 0.15] m,
    theta ~ U[-pi/2, pi/2]), inst [n, 1] (pusher friction ~ U[0.3, 0.5])."""
    rng = np.random.default_rng(seed)
    goal = np.empty((n, 3))
    goal[:, 0] = rng.uniform(-0.15, 0.15, n)
    goal[:, 1] = rng.uniform(-0.15, 0.15, n)
    goal[:, 2] = rng.uniform(-np.pi / 2, np.pi / 2, n)
    mu = rng.uniform(0.3, 0.5, n)
    face = rng.integers(0, 4, n)
    x0 = np.zeros((n, 5))
    x0[:, 3:] = _FREE_START[face]
    return x0, goal, mu.reshape(n, 1)


def orders_batch(x0, goal, inst, pair, orders, knots) -> dict:
    """Sequences given one by one: pair [B] indexes x0/goal/inst, orders / knots are lists
    of B lists (segment ids, intervals per segment)."""
    B = len(orders)
    modes = np.zeros((B, MAXSEG), np.int32)
    kn = np.zeros((B, MAXSEG), np.int32)
    nseg = np.zeros(B, np.int32)
    for i, (o, k) in enumerate(zip(orders, knots)):
        nseg[i] = len(o)
        modes[i, :len(o)] = o
        kn[i, :len(k)] = k
    pair = np.asarray(pair)
    return dict(x0=x0[pair].copy(), goal=goal[pair].copy(), inst=inst[pair].copy(), nseg=nseg, modes=modes,
                knots=kn, pair=pair)


def flip_tiny(seed: int = 3000, B: int = 512) -> dict:
    """Small flipping batch for parity: K ~ U{1..3}, 5 intervals per segment."""
    return flip_batch(seed, B, n_pairs=8, kmin=1, kmax=3, knots=5)
