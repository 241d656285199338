"""Oracle of the uniform-sampling allocation policy (the baseline of Sec. IV-B that draws
complete admissible orders uniformly without replacement), over the evaluator oracles.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading of "uniformly without replacement" (the paper gives no procedure): each round makes
a fixed number of draws from one SplitMix64 stream (Steele, Lea and Flood, OOPSLA 2014; the
generator of Java's SplittableRandom), draw c taking outputs 8c .. 8c+6: the segment count
K = 1 + out(8c) mod kcap, then id j = out(8c+1+j) mod M.  Draws outside the task's
language, already evaluated, or repeating an earlier draw of the round are dropped, and
the round's batch is the first `room` remaining draws in draw order.  Each segment count is
equally likely and, given the count, every admissible order (rejection sampling).  For
pushing with free motion, whose admissible orders of eight segments are 1 in 28,500 of the
product space, draw c instead takes t = out(8c+1) mod (number of admissible orders of K
segments) and the t-th of them in key order: uniform over that count without rejection.
The search then evaluates batch after batch up to the budget and refines like the
expansion.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15


def splitmix64(seed: int, i: int) -> int:
    """Output i (0-based) of the SplitMix64 stream whose state starts at `seed`."""
    z = (seed + (i + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def splitmix64_array(seed: int, idx: np.ndarray) -> np.ndarray:
    """splitmix64 over an array of output indices (uint64 arithmetic wraps mod 2^64)."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + (idx.astype(np.uint64) + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def key_make(modes) -> int:
    k = len(modes) << 60
    for i, m in enumerate(modes):
        k |= int(m) << (50 - 10 * i)
    return k


def key_modes(k: int):
    return [(k >> (50 - 10 * i)) & 1023 for i in range(k >> 60)]


def draws(seed: int, first: int, n: int, kcap: int, n_modes: int):
    """The orders of draws first .. first+n-1 (lists of mode ids)."""
    c = np.arange(first, first + n, dtype=np.uint64)
    K = 1 + (splitmix64_array(seed, c * np.uint64(8)) % np.uint64(kcap)).astype(np.int64)
    ids = np.stack([(splitmix64_array(seed, c * np.uint64(8) + np.uint64(1 + j)) % np.uint64(n_modes)).astype(np.int64)
                    for j in range(kcap)], 1)
    return [list(ids[i, :K[i]]) for i in range(n)]


def free_counts():
    """c[r][a] = number of id sequences of length r allowed after id a (c[0][a] = 1), from
    the free-motion oracle's admissibility of two-segment orders."""
    from . import free as F
    step = [[F.admissible([a, b]) for b in range(16)] for a in range(16)]
    c = [[1] * 16]
    for r in range(1, 8):
        c.append([sum(c[r - 1][b] for b in range(16) if step[a][b]) for a in range(16)])
    return c, step


def free_unrank(K: int, t: int, counts=None):
    """The t-th (from 0) admissible free-motion order of K segments in key order."""
    c, step = counts or free_counts()
    out, prev = [], None
    for d in range(K):
        rest = K - 1 - d
        for b in range(16):
            if prev is not None and not step[prev][b]:
                continue
            if t < c[rest][b]:
                out.append(b)
                break
            t -= c[rest][b]
        prev = out[-1]
    return out


def free_draws(seed: int, first: int, n: int, kcap: int):
    """The orders of draws first .. first+n-1 of the free-motion task (unranked)."""
    counts = free_counts()
    c = np.arange(first, first + n, dtype=np.uint64)
    K = 1 + (splitmix64_array(seed, c * np.uint64(8)) % np.uint64(kcap)).astype(np.int64)
    u = splitmix64_array(seed, c * np.uint64(8) + np.uint64(1))
    tot = [0] + [sum(counts[0][k - 1][a] for a in range(16)) for k in range(1, 9)]   # orders of exactly K segments
    return [free_unrank(int(K[i]), int(u[i] % np.uint64(tot[int(K[i])])), counts) for i in range(n)]


def sample_round(task: int, seed: int, first: int, n_draws: int, kcap: int, seen: set, room: int):
    """One round's batch: the first `room` draws that are in the language, unseen and not
    repeated earlier in the round, in draw order (keys)."""
    if task == 3:
        from . import free as F
        out, round_seen = [], set()
        for m in free_draws(seed, first, n_draws, kcap):
            if len(out) >= room:
                break
            k = F.key_make(m)
            if k in seen or k in round_seen:
                continue
            round_seen.add(k)
            out.append(k)
        return out
    if task == 1:
        from . import flip as F
        admissible, n_modes = F.admissible, 845
    else:
        admissible, n_modes = (lambda m: True), 12
    out, round_seen = [], set()
    for m in draws(seed, first, n_draws, kcap, n_modes):
        if len(out) >= room:
            break
        k = key_make(m)
        if k in seen or k in round_seen or not admissible(m):
            continue
        round_seen.add(k)
        out.append(k)
    return out


def _evaluate(task, keys, x0, goal, inst, knots_per_segment, params):
    B = len(keys)
    nseg = np.array([k >> 60 for k in keys], np.int32)
    S = 8 if task == 3 else 6
    modes = np.zeros((B, S), np.int32)
    knots = np.zeros((B, S), np.int32)
    if task == 3:
        from . import free as F
    for b, k in enumerate(keys):
        m = F.key_modes(k) if task == 3 else key_modes(k)
        modes[b, :len(m)] = m
        knots[b, :len(m)] = knots_per_segment
    X0 = np.tile(np.asarray(x0, np.float64), (B, 1))
    G = np.tile(np.asarray(goal, np.float64), (B, 1))
    Iv = np.tile(np.asarray(inst, np.float64).reshape(1, -1), (B, 1))
    nmax = int(max(1, knots.sum(1).max(initial=1)))
    if task == 1:
        from . import flip as F
        r = F.evaluate(X0, G, Iv, nseg, modes, knots, params=params, nmax=nmax)
    elif task == 3:
        r = F.evaluate(X0, G, Iv, nseg, modes, knots, params=params, nmax=nmax)
    else:
        import oracle
        r = oracle.evaluate(X0, G, Iv, nseg, modes, knots, params=params, nmax=nmax)
    return r["cost"], r["viol"]


def uniform_search(task, x0, goal, inst, kcap, rounds, batch_B, eval_budget, n_draws, seed, knots_per_segment, k_ref,
                   params=None, ref_params=None):
    """Rounds 0..rounds of sampled batches up to the budget, then refinement of the k_ref
    best feasible orders by (J, key); returns (best key or 0, refined J, refined v, evaluated
    keys, their J, v)."""
    import oracle
    params = params or oracle.Params()
    ref_params = ref_params or oracle.Params(**{**params.__dict__, **oracle.REFINE})
    keys, Js, vs = [], [], []
    seen = set()
    for s in range(rounds + 1):
        room = min(batch_B, eval_budget - len(keys))
        if room <= 0:
            break
        batch = sample_round(task, seed, s * n_draws, n_draws, kcap, seen, room)
        if not batch:
            continue
        seen.update(batch)
        J, v = _evaluate(task, batch, x0, goal, inst, knots_per_segment, params)
        keys += batch
        Js += list(J)
        vs += list(v)
    eps = params.eps_feas
    feas = [(Js[i], keys[i]) for i in range(len(keys)) if vs[i] <= eps and np.isfinite(Js[i])]
    feas.sort()
    ref = [k for _, k in feas[:k_ref]]
    best = (0, np.nan, np.inf)
    if ref:
        J, v = _evaluate(task, ref, x0, goal, inst, knots_per_segment, ref_params)
        for k, Jr, vr in zip(ref, J, v):
            if vr <= ref_params.eps_feas and np.isfinite(Jr):
                if best[0] == 0 or Jr < best[1] or (Jr == best[1] and k < best[0]):
                    best = (k, Jr, vr)
    return best[0], best[1], best[2], keys, np.array(Js), np.array(vs)
