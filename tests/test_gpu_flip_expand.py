"""GPU parity of the device expansion (Alg. 1) over the flip language against the flip
oracle: bit-exact batch construction on identical (key, merit) inputs, the filtered seed,
and a whole small expansion whose returned plan the oracle confirms."""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def _ctx(max_batch=4096, max_intervals=30):
    from paper_2609_21803_amd import native
    return native.Context(max_batch=max_batch, max_segments=6, max_intervals=max_intervals, task=native.TASK_FLIP)


def _random_V(rng, n, kcap):
    from oracle import flip as F
    ones = [F.key_modes(int(k))[0] for k in F.seed(1)]
    keys = set()
    while len(keys) < n:
        K = int(rng.integers(1, kcap + 1))
        m = [ones[int(rng.integers(len(ones)))] for _ in range(K)]
        if F.admissible(m):
            keys.add(F.key_make(m))
    keys = np.array(sorted(keys), np.uint64)
    rng.shuffle(keys)
    merit = rng.choice([0.1, 0.5, 1.0, np.inf, np.nan], size=n) + np.where(rng.random(n) < 0.5, 0.0, rng.random(n))
    return keys, merit


@pytest.mark.parametrize("radius,kcap,n,W,room", [(1, 2, 40, 4096, 3000), (1, 3, 300, 16, 20000), (1, 4, 20, 2, 5000),
                                                 (2, 2, 3, 2, 4000), (1, 2, 1, 1, 7)])
def test_flip_batch_construction_is_bit_exact(radius, kcap, n, W, room):
    import torch
    from oracle import flip as F
    from paper_2609_21803_amd import native
    rng = np.random.default_rng(10 * radius + n)
    keys, merit = _random_V(rng, n, kcap)
    ref = F.expand_next(keys, merit, kcap, radius, W, room)
    ctx = _ctx(max_batch=max(room, 8))
    prm = native.ExpandParams(kcap=kcap, radius=radius, frontier_W=W, batch_B=room, eval_budget=max(n, 1),
                              knots_per_segment=5, rounds=1, k_ref=1, seed_max_segments=1)
    got = native.expand_next(ctx, torch.as_tensor(keys.view(np.int64)).cuda(), torch.as_tensor(merit).cuda(), prm,
                             room)
    got = got.cpu().numpy().view(np.uint64)
    assert len(got) == len(ref) and np.array_equal(got, ref), (len(got), len(ref))


def test_flip_expansion_seed_rounds_and_plan_match_oracle():
    """One instance with a reachable pivot goal: the device evaluates the filtered seed in
    key order, builds its next batch from the same language, and returns a plan that the
    oracle re-solves to the same cost; the oracle's own expansion finds a plan as well."""
    import torch
    from oracle import flip as F
    from paper_2609_21803_amd import native
    import oracle
    th = 1.2
    c = np.array([-0.1, -0.05])
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    goal = np.array([-0.1 - (R @ c)[0], th])
    x0 = np.array(I.FLIP_X0)
    ep = dict(kcap=2, seed_max_segments=1, radius=1, rounds=1, frontier_W=8, knots_per_segment=10, k_ref=16,
              batch_B=2048, eval_budget=2400)
    ctx = _ctx(max_batch=2048, max_intervals=20)
    prm = native.ExpandParams(**ep)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    o, st = native.expand(ctx, t(x0), t(goal), t([0.7]), prm)
    torch.cuda.synchronize()
    keys, J, v = native.expand_trace(ctx)
    keys = keys.cpu().numpy().view(np.uint64)
    seed = F.seed(1)
    assert np.array_equal(keys[:len(seed)], seed)
    print("device: evaluated", st["evaluated"], "feasible", st["n_feasible"], "first", st["first_feasible_index"],
          "plan", o["modes"].cpu().numpy()[:int(o["nseg"].item())], float(o["cost"].item()))
    e = oracle.Expand()
    for k, val in ep.items():
        setattr(e, k, val)
    bk, bJ, bv, cnt, ek, eJ, ev = F.expand(x0, goal, 0.7, e)
    print("oracle: evaluated", cnt[0], "feasible", cnt[2], "first", cnt[3], "plan", F.key_modes(int(bk)), bJ)
    assert st["evaluated"] == cnt[0]
    assert np.array_equal(keys[:len(seed)], ek[:len(seed)])
    # every device merit of the seed round agrees with the oracle's evaluation
    scale = np.maximum(np.abs(eJ[:len(seed)]), 1e-3)
    assert (np.abs(J.cpu().numpy()[:len(seed)] - eJ[:len(seed)]) <= 1e-4 * scale).mean() >= 0.95
    K = int(o["nseg"].item())
    assert K >= 1 and bk != 0
    m = o["modes"].cpu().numpy()[:K]
    r = F.evaluate(x0[None], goal[None], np.array([0.7]), np.array([K]), np.array([list(m) + [0] * (6 - K)]),
                   np.array([[10] * K + [0] * (6 - K)]), params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"].item())) <= 1e-4 * abs(r["cost"][0])
    if F.key_modes(int(bk)) != list(m):
        assert abs(bJ - float(o["cost"].item())) <= 1e-3 * abs(bJ)   # a tie within the margin


def test_configured_flip_expansion_at_scale():
    """The flipping expansion at its configured scale: goals th ~ U[pi/2, pi], px ~ U[-0.2,
    0.2] m (the configured range), orders of up to six segments, 10 intervals per segment,
    32,768 orders per round, an evaluation budget of 200,000, frontier W = 4,096.  Every
    batch the device admitted equals the flip oracle's batch-construction step on the
    device's own (key, Eq. (5) merit) of everything evaluated before it; a returned plan (if
    any: none is a result too) is re-solved by the flip oracle at the refinement budget to
    the same cost.  Prints plans found, evaluations and time per round."""
    import time
    import torch
    import oracle
    from oracle import flip as F
    from paper_2609_21803_amd import native
    B, W = 32768, 4096
    x0s, goals, insts = I.flip_pairs(3000, 1)
    ep = dict(kcap=6, seed_max_segments=1, radius=1, rounds=6, frontier_W=W, knots_per_segment=10, k_ref=16,
              batch_B=B, eval_budget=200000)
    ctx = _ctx(max_batch=B, max_intervals=60)
    prm = native.ExpandParams(**ep)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    t0 = time.time()
    o, st = native.expand(ctx, t(x0s[0]), t(goals[0]), t(insts[0]), prm)
    torch.cuda.synchronize()
    wall = time.time() - t0
    keys, J, v = [a.cpu().numpy() for a in native.expand_trace(ctx)]
    keys = keys.view(np.uint64)
    merit = np.array([oracle.merit(a, b) for a, b in zip(J, v)])
    seed = F.seed(1)
    assert np.array_equal(keys[:len(seed)], seed)
    pos, sizes = len(seed), [len(seed)]
    while pos < len(keys):
        nxt = F.expand_next(keys[:pos], merit[:pos], 6, 1, W, min(B, 200000 - pos))
        assert len(nxt) > 0 and np.array_equal(keys[pos:pos + len(nxt)], nxt), (pos, len(nxt))
        pos += len(nxt)
        sizes.append(len(nxt))
    K = int(o["nseg"].item())
    print(f"flip at scale: goal {goals[0]}, batches {sizes}, evaluated {st['evaluated']}, feasible "
          f"{st['n_feasible']}, plan {o['modes'].cpu().numpy()[:K]} cost {float(o['cost'].item()):.5f}, device "
          f"{st['t_total_ms']:.0f} ms ({st['t_total_ms'] / max(1, st['rounds_done']):.0f} ms per round), wall "
          f"{wall:.1f} s", flush=True)
    assert st["evaluated"] == len(keys) <= 200000 and max(sizes) <= B
    if K >= 1:
        m = o["modes"].cpu().numpy()[:K]
        f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
        r = F.evaluate(f32(x0s[:1]), f32(goals[:1]), f32(insts[:1]), np.array([K]), np.array([list(m) + [0] * (6 - K)]),
                       np.array([[10] * K + [0] * (6 - K)]), params=oracle.Params(**oracle.REFINE))
        assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"].item())) <= 1e-4 * abs(r["cost"][0])
    else:
        assert st["n_feasible"] == 0 or st["n_refined"] > 0
