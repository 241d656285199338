"""GPU parity of free-motion pushing (COMET_TASK_PUSH_FREE: the admissible language of Sec.
III-A, with the pusher position in the state and non-penetration rows) against the FP64
free-motion oracle, called through the C ABI.

* Evaluation, sequence by sequence with the rule of tests/parity.py (margin sequences agree
  on the feasible flag, and on cost within 1e-4 and violation within 1e-5 where both are
  feasible; a disagreement is excused only where the oracle itself moves under float32-level
  perturbations), on every admissible order of at most two segments and on a ragged batch
  of admissible orders of up to four segments, and on a strided sample of the benchmark's
  launch (every admissible order of at most six segments on 8 instances).
* The closed form of a free approach followed by a straight push.
* The device expansion over this language: bit-exact batch construction against the
  oracle's batch step, and a whole expansion whose evaluated orders are all admissible and
  whose returned plan the oracle confirms.
Inputs are rounded to float32 before they reach the oracle.
"""
import numpy as np
import pytest

import parity
from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu

# what the device keeps in float32, as the oracle's rounding switch for the excuse draws:
# step (1), multipliers (2), scaled Jacobians (4), gains with the forward recursion (8)
ROUND32 = 1 | 2 | 4 | 8


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def run_gpu(batch, max_intervals):
    import torch
    from paper_2609_21803_amd import native
    B = len(batch["nseg"])
    ctx = native.Context(max_batch=max(B, 1), max_segments=6, max_intervals=max_intervals,
                         task=native.TASK_PUSH_FREE)
    out = ctx.evaluate(**native.to_device(batch))
    torch.cuda.synchronize()
    ctx.check()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def run_oracle(batch, nmax, params=None):
    import oracle
    from oracle import free as F
    return F.evaluate(f32(batch["x0"]), f32(batch["goal"]), f32(batch["inst"]), batch["nseg"], batch["modes"],
                      batch["knots"], params=params or oracle.Params(), nmax=nmax)


def compare(g, o, batch, label, nmax):
    import oracle

    def solve(sub, rows, r32):
        return run_oracle(sub, nmax, oracle.Params(round32=r32))
    parity.check(g, o, batch, solve, label, round32=ROUND32)


def _orders(kmax):
    from oracle import free as F
    return [F.key_modes(int(k)) for k in F.seed(kmax)]


def test_all_short_orders_match_oracle():
    """8 instances x all 72 admissible orders of one and two segments, 10 intervals each."""
    x0, goal, inst = I.push_free_pairs(5000, 8)
    orders = _orders(2)
    pair = np.repeat(np.arange(8), len(orders))
    b = I.orders_batch(x0, goal, inst, pair, orders * 8, [[10] * len(o) for o in orders] * 8)
    g = run_gpu(b, 20)
    o = run_oracle(b, 20)
    print("feasible oracle / device:", int(o["feasible"].sum()), int(g["feasible"].sum()))
    assert o["feasible"].sum() >= 8
    compare(g, o, b, "free <= 2 segments", 20)


def test_ragged_orders_match_oracle():
    """1,024 admissible orders of 1..4 segments drawn uniformly, 4..10 intervals per segment,
    on 16 instances."""
    rng = np.random.default_rng(5100)
    x0, goal, inst = I.push_free_pairs(5101, 16)
    pool = _orders(4)
    pick = rng.integers(0, len(pool), 1024)
    orders = [pool[i] for i in pick]
    knots = [list(rng.integers(4, 11, len(o))) for o in orders]
    b = I.orders_batch(x0, goal, inst, rng.integers(0, 16, 1024), orders, knots)
    g = run_gpu(b, 40)
    o = run_oracle(b, 40)
    print("feasible oracle / device:", int(o["feasible"].sum()), int(g["feasible"].sum()))
    compare(g, o, b, "free ragged", 40)


def test_free_full_size_workload_sampled():
    """Every admissible order of at most six segments (14,760) on 8 instances, 10 intervals per
    segment (118,080 TOs, up to 60 intervals) in one launch, as the benchmark times it;
    1,024 evenly strided sequences checked against the oracle one by one."""
    from oracle import free as F
    orders = [F.key_modes(int(k)) for k in F.seed(6)]
    assert len(orders) == 14760
    x0, goal, inst = I.push_free_pairs(5400, 8)
    pair = np.repeat(np.arange(8), len(orders))
    b = I.orders_batch(x0, goal, inst, pair, orders * 8, [[10] * len(o) for o in orders] * 8)
    g = run_gpu(b, 60)
    idx = np.linspace(0, len(b["nseg"]) - 1, 1024).astype(np.int64)
    sub = I.subset(b, idx)
    o = run_oracle(sub, 60)
    print("feasible in the launch:", int(g["feasible"].sum()), "sampled oracle / device:", int(o["feasible"].sum()),
          int(g["feasible"][idx].sum()))
    compare({k: v[idx] for k, v in g.items()}, o, sub, "free full size (1,024 strided)", 60)


def test_free_approach_then_straight_push_on_gpu():
    """Pusher 3 cm in front of face 2, goal (d, 0, 0), order [free in front of face 2, stick
    on face 2]: J* = 0.03^2 / (N1 dt) + d^2 / (N2 dt) (see the oracle's pins), reached within
    1e-3 at the exploration budget; the pusher arrives at the face centre."""
    from oracle import free as F
    cases = [(0.05, 6, 10), (0.12, 10, 12), (0.02, 4, 6)]
    x0 = np.tile([0.0, 0.0, 0.0, -0.08, 0.0], (len(cases), 1))
    goal = np.array([[d, 0.0, 0.0] for d, _, _ in cases])
    b = I.orders_batch(x0, goal, np.full((len(cases), 1), 0.4), np.arange(len(cases)),
                       [[F.free(2), F.contact(2, 0)]] * len(cases), [[n1, n2] for _, n1, n2 in cases])
    g = run_gpu(b, 24)
    for i, (d, n1, n2) in enumerate(cases):
        Jstar = 0.03 ** 2 / (n1 * 0.1) + d ** 2 / (n2 * 0.1)
        assert g["feasible"][i] == 1 and abs(g["cost"][i] - Jstar) <= 1e-3 * Jstar, (i, g["cost"][i], Jstar)
        assert np.allclose(g["traj"][i, n1, 3:5], [-0.05, 0.0], atol=1e-4)


def _ctx(max_batch=4096, max_intervals=40, max_segments=6):
    from paper_2609_21803_amd import native
    return native.Context(max_batch=max_batch, max_segments=max_segments, max_intervals=max_intervals,
                          task=native.TASK_PUSH_FREE)


@pytest.mark.parametrize("radius,kcap,n,W,room", [(1, 3, 40, 4096, 3000), (2, 3, 30, 8, 20000), (1, 6, 300, 64, 5000),
                                                 (2, 4, 5, 3, 4000), (1, 2, 1, 1, 7), (2, 8, 60, 16, 30000),
                                                 (1, 8, 500, 500, 60000)])
def test_free_batch_construction_is_bit_exact(radius, kcap, n, W, room):
    import torch
    from oracle import free as F
    from paper_2609_21803_amd import native
    rng = np.random.default_rng(20 * radius + n)
    pool = [int(k) for k in F.seed(min(kcap, 4))] if kcap < 8 else [int(k) for k in F.seed(8)[::97]]
    keys = np.array([pool[i] for i in rng.choice(len(pool), n, replace=False)], np.uint64)
    merit = rng.choice([0.1, 0.5, 1.0, np.inf, np.nan], size=n) + np.where(rng.random(n) < 0.5, 0.0, rng.random(n))
    ref = F.expand_next(keys, merit, kcap, radius, W, room)
    ctx = _ctx(max_batch=max(room, 8), max_segments=max(kcap, 6))
    prm = native.ExpandParams(kcap=kcap, radius=radius, frontier_W=W, batch_B=room, eval_budget=max(n, 1),
                              knots_per_segment=5, rounds=1, k_ref=1, seed_max_segments=1)
    got = native.expand_next(ctx, torch.as_tensor(keys.view(np.int64)).cuda(), torch.as_tensor(merit).cuda(), prm,
                             room)
    got = got.cpu().numpy().view(np.uint64)
    assert len(got) == len(ref) and np.array_equal(got, ref), (len(got), len(ref))


@pytest.mark.parametrize("seed", [5200, 5201])
def test_free_expansion_stays_in_the_language_and_its_plan_is_confirmed(seed):
    """Seed = every admissible order of at most two segments (72, in key order), two rounds of
    one-edit neighbourhoods; every evaluated order is admissible, the first batch is the seed,
    and the returned plan is feasible and re-solved by the oracle (refinement budget) to the
    same cost within 1e-3."""
    import torch
    import oracle
    from oracle import free as F
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(seed, 1)
    prm = native.ExpandParams(kcap=4, seed_max_segments=2, radius=1, rounds=2, frontier_W=64, knots_per_segment=10,
                              k_ref=16, batch_B=4096, eval_budget=20000)
    ctx = _ctx(max_batch=4096, max_intervals=40)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
    torch.cuda.synchronize()
    o = {k: v.cpu().numpy() for k, v in o.items()}
    keys, J, v = native.expand_trace(ctx)
    keys = [int(k) for k in keys.cpu().numpy().view(np.uint64)]
    seedk = [int(k) for k in F.seed(2)]
    K = int(o["nseg"][0])
    print("evaluated", len(keys), "feasible", int((v.cpu().numpy() <= 1e-5).sum()), "plan", list(o["modes"][:K]),
          "cost", float(o["cost"][0]), flush=True)
    assert keys[:len(seedk)] == seedk
    assert all(F.admissible(F.key_modes(k)) for k in keys)
    assert len(set(keys)) == len(keys)
    assert K >= 1 and float(o["viol"][0]) <= 1e-5
    modes = np.zeros((1, 6), np.int32)
    knots = np.zeros((1, 6), np.int32)
    modes[0, :K] = o["modes"][:K]
    knots[0, :K] = o["knots"][:K]
    assert F.admissible(list(modes[0, :K]))
    r = F.evaluate(f32(x0), f32(goal), f32(inst), np.array([K]), modes, knots,
                   params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"][0])) <= 1e-3 * abs(r["cost"][0]), \
        (r["cost"][0], float(o["cost"][0]))


def test_free_invalid_sequences_empty_batch_and_network_hooks():
    """Invalid orders (an id outside the 16 of this task, no segment, a non-finite pusher
    position or goal, more intervals than the context holds) come back with NaN cost, +inf
    violation and status 3 and raise the device error counter; the valid orders beside them
    are solved.  An empty batch is a no-op; the learned network does not serve this task."""
    import torch
    from oracle import free as F
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(5500, 8)
    orders = [[F.free(3), F.contact(3, 0)]] * 8
    b = I.orders_batch(x0, goal, inst, np.arange(8), orders, [[5, 5]] * 8)
    b["modes"][1, 1] = 16            # outside the 16 ids
    b["nseg"][2] = 0                 # no segment
    b["x0"][3, 4] = np.nan           # pusher position not finite
    b["goal"][4, 2] = np.inf         # goal not finite
    b["knots"][5, 1] = 40            # 45 intervals > 20
    ctx = _ctx(max_batch=8, max_intervals=20)
    out = ctx.evaluate(**native.to_device(b))
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    for i in (1, 2, 3, 4, 5):
        assert np.isnan(g["cost"][i]) and np.isinf(g["viol"][i]) and g["feasible"][i] == 0, i
        assert g["stats"][i, 3] == 3, i
    assert np.all(np.isfinite(g["cost"][[0, 6, 7]]))
    with pytest.raises(native.CometError):
        ctx.check()
    ctx.check()                      # the counter was cleared
    e = {k: v[:0] for k, v in native.to_device(b).items()}
    assert ctx.evaluate(**e)["cost"].numel() == 0


def test_free_maximum_length_orders_match_oracle():
    """Orders at the longest work-space height (510 of 512 intervals): a free approach of
    255 intervals then a straight push of 255, whose optimum is 0.03^2 / (N1 dt) + d^2 /
    (N2 dt), and three admissible six-segment orders of 85 intervals per segment.  Where
    both sides converge the flags agree and the costs agree within 1e-3 (the stopping
    region is wide over 510 stages, as for the pushing tasks); the straight push converges
    on both sides and reaches its closed form within 5e-3; trajectory rows past the last
    knot stay zero."""
    import oracle
    from oracle import free as F
    x0 = np.array([[0.0, 0.0, 0.0, -0.08, 0.0]] * 4)
    goal = np.array([[0.1, 0.0, 0.0], [0.05, 0.05, 0.3], [-0.05, 0.08, -0.4], [0.08, -0.03, 0.5]])
    six = [[14, 6, 14, 15, 9, 15], [14, 6, 7, 14, 13, 4], [14, 8, 14, 15, 12, 1]]
    assert all(F.admissible(o) for o in six)
    orders = [[F.free(2), F.contact(2, 0)]] + six
    knots = [[255, 255]] + [[85] * 6] * 3
    b = I.orders_batch(x0, goal, np.full((4, 1), 0.4), np.arange(4), orders, knots)
    g = run_gpu(b, 512)
    o = run_oracle(b, 512)
    conv = (g["stats"][:, 3] == 1) & (o["stats"][:, 3] == 1)
    rel = np.abs(g["cost"].astype(np.float64) - o["cost"]) / np.maximum(np.abs(o["cost"]), 1e-12)
    print("statuses gpu / oracle:", g["stats"][:, 3], o["stats"][:, 3], "feasible:", g["feasible"], o["feasible"],
          "rel cost:", rel, flush=True)
    assert conv[0]
    Jstar = 0.03 ** 2 / (255 * 0.1) + 0.1 ** 2 / (255 * 0.1)
    assert abs(g["cost"][0] - Jstar) <= 5e-3 * Jstar and abs(o["cost"][0] - Jstar) <= 5e-3 * Jstar
    assert np.all(g["feasible"][conv] == o["feasible"][conv]) and np.all(rel[conv] <= 1e-3)
    assert np.all(g["traj"][:, 511:] == 0) and np.all(g["traj"][:, 510, 5:] == 0)


def test_free_seed_of_eight_segments_is_the_whole_language():
    """Full enumeration at the segment cap of eight (Sec. IV-A): the seed pass of an
    expansion with s = 8 and no further round evaluates exactly the oracle's admissible
    orders of 1..8 segments (205,632), in key order; the order of every evaluated key's
    batch row is the key's own (segment count, ids, two intervals per segment)."""
    import torch
    from oracle import free as F
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(5600, 1)
    ref = F.seed(8)
    assert len(ref) == 205632
    prm = native.ExpandParams(kcap=8, seed_max_segments=8, radius=1, rounds=0, frontier_W=1, knots_per_segment=2,
                              k_ref=1, batch_B=len(ref), eval_budget=len(ref))
    ctx = _ctx(max_batch=len(ref), max_intervals=16, max_segments=8)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
    torch.cuda.synchronize()
    keys = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
    print("evaluated", st["evaluated"], "feasible", st["n_feasible"], "plan", o["modes"].cpu().numpy()[:int(o["nseg"])],
          flush=True)
    assert st["evaluated"] == len(ref) and np.array_equal(keys, ref)
    K = int(o["nseg"].item())
    if K:
        assert F.admissible(list(o["modes"].cpu().numpy()[:K])) and np.all(o["knots"].cpu().numpy()[:K] == 2)


@pytest.mark.parametrize("policy", ["uniform", "mcts"])
def test_free_sampling_and_mcts_stay_in_the_eight_segment_language(policy):
    """The ablation policies over the free-motion evaluator at the segment cap of eight:
    every evaluated order is admissible and distinct, at most the budget is spent, and the
    returned plan is admissible, feasible and re-solved by the oracle to the same cost."""
    import torch
    import oracle
    from oracle import free as F
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(5700, 1)
    pol = native.POLICY_UNIFORM if policy == "uniform" else native.POLICY_MCTS
    prm = native.ExpandParams(kcap=8, seed_max_segments=2, radius=1, rounds=3, frontier_W=64, knots_per_segment=6,
                              k_ref=16, batch_B=1024, eval_budget=3072, policy=pol, sample_seed=17, sample_draws=8192)
    ctx = _ctx(max_batch=1024, max_intervals=48, max_segments=8)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
    torch.cuda.synchronize()
    keys = [int(k) for k in native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)]
    K = int(o["nseg"].item())
    print(policy, "evaluated", len(keys), "feasible", st["n_feasible"], "lengths",
          np.bincount([k >> 60 for k in keys], minlength=9)[1:], "plan", list(o["modes"].cpu().numpy()[:K]),
          float(o["cost"].item()), flush=True)
    assert 0 < len(keys) <= 3072 and len(set(keys)) == len(keys)
    assert all(F.admissible(F.key_modes(k)) for k in keys)
    assert K >= 1 and float(o["viol"][0]) <= 1e-5
    modes = np.zeros((1, 8), np.int32)
    knots = np.zeros((1, 8), np.int32)
    modes[0, :K] = o["modes"].cpu().numpy()[:K]
    knots[0, :K] = o["knots"].cpu().numpy()[:K]
    assert F.admissible(list(modes[0, :K]))
    r = F.evaluate(f32(x0), f32(goal), f32(inst), np.array([K]), modes, knots, params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"][0])) <= 1e-3 * abs(r["cost"][0])


def test_free_uniform_sampling_batches_are_the_oracles():
    """Uniform sampling over the free-motion language at the segment cap of eight: each draw
    picks a segment count, then the index of an admissible order of that count (unranked),
    so long orders are drawn as often as short ones; the evaluated orders equal the oracle's
    draws bit for bit, and the returned plan is confirmed by the oracle's refinement."""
    import torch
    import oracle
    from oracle import free as F
    from oracle import sample as S
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(5800, 1)
    ep = dict(kcap=8, rounds=2, knots_per_segment=5, k_ref=16, batch_B=512, eval_budget=1280)
    prm = native.ExpandParams(**ep, policy=native.POLICY_UNIFORM, sample_seed=23, sample_draws=1024)
    ctx = _ctx(max_batch=512, max_intervals=40, max_segments=8)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
    torch.cuda.synchronize()
    keys = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
    bk, bJ, bv, okeys, J, v = S.uniform_search(3, f32(x0[0]), f32(goal[0]), f32(inst[0]), ep["kcap"], ep["rounds"],
                                               ep["batch_B"], ep["eval_budget"], 1024, 23, ep["knots_per_segment"],
                                               ep["k_ref"])
    K = int(o["nseg"].item())
    m = list(o["modes"].cpu().numpy()[:K])
    lens = np.bincount([int(k) >> 60 for k in keys], minlength=9)[1:]
    print("free uniform: evaluated", len(keys), "lengths", lens, "device plan", m, float(o["cost"].item()),
          "oracle plan", F.key_modes(bk), bJ, flush=True)
    assert np.array_equal(keys, np.array(okeys, np.uint64)) and st["evaluated"] == len(okeys) == 1280
    assert lens[0] == 16 and lens[2:].min() >= 100    # long orders as often as short ones
    assert K >= 1 and float(o["viol"][0]) <= 1e-5
    modes = np.zeros((1, 8), np.int32)
    knots = np.zeros((1, 8), np.int32)
    modes[0, :K] = m
    knots[0, :K] = 5
    r = F.evaluate(f32(x0), f32(goal), f32(inst), np.array([K]), modes, knots, params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"][0])) <= 1e-3 * abs(r["cost"][0])
    if F.key_modes(bk) != m:
        assert abs(bJ - float(o["cost"].item())) <= 1e-3 * abs(bJ)


def test_free_expansion_at_the_paper_configuration_replays_on_the_oracle():
    """The free-motion expansion as the paper configures it (Sec. IV-A): segment cap eight,
    seed of every admissible order of at most six segments, three rounds of two-edit
    neighbourhoods, 50 intervals per order, refinement of the 256 best.  The seed batch is
    the oracle's, every later batch equals the oracle's batch step on the device's own
    (key, Eq. (5) merit) of everything evaluated before it, and the returned plan is
    re-solved by the oracle at the refinement budget to the same cost."""
    import torch
    import oracle
    from oracle import free as F
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(5300, 1)
    B, W, budget = 16384, 1024, 205632
    prm = native.ExpandParams(kcap=8, seed_max_segments=6, radius=2, rounds=3, frontier_W=W, knots_per_segment=0,
                              n_total=50, k_ref=256, batch_B=B, eval_budget=budget)
    ctx = _ctx(max_batch=B, max_intervals=50, max_segments=8)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
    torch.cuda.synchronize()
    keys, J, v = [a.cpu().numpy() for a in native.expand_trace(ctx)]
    keys = keys.view(np.uint64)
    merit = np.array([oracle.merit(a, b) for a, b in zip(J, v)])
    seed = F.seed(6)
    assert np.array_equal(keys[:len(seed)], seed)
    pos, sizes = len(seed), [len(seed)]
    while pos < len(keys):
        nxt = F.expand_next(keys[:pos], merit[:pos], 8, 2, W, min(B, budget - pos))
        assert len(nxt) > 0 and np.array_equal(keys[pos:pos + len(nxt)], nxt), (pos, len(nxt))
        pos += len(nxt)
        sizes.append(len(nxt))
    K = int(o["nseg"].item())
    print(f"free expansion: batches {sizes}, evaluated {st['evaluated']}, feasible {st['n_feasible']}, plan "
          f"{o['modes'].cpu().numpy()[:K]} knots {o['knots'].cpu().numpy()[:K]} cost {float(o['cost'].item()):.6f}",
          flush=True)
    assert st["evaluated"] == len(keys) and len(sizes) == st["rounds_done"]
    assert K >= 1 and float(o["viol"][0]) <= 1e-5 and int(o["knots"].cpu().numpy()[:K].sum()) == 50
    modes = np.zeros((1, 8), np.int32)
    knots = np.zeros((1, 8), np.int32)
    modes[0, :K] = o["modes"].cpu().numpy()[:K]
    knots[0, :K] = o["knots"].cpu().numpy()[:K]
    r = F.evaluate(f32(x0), f32(goal), f32(inst), np.array([K]), modes, knots, params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"][0])) <= 1e-3 * abs(r["cost"][0])
