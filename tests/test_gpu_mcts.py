"""GPU MCTS allocation (UCT with virtual loss and random rollouts, Sec. IV-A / IV-B) against the
MCTS oracle: the first batch (before any reward) is the oracle's selection bit for bit on
both tasks; a whole search evaluates distinct orders of the language within the budget and
returns a plan the oracle confirms.  Later batches depend on rewards computed from each
side's own evaluations; replaying the oracle's search on the device's own (J, v) of every
order makes the whole selection sequence comparable bit for bit."""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.asarray(a, np.float32)).cuda()


@pytest.mark.parametrize("task,kcap,P,seed", [(0, 3, 64, 5), (0, 2, 200, 8), (1, 2, 64, 3), (1, 3, 256, 12)])
def test_first_batch_is_the_oracle_selection(task, kcap, P, seed):
    import torch
    from oracle import mcts as T
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=max(P, 64), max_segments=6, max_intervals=kcap * 5, task=task)
    prm = native.ExpandParams(kcap=kcap, knots_per_segment=5, k_ref=4, batch_B=P, eval_budget=P,
                              policy=native.POLICY_MCTS, sample_seed=seed)
    pairs = I.flip_pivot_pairs(seed, 1) if task == 1 else I.push_pairs(seed, 1)
    o, st = native.expand(ctx, _t(pairs[0][0]), _t(pairs[1][0]), _t(pairs[2][0]), prm)
    torch.cuda.synchronize()
    got = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
    ref = np.array(T.first_batch(task, kcap, P, seed, eval_budget=P), np.uint64)
    # repeated selections leave room in the budget: a second, reward-dependent batch follows
    print(f"task {task}: evaluated {len(got)} orders, first batch of the oracle {len(ref)}")
    assert len(got) <= P and np.array_equal(got[:len(ref)], ref)


def test_push_mcts_search_plan_confirmed_by_oracle():
    import torch
    import oracle
    from oracle import mcts as T
    from oracle.sample import key_modes
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_pairs(9100, 1)
    ep = dict(kcap=3, knots_per_segment=8, k_ref=32, batch_B=64, eval_budget=1500)
    ctx = native.Context(max_batch=64, max_segments=6, max_intervals=24)
    prm = native.ExpandParams(**ep, policy=native.POLICY_MCTS, sample_seed=7)
    o, st = native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), prm)
    torch.cuda.synchronize()
    keys = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
    bk, bJ, bv, okeys, J, v, nb, _ = T.mcts_search(0, x0[0], goal[0], inst[0], ep["kcap"], ep["batch_B"],
                                                   ep["eval_budget"], 7, ep["knots_per_segment"], ep["k_ref"])
    K = int(o["nseg"].item())
    print("device", st, o["modes"].cpu().numpy()[:K], float(o["cost"].item()), "oracle", len(okeys), nb,
          key_modes(bk), bJ, "common orders", len(set(keys.tolist()) & set(okeys)))
    assert len(keys) == st["evaluated"] <= ep["eval_budget"] and len(set(keys.tolist())) == len(keys)
    fb = T.first_batch(0, ep["kcap"], ep["batch_B"], 7)
    assert np.array_equal(keys[:len(fb)], np.array(fb, np.uint64)) and okeys[:len(fb)] == fb   # the first batch
    assert K >= 1
    m = list(o["modes"].cpu().numpy()[:K])
    r = oracle.evaluate(np.asarray(x0[:1], np.float32).astype(np.float64),
                        np.asarray(goal[:1], np.float32).astype(np.float64),
                        np.asarray(inst[:1], np.float32).astype(np.float64), np.array([K]),
                        np.array([m + [0] * (6 - K)]), np.array([[8] * K + [0] * (6 - K)]),
                        params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"].item())) <= 1e-4 * abs(r["cost"][0])
    # both searches return plans of comparable cost (their trees part after the first rewards)
    assert abs(bJ - float(o["cost"].item())) <= 0.05 * abs(bJ)


def test_mcts_parameters_are_checked():
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=64, max_segments=6, max_intervals=10)
    x0, goal, inst = I.push_pairs(1, 1)
    with pytest.raises(native.CometError):
        native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), native.ExpandParams(
            kcap=2, knots_per_segment=5, batch_B=64, eval_budget=100, policy=native.POLICY_MCTS, uct_c=-1.0))
    mlp = native.MLP(max_batch=64, seed=1)
    with pytest.raises(native.CometError):
        native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), native.ExpandParams(
            kcap=2, knots_per_segment=5, batch_B=64, eval_budget=100, policy=native.POLICY_MCTS), learned=mlp)


def test_flip_mcts_search_plan_confirmed_by_oracle():
    """Flipping (reward M_best / M): distinct orders of the language within the budget, the
    oracle's first batch, and a returned plan the oracle re-solves to the same cost."""
    import torch
    import oracle
    from oracle import flip as F
    from oracle import mcts as T
    from oracle.sample import key_modes
    from paper_2609_21803_amd import native
    x0, goal, inst = I.flip_pivot_pairs(9400, 1)
    ep = dict(kcap=2, knots_per_segment=10, k_ref=8, batch_B=128, eval_budget=640)
    ctx = native.Context(max_batch=128, max_segments=6, max_intervals=20, task=native.TASK_FLIP)
    prm = native.ExpandParams(**ep, policy=native.POLICY_MCTS, sample_seed=3)
    o, st = native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), prm)
    torch.cuda.synchronize()
    keys = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
    K = int(o["nseg"].item())
    print("device", st, o["modes"].cpu().numpy()[:K], float(o["cost"].item()))
    assert len(keys) == st["evaluated"] <= ep["eval_budget"] and len(set(keys.tolist())) == len(keys)
    assert all(F.admissible(key_modes(int(k))) for k in keys)
    fb = T.first_batch(1, ep["kcap"], ep["batch_B"], 3)
    assert np.array_equal(keys[:len(fb)], np.array(fb, np.uint64))
    assert K >= 1
    m = list(o["modes"].cpu().numpy()[:K])
    r = F.evaluate(np.asarray(x0[:1], np.float32).astype(np.float64), np.asarray(goal[:1], np.float32).astype(np.float64),
                   np.asarray(inst[:1], np.float32).astype(np.float64), np.array([K]), np.array([m + [0] * (6 - K)]),
                   np.array([[10] * K + [0] * (6 - K)]), params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"].item())) <= 1e-4 * abs(r["cost"][0])


@pytest.mark.parametrize("task,kcap,P,budget,seed", [(0, 3, 64, 1500, 7), (0, 3, 256, 1200, 11), (1, 2, 128, 640, 3)])
def test_whole_search_replays_bit_for_bit_on_device_results(task, kcap, P, budget, seed):
    """The oracle's search, fed the device's per-order (J, v) from the expansion trace in
    place of its own evaluator, selects the device's evaluated orders in the same order,
    batch after batch, to the end of the search (tree rules, virtual loss, rollouts,
    rewards and the budget rule of both sides agree exactly)."""
    import torch
    from oracle import mcts as T
    from paper_2609_21803_amd import native
    kn = 10 if task == 1 else 8
    ctx = native.Context(max_batch=P, max_segments=6, max_intervals=kcap * kn, task=task)
    prm = native.ExpandParams(kcap=kcap, knots_per_segment=kn, k_ref=8, batch_B=P, eval_budget=budget,
                              policy=native.POLICY_MCTS, sample_seed=seed)
    pairs = I.flip_pivot_pairs(9400 + seed, 1) if task == 1 else I.push_pairs(9100 + seed, 1)
    o, st = native.expand(ctx, _t(pairs[0][0]), _t(pairs[1][0]), _t(pairs[2][0]), prm)
    torch.cuda.synchronize()
    k_dev, J_dev, v_dev = (a.cpu().numpy() for a in native.expand_trace(ctx))
    k_dev = k_dev.view(np.uint64)
    table = {int(k): (float(a), float(b)) for k, a, b in zip(k_dev, J_dev, v_dev)}
    missing = []

    def device_results(keys, refine):
        if refine:                      # refinement does not steer the search
            return np.zeros(len(keys)), np.full(len(keys), np.inf)
        out = [table.get(int(k)) for k in keys]
        missing.extend(int(k) for k, r in zip(keys, out) if r is None)
        return (np.array([r[0] if r else np.nan for r in out]), np.array([r[1] if r else np.inf for r in out]))

    _, _, _, keys, _, _, nb, _ = T.mcts_search(task, None, None, None, kcap, P, budget, seed, kn, 8,
                                               evaluate=device_results)
    print(f"task {task}: device {len(k_dev)} orders, replay {len(keys)} orders in {nb} batches, "
          f"missing {len(missing)}")
    assert not missing and np.array_equal(np.array(keys, np.uint64), k_dev)
