"""GPU parity of the uniform-sampling allocation policy (the baseline of Sec. IV-B) against the
sampling oracle: the device draws exactly the oracle's batches (bit-exact keys, both
tasks), and a whole flipping search returns a plan the oracle confirms."""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.as_tensor(np.asarray(a, np.float32)).cuda()


def _oracle_batches(task, seed, rounds, draws, kcap, batch_B, budget):
    from oracle import sample as S
    keys, seen = [], set()
    for s in range(rounds + 1):
        room = min(batch_B, budget - len(keys))
        if room <= 0:
            break
        b = S.sample_round(task, seed, s * draws, draws, kcap, seen, room)
        seen.update(b)
        keys += b
    return np.array(keys, np.uint64)


@pytest.mark.parametrize("task,kcap,draws,batch_B,budget,seed", [(1, 2, 20000, 300, 900, 17), (1, 3, 50000, 700, 1500, 4),
                                                                 (0, 3, 2000, 200, 600, 9), (0, 1, 50, 16, 40, 2)])
def test_sampled_batches_are_bit_exact(task, kcap, draws, batch_B, budget, seed):
    import torch
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=max(batch_B, 64), max_segments=6, max_intervals=kcap * 5, task=task)
    prm = native.ExpandParams(kcap=kcap, rounds=2, knots_per_segment=5, k_ref=4, batch_B=batch_B, eval_budget=budget,
                              policy=native.POLICY_UNIFORM, sample_seed=seed, sample_draws=draws)
    if task == 1:
        x0, goal, inst = I.flip_pivot_pairs(seed, 1)
        o, st = native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), prm)
    else:
        x0, goal, inst = I.push_pairs(seed, 1)
        o, st = native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), prm)
    torch.cuda.synchronize()
    keys, _, _ = native.expand_trace(ctx)
    got = keys.cpu().numpy().view(np.uint64)
    ref = _oracle_batches(task, seed, 2, draws, kcap, batch_B, budget)
    print(f"task {task}: {len(got)} sampled orders over {st['rounds_done']} rounds, oracle {len(ref)}")
    assert len(got) == len(ref) and np.array_equal(got, ref)
    assert st["evaluated"] == len(ref)


def test_uniform_flip_search_returns_a_plan_the_oracle_confirms():
    import torch
    import oracle
    from oracle import flip as F
    from oracle import sample as S
    from paper_2609_21803_amd import native
    x0, goal, inst = I.flip_pivot_pairs(9400, 1)
    ep = dict(kcap=2, rounds=1, knots_per_segment=10, k_ref=8, batch_B=1024, eval_budget=2048)
    ctx = native.Context(max_batch=1024, max_segments=6, max_intervals=20, task=native.TASK_FLIP)
    prm = native.ExpandParams(**ep, policy=native.POLICY_UNIFORM, sample_seed=21, sample_draws=65536)
    o, st = native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), prm)
    torch.cuda.synchronize()
    K = int(o["nseg"].item())
    bk, bJ, bv, keys, J, v = S.uniform_search(1, x0[0], goal[0], inst[0], ep["kcap"], ep["rounds"], ep["batch_B"],
                                              ep["eval_budget"], 65536, 21, ep["knots_per_segment"], ep["k_ref"])
    print("device", st, o["modes"].cpu().numpy()[:K], float(o["cost"].item()), "oracle", S.key_modes(bk), bJ,
          "oracle feasible", int((v <= 1e-5).sum()))
    assert st["evaluated"] == len(keys)
    assert abs(st["n_feasible"] - int((v <= 1e-5).sum())) <= max(3, 0.05 * st["n_feasible"])
    assert K >= 1 and bk != 0
    m = list(o["modes"].cpu().numpy()[:K])
    r = F.evaluate(np.asarray(x0[:1], np.float32).astype(np.float64), np.asarray(goal[:1], np.float32).astype(np.float64),
                   np.asarray(inst[:1], np.float32).astype(np.float64), np.array([K]),
                   np.array([m + [0] * (6 - K)]), np.array([[10] * K + [0] * (6 - K)]),
                   params=oracle.Params(**oracle.REFINE))
    assert r["feasible"][0] == 1 and abs(r["cost"][0] - float(o["cost"].item())) <= 1e-4 * abs(r["cost"][0])
    if S.key_modes(bk) != m:
        assert abs(bJ - float(o["cost"].item())) <= 1e-3 * abs(bJ)   # a near tie


def test_sampling_parameters_are_checked():
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=64, max_segments=6, max_intervals=10)
    x0, goal, inst = I.push_pairs(1, 1)
    bad = native.ExpandParams(kcap=2, rounds=1, knots_per_segment=5, batch_B=64, eval_budget=100,
                              policy=native.POLICY_UNIFORM, sample_draws=0)
    with pytest.raises(native.CometError):
        native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), bad)
    with pytest.raises(native.CometError):
        native.expand(ctx, _t(x0[0]), _t(goal[0]), _t(inst[0]), native.ExpandParams(
            kcap=2, rounds=1, knots_per_segment=5, batch_B=64, eval_budget=100, policy=3))
    import torch
    keys = torch.zeros(4, dtype=torch.int64, device="cuda")
    merit = torch.zeros(4, dtype=torch.float64, device="cuda")
    with pytest.raises(native.CometError):
        native.expand_next(ctx, keys, merit, native.ExpandParams(kcap=2, knots_per_segment=5, batch_B=64,
                                                                 eval_budget=100, policy=native.POLICY_UNIFORM), 8)
