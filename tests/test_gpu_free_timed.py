"""GPU parity of pushing with free motion and optimised timing (COMET_TASK_PUSH_FREE_TIMED:
the language of Sec. III-A, the interval durations as controls with bounds, the paper's
pushing transcription) against the FP64 oracle built with -DFREE_TIMED, through the C ABI.

* Evaluation, sequence by sequence with the rule of tests/parity.py (allowance 2e-3 of the
  margin sequences, as for timed pushing), on every admissible order of at most two
  segments, a ragged batch of up to four segments, and a strided sample of every
  admissible order of at most six segments with 50 intervals per order on 8 instances.
* The same at the planner's budgets of this transcription (exploration and refinement).
* Row scales equal to the oracle's; closed forms of a free approach and a straight push
  with the durations inside and at both bounds.
* The expansion in the paper's configuration (cap eight, seed of at most six segments,
  three two-edit rounds, 50 intervals per order): every batch equals the oracle's step on
  the device's own merits, and the oracle re-solves the returned plan to the same cost.
Inputs are rounded to float32 before they reach the oracle.
"""
import numpy as np
import pytest

import parity
from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu

ROUND32 = 1 | 2 | 4 | 8
HMIN, HMAX, WT = 0.02, 0.2, 0.01


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def _ctx(max_batch, max_intervals, max_segments=8):
    from paper_2609_21803_amd import native
    return native.Context(max_batch=max_batch, max_segments=max_segments, max_intervals=max_intervals,
                          task=native.TASK_PUSH_FREE_TIMED)


def run_gpu(batch, max_intervals):
    import torch
    from paper_2609_21803_amd import native
    ctx = _ctx(max(len(batch["nseg"]), 1), max_intervals, max(batch["modes"].shape[1], 6))
    out = ctx.evaluate(**native.to_device(batch))
    torch.cuda.synchronize()
    ctx.check()
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def run_oracle(batch, nmax, params=None):
    import oracle
    from oracle import free as F
    return F.evaluate(f32(batch["x0"]), f32(batch["goal"]), f32(batch["inst"]), batch["nseg"], batch["modes"],
                      batch["knots"], params=params or oracle.Params(), nmax=nmax, timed=True)


def compare(g, o, batch, label, nmax):
    import oracle

    def solve(sub, rows, r32):
        return run_oracle(sub, nmax, oracle.Params(round32=r32))
    parity.check(g, o, batch, solve, label, round32=ROUND32, allow=2e-3)


def _orders(kmax):
    from oracle import free as F
    return [F.key_modes(int(k)) for k in F.seed(kmax)]


def _split(K, n=50):
    return [n // K + (1 if j < n % K else 0) for j in range(K)]


def test_all_short_orders_match_oracle():
    """8 instances x all 72 admissible orders of one and two segments, 10 intervals each."""
    x0, goal, inst = I.push_free_pairs(5000, 8)
    orders = _orders(2)
    pair = np.repeat(np.arange(8), len(orders))
    b = I.orders_batch(x0, goal, inst, pair, orders * 8, [[10] * len(o) for o in orders] * 8)
    g = run_gpu(b, 20)
    o = run_oracle(b, 20)
    print("feasible oracle / device:", int(o["feasible"].sum()), int(g["feasible"].sum()))
    assert o["feasible"].sum() >= 3       # at the exploration budget few two-segment solves converge here
    compare(g, o, b, "free timed <= 2 segments", 20)
    fe = g["feasible"] == 1           # a feasible trajectory keeps its durations within the bounds
    h = g["traj"][fe, :20, 9][np.arange(20)[None, :] < I.n_intervals(b)[fe][:, None]]
    assert np.all(h >= HMIN - 2e-5) and np.all(h <= HMAX + 2e-5)


def test_ragged_orders_match_oracle():
    """1,024 admissible orders of 1..4 segments, 4..10 intervals per segment, 16 instances."""
    rng = np.random.default_rng(6100)
    x0, goal, inst = I.push_free_pairs(6101, 16)
    pool = _orders(4)
    pick = rng.integers(0, len(pool), 1024)
    orders = [pool[i] for i in pick]
    knots = [list(rng.integers(4, 11, len(o))) for o in orders]
    b = I.orders_batch(x0, goal, inst, rng.integers(0, 16, 1024), orders, knots)
    g = run_gpu(b, 40)
    o = run_oracle(b, 40)
    print("feasible oracle / device:", int(o["feasible"].sum()), int(g["feasible"].sum()))
    compare(g, o, b, "free timed ragged", 40)


def test_paper_transcription_sampled():
    """Every admissible order of at most six segments with 50 intervals per order (split
    evenly, the remainder to the first segments) on 8 instances: 118,080 TOs in one launch;
    1,024 evenly strided sequences checked against the oracle one by one."""
    orders = _orders(6)
    x0, goal, inst = I.push_free_pairs(6200, 8)
    pair = np.repeat(np.arange(8), len(orders))
    b = I.orders_batch(x0, goal, inst, pair, orders * 8, [_split(len(o)) for o in orders] * 8)
    g = run_gpu(b, 50)
    idx = np.linspace(0, len(b["nseg"]) - 1, 1024).astype(np.int64)
    sub = I.subset(b, idx)
    o = run_oracle(sub, 50)
    print("feasible in the launch:", int(g["feasible"].sum()), "sampled oracle / device:", int(o["feasible"].sum()),
          int(g["feasible"][idx].sum()))
    compare({k: v[idx] for k, v in g.items()}, o, sub, "free timed, 50 intervals (1,024 strided)", 50)


def test_paper_budgets_sampled():
    """The planner's budgets of this transcription (t_exp = 300 read as at most 30 x 10
    Gauss-Newton iterations, t_ref = 1,500 as 60 x 25): the 118,080-order launch at the
    exploration budget with 1,024 evenly strided sequences checked one by one, and 256
    strided orders at the refinement budget (comet_evaluate's refine flag)."""
    import torch
    import oracle
    from paper_2609_21803_amd import native
    orders = _orders(6)
    x0, goal, inst = I.push_free_pairs(6300, 8)
    pair = np.repeat(np.arange(8), len(orders))
    b = I.orders_batch(x0, goal, inst, pair, orders * 8, [_split(len(o)) for o in orders] * 8)
    n = len(b["nseg"])
    ctx = native.Context(max_batch=n, max_segments=6, max_intervals=50, task=native.TASK_PUSH_FREE_TIMED,
                         params=native.SolverParams(al_max=30, gn_max=10, ref_al_max=60, ref_gn_max=25))
    d = native.to_device(b)
    for refine, m, prm in ((0, 1024, dict(al_max=30, gn_max=10)), (1, 256, dict(al_max=60, gn_max=25))):
        idx = np.linspace(0, n - 1, m).astype(np.int64)
        if refine:
            sub = I.subset(b, idx)
            out = ctx.evaluate(**native.to_device(sub), refine=1)
            sel = slice(None)
        else:
            sub = I.subset(b, idx)
            out = ctx.evaluate(**d)
            sel = idx
        torch.cuda.synchronize()
        ctx.check()
        g = {k: v.cpu().numpy()[sel] for k, v in out.items() if v is not None}
        o = run_oracle(sub, 50, oracle.Params(**prm))
        print(f"budget {prm}: feasible oracle / device {int(o['feasible'].sum())} / {int(g['feasible'].sum())}, "
              f"mean GN iterations {g['stats'][:, 1].mean():.1f} / {o['stats'][:, 1].mean():.1f}")

        def solve(s2, rows, r32, prm=prm):
            return run_oracle(s2, 50, oracle.Params(**prm, round32=r32))
        parity.check(g, o, sub, solve, f"free timed, paper budget {prm}", round32=ROUND32, allow=2e-3)


def test_row_scales_agree_with_oracle():
    from oracle import free as F
    s = _ctx(8, 10).row_scales()
    ref = F.scales(timed=True)
    assert np.allclose(s, ref[:len(s)], rtol=1e-12), (s, ref)


@pytest.mark.parametrize("d,N1,N2", [(0.05, 6, 10), (0.12, 10, 12), (0.3, 6, 10), (0.005, 4, 10)])
def test_free_approach_then_straight_push_closed_form_on_gpu(d, N1, N2):
    """Pusher 3 cm in front of face 2, goal (d, 0, 0), [free in front of face 2, stick on
    face 2], durations free: J* = sum over the two moves (D = 0.03, then d) of 2 D sqrt(w_T)
    inside the duration bounds, D^2 / (N h) + N h w_T with h at the bound otherwise;
    reached within 1e-3 at the exploration budget."""
    from oracle import free as F

    def seg(D, N):
        h = min(max(D / (N * np.sqrt(WT)), HMIN), HMAX)
        return D ** 2 / (N * h) + N * h * WT
    Jstar = seg(0.03, N1) + seg(d, N2)
    x0 = np.array([[0.0, 0.0, 0.0, -0.08, 0.0]])
    b = I.orders_batch(x0, np.array([[d, 0.0, 0.0]]), np.array([[0.4]]), np.array([0]), [[F.free(2), F.contact(2, 0)]],
                       [[N1, N2]])
    g = run_gpu(b, N1 + N2)
    assert g["feasible"][0] == 1 and abs(g["cost"][0] - Jstar) <= 1e-3 * Jstar, (g["cost"][0], Jstar)
    assert np.allclose(g["traj"][0, N1, 3:5], [-0.05, 0.0], atol=1e-4)


def test_expansion_at_the_paper_configuration_replays_on_the_oracle():
    """Segment cap eight, seed of every admissible order of at most six segments, three
    rounds of two-edit neighbourhoods (W = 1,024, batches of up to 16,384), 50 intervals per
    order, refinement of the 256 best: every batch after the seed equals the oracle's step on
    the device's (key, Eq. (5) merit); the returned plan re-solves to the same cost."""
    import torch
    import oracle
    from oracle import free as F
    from paper_2609_21803_amd import native
    x0, goal, inst = I.push_free_pairs(5300, 1)
    B, W, budget = 16384, 1024, 205632
    prm = native.ExpandParams(kcap=8, seed_max_segments=6, radius=2, rounds=3, frontier_W=W, knots_per_segment=0,
                              n_total=50, k_ref=256, batch_B=B, eval_budget=budget)
    ctx = _ctx(B, 50)
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
    print(f"free timed expansion: batches {sizes}, evaluated {st['evaluated']}, feasible {st['n_feasible']}, plan "
          f"{o['modes'].cpu().numpy()[:K]} cost {float(o['cost'].item()):.6f}, device {st['t_total_ms']:.0f} ms",
          flush=True)
    assert K >= 1 and float(o["viol"][0]) <= 1e-5
    modes = np.zeros((1, 8), np.int32)
    knots = np.zeros((1, 8), np.int32)
    modes[0, :K] = o["modes"].cpu().numpy()[:K]
    knots[0, :K] = o["knots"].cpu().numpy()[:K]
    plan = dict(x0=x0[:1], goal=goal[:1], inst=inst[:1], nseg=np.array([K], np.int32), modes=modes, knots=knots)

    def refine(sub, rows=None, r32=0):
        return F.evaluate(f32(sub["x0"]), f32(sub["goal"]), f32(sub["inst"]), sub["nseg"], sub["modes"], sub["knots"],
                          params=oracle.Params(**oracle.REFINE, round32=r32), timed=True)
    r = refine(plan)
    print("plan re-solved by the oracle: feasible", int(r["feasible"][0]), "cost", r["cost"][0], "viol", r["viol"][0],
          "device viol", float(o["viol"][0]), flush=True)
    # the per-sequence rule at the refinement budget: agreement, or the oracle itself moves
    parity.check({"cost": o["cost"].cpu().numpy()[:1], "viol": o["viol"].cpu().numpy()[:1], "feasible": np.array([1])},
                 r, plan, refine, "free timed plan at the refinement budget", round32=ROUND32, allow=0.0)
    assert abs(r["cost"][0] - float(o["cost"][0])) <= 1e-3 * abs(r["cost"][0])   # the same optimum either way
