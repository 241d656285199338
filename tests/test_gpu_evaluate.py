"""GPU parity of the HIP evaluator against the FP64 oracle (called through the C ABI).

Sequence by sequence (the rule of tests/parity.py): on every margin sequence (oracle
violation <= 0.1 eps_feas or >= eps_feas + 1e-3) the device and the oracle return the same
feasible flag, and where both are feasible the objective within 1e-4 relative and the
violation within 1e-5 absolute.  A disagreeing margin sequence is excused only where the
FP64 oracle itself changes its answer under float32-level perturbations (one-ulp input
moves, and those together with the oracle's float32 rounding of what the device keeps in
float32): a decision boundary of the local solver.  Each excused sequence is printed, and
at most 1 in 1,000 margin sequences may stay unexcused (each printed).
Inputs are rounded to float32 before they reach the oracle, so both sides solve the same
problem.
"""
import numpy as np
import pytest

import parity
from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu

EPS = 1e-5
# the quantities this evaluator keeps in float32, as the oracle's rounding switch for the
# excuse draws: the step direction (1), multipliers (2), scaled row Jacobians (4), and the
# gains with the forward recursion dz = k + K dx in float32 (8)
ROUND32 = 1 | 2 | 4 | 8


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


def run_gpu(batch, max_intervals, refine=0, warm=None, params=None):
    import torch
    from paper_2609_21803_amd import native
    B = len(batch["nseg"])
    ctx = native.Context(max_batch=max(B, 1), max_segments=6, max_intervals=max_intervals, params=params)
    d = native.to_device(batch)
    w = None if warm is None else torch.as_tensor(warm, dtype=torch.float32).contiguous().cuda()
    out = ctx.evaluate(**d, warm=w, refine=refine)
    torch.cuda.synchronize()
    res = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    res["ctx"] = ctx
    return res


def run_oracle(batch, nmax, params=None, warm=None):
    import oracle
    return oracle.evaluate(f32(batch["x0"]), f32(batch["goal"]), f32(batch["inst"]), batch["nseg"], batch["modes"],
                           batch["knots"], params=params, nmax=nmax, warm=warm)


def compare(g, o, batch, label, nmax, params=None, warm=None, idx=None):
    """The per-sequence rule; excuses are checked by re-solving nudged inputs with the
    oracle under the same parameters (and the same warm start, if any)."""
    import oracle
    base = params or oracle.Params()

    def solve(sub, rows, r32):
        prm = oracle.Params(**{**base.__dict__, "round32": r32})
        return run_oracle(sub, nmax, params=prm, warm=None if warm is None else warm[rows])
    return parity.check(g, o, batch, solve, label, idx=idx, round32=ROUND32)


def test_tiny_workload_all_orders_match_oracle(orc):
    """8 start/goal pairs x all 144 two-segment orders, 5+5 intervals: every TO."""
    b = I.push_tiny()
    g = run_gpu(b, 10)
    g["ctx"].check()
    o = run_oracle(b, 10)
    compare(g, o, b, "tiny", 10)
    # brute-force mode selection over the 144 orders picks the same order per pair where
    # the best feasible cost beats the runner-up by more than 1e-3 relative
    for p in range(8):
        sel = b["pair"] == p
        oc = np.where(o["feasible"][sel] == 1, o["cost"][sel], np.inf)
        gc = np.where(g["feasible"][sel] == 1, g["cost"][sel].astype(np.float64), np.inf)
        order = np.argsort(oc)
        if np.isfinite(oc[order[1]]) and (oc[order[1]] - oc[order[0]]) / max(abs(oc[order[0]]), 1e-12) > 1e-3:
            assert np.argmin(gc) == order[0], p


@pytest.mark.parametrize("trials", [3, 12])
def test_line_search_trial_counts_match_oracle(orc, trials):
    """Other trial-step counts than the default eight (the forward pass has a separate
    variant for more than eight trials): the tiny workload against the oracle with the
    same count."""
    import oracle
    from paper_2609_21803_amd import native
    b = I.push_tiny()
    g = run_gpu(b, 10, params=native.SolverParams(ls_trials=trials))
    g["ctx"].check()
    o = run_oracle(b, 10, params=oracle.Params(ls_trials=trials))
    compare(g, o, b, f"tiny, {trials} trials", 10, params=oracle.Params(ls_trials=trials))


def test_ragged_batch_matches_oracle(orc):
    """Uneven segment counts (1..5) and interval counts (5..15 per segment) in one launch."""
    b = I.push_hetero(B=2048, seed=77)
    nmax = int(I.n_intervals(b).max())
    g = run_gpu(b, 75)
    o = run_oracle(b, 75)
    compare(g, o, b, "ragged", 75)
    # trajectory rows beyond N are zero and row N carries u = 0
    N = I.n_intervals(b)
    for i in range(0, 2048, 97):
        assert np.all(g["traj"][i, N[i] + 1:] == 0) and np.all(g["traj"][i, N[i], 4:] == 0)
    assert nmax <= 75


def test_full_size_plain_workload_all_sequences(orc):
    """64 pairs x 1,728 three-segment orders (110,592 TOs) in the launch the benchmark
    times; every sequence is compared with the oracle's (about a minute of the oracle on
    16 host threads)."""
    b = I.push_plain()
    g = run_gpu(b, 24)
    g["ctx"].check()
    o = run_oracle(b, 24)
    compare(g, o, b, "plain, all 110,592", 24)
    assert np.all(np.isfinite(g["cost"][g["feasible"] == 1]))


def test_closed_form_and_zero_goal_on_gpu(orc):
    """Straight sticking push reaches d^2/T within 1e-4; goal = start is feasible at ~0 cost."""
    x0 = np.zeros((2, 4))
    goal = np.array([[0.2, 0, 0], [0, 0, 0]])
    inst = np.array([[0.4], [0.35]])
    modes = np.zeros((2, 6), np.int32)
    knots = np.zeros((2, 6), np.int32)
    modes[0, 0], knots[0, 0] = 6, 10
    modes[1, :2], knots[1, :2] = (3, 8), (5, 5)
    b = dict(x0=x0, goal=goal, inst=inst, nseg=np.array([1, 2], np.int32), modes=modes, knots=knots)
    g = run_gpu(b, 10)
    assert g["feasible"][0] == 1 and abs(g["cost"][0] - 0.04) <= 1e-4 * 0.04
    assert g["feasible"][1] == 1 and g["cost"][1] <= 1e-6


def test_invalid_sequences_flagged_and_counted():
    from paper_2609_21803_amd import native
    b = I.subset(I.push_tiny(), np.arange(8))
    b["modes"][1, 0] = 12           # out-of-range id
    b["nseg"][2] = 0                # no segment
    b["goal"][3, 0] = np.nan        # non-finite input
    b["knots"][4, 1] = 30           # more intervals than the context allows
    # knot counts whose int32 sum wraps: four segments of 2^30 sum to 0 (mod 2^32), and
    # INT32_MAX + 5 is negative; both must be rejected before any interval is written
    b["nseg"][6], b["modes"][6, :4], b["knots"][6, :4] = 4, 3, 2 ** 30
    b["knots"][7, :2] = (2 ** 31 - 1, 5)
    g = run_gpu(b, 10)
    for i in (1, 2, 3, 4, 6, 7):
        assert np.isnan(g["cost"][i]) and np.isinf(g["viol"][i]) and g["feasible"][i] == 0
        assert g["stats"][i, 3] == 3
    assert np.isfinite(g["cost"][0]) and np.isfinite(g["cost"][5])
    with pytest.raises(native.CometError):
        g["ctx"].check()
    g["ctx"].check()                # the counter was cleared


def test_results_do_not_depend_on_batch_and_are_deterministic():
    b = I.push_hetero(B=512, seed=5)
    g1 = run_gpu(b, 75)
    g2 = run_gpu(b, 75)
    assert np.array_equal(g1["cost"], g2["cost"], equal_nan=True) and np.array_equal(g1["traj"], g2["traj"])
    sub = np.arange(100, 300, 3)
    g3 = run_gpu(I.subset(b, sub), 75)
    assert np.array_equal(g3["cost"], g1["cost"][sub], equal_nan=True)
    assert np.array_equal(g3["viol"], g1["viol"][sub])


def test_empty_batch_and_host_argument_errors():
    import torch
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=8, max_intervals=10)
    e = lambda *s: torch.empty(s, dtype=torch.float32, device="cuda")
    ei = lambda *s: torch.empty(s, dtype=torch.int32, device="cuda")
    out = ctx.evaluate(e(0, 4), e(0, 3), e(0, 1), ei(0), ei(0, 6), ei(0, 6))
    assert out["cost"].numel() == 0
    with pytest.raises(native.CometError):
        ctx.evaluate(e(9, 4), e(9, 3), e(9, 1), ei(9), ei(9, 6), ei(9, 6))   # B > max_batch
    with pytest.raises(native.CometError):
        native.Context(max_batch=8, max_segments=7)


def test_warm_start_matches_oracle_with_same_warm_start(orc):
    """A warm start replaces the schedule-derived primal (multipliers start at zero);
    both sides start from the same float32 trajectory: the oracle's solution."""
    b = I.subset(I.push_tiny(), np.arange(0, 1152, 7))
    o = run_oracle(b, 10)
    warm = o["traj"].astype(np.float32)
    g = run_gpu(b, 10, warm=warm)
    o2 = run_oracle(b, 10, warm=warm.astype(np.float64))
    compare(g, o2, b, "warm", 10, warm=warm.astype(np.float64))


def test_refinement_budget_matches_oracle(orc):
    """Refinement budget (AL <= 40, GN <= 25).  Five times the iterations of the
    exploration budget give proportionally more near-tie trial steps, so the bar is 97 %;
    the oracle's own sensitivity to a one-ulp goal perturbation at this budget is printed."""
    import oracle
    b = I.subset(I.push_tiny(seed=3), np.arange(0, 1152, 2))
    g = run_gpu(b, 10, refine=1)
    prm = oracle.Params(**oracle.REFINE)
    o = run_oracle(b, 10, params=prm)
    compare(g, o, b, "refine", 10, params=prm)
    o2 = run_oracle(parity.nudge(b, np.random.default_rng(2)), 10, params=prm)
    m = parity.margin_mask(o["viol"])
    print(f"refinement budget: the oracle changes its answer on {(~parity.agrees(o2, o))[m].mean():.4f} of the "
          f"margin sequences under one-ulp input moves")


@pytest.mark.parametrize("kw", [dict(chol_retries=0), dict(rho_max=1e-6), dict(al_max=1), dict(rho0=-1.0),
                                dict(rho0=-1.0, chol_retries=0)])
def test_forced_failure_paths_match_oracle(orc, kw):
    """The solver's failure paths forced by its parameters on both sides (normal-exit
    solves): no retry after a failed factorisation, a damping cap of 1e-6, one outer
    iteration, an indefinite start (rho0 = -1: the first factorisation of every solve fails),
    and the indefinite start without retries (every factorisation fails, every step is
    rejected).  Per-sequence parity on the two-segment workload, the feasible flag equal to
    v <= eps_feas, and the Cholesky failure counts of both sides equal where the path is
    forced."""
    import oracle
    from paper_2609_21803_amd import native
    b = I.subset(I.push_tiny(), np.arange(0, 1152, 3))
    g = run_gpu(b, 10, params=native.SolverParams(**kw))
    g["ctx"].check()
    prm = oracle.Params(**kw)
    o = run_oracle(b, 10, params=prm)
    compare(g, o, b, f"forced {kw}", 10, params=prm)
    assert np.array_equal(g["feasible"] == 1, g["viol"] <= EPS)
    assert set(np.unique(g["stats"][:, 3])) <= {0, 1, 2}
    if kw.get("al_max") == 1:
        assert np.all(g["stats"][:, 0] == 1)
    if kw.get("rho0") == -1.0:
        assert np.all(g["stats"][:, 2] >= 1)
        if kw.get("chol_retries") == 0:
            assert np.array_equal(g["stats"], o["stats"]) and np.all(g["feasible"] == 0)


def test_row_scales_agree_with_oracle(orc):
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=1, max_intervals=4)
    assert np.allclose(ctx.row_scales(), orc.scales()[:12], rtol=1e-12, atol=0)


def test_oracle_self_sensitivity(orc):
    """Context for the excuses above: how often the FP64 oracle changes its own answer
    when the inputs move by at most one float32 ulp, on the long ragged workload."""
    b = I.push_hetero(B=1024, seed=77)
    o = run_oracle(b, 75)
    o2 = run_oracle(parity.nudge(b, np.random.default_rng(1)), 75)
    m = parity.margin_mask(o["viol"])
    frac = (~parity.agrees(o2, o))[m].mean()
    print(f"oracle vs nudged oracle: {frac:.4f} of {m.sum()} margin sequences change")
    assert frac < 0.05


def test_schedules_give_identical_results_and_autotuner_picks_one():
    """The persistent pool, its width and the length-sorted queue change only where an
    order is solved, never its arithmetic: outputs are bitwise identical."""
    import torch
    from paper_2609_21803_amd import native
    b = I.push_hetero(B=3000, seed=21)
    d = native.to_device(b)
    ctx = native.Context(max_batch=3000, max_intervals=75)
    outs = []
    for wpc, srt in [(0, 0), (1, 1), (3, 0), (8, 1)]:
        ctx.set_schedule(wpc, srt)
        o = ctx.evaluate(**d)
        torch.cuda.synchronize()
        outs.append({k: v.cpu().numpy() for k, v in o.items()})
    for o in outs[1:]:
        for k in ("cost", "viol", "feasible", "traj", "stats"):
            assert np.array_equal(o[k], outs[0][k], equal_nan=True), k
    out = dict(cost=torch.empty(3000, device="cuda"), viol=torch.empty(3000, device="cuda"),
               feasible=torch.empty(3000, dtype=torch.uint8, device="cuda"))
    sched, ms = ctx.autotune(**d, out=out)
    assert ms > 0 and ctx.schedule()["waves_per_cu"] == sched["waves_per_cu"]
    assert np.array_equal(out["cost"].cpu().numpy(), outs[0]["cost"], equal_nan=True)
    print("autotuned schedule", sched, f"{ms:.2f} ms", ctx.schedule())


def _max_length_batch():
    rng = np.random.default_rng(510)
    B = 32
    x0, goal, inst = I.push_pairs(510, B)
    b = dict(x0=np.asarray(x0, np.float32), goal=np.asarray(goal, np.float32), inst=np.asarray(inst, np.float32),
             nseg=np.full(B, 6, np.int32), modes=rng.integers(0, 12, (B, 6)).astype(np.int32),
             knots=np.full((B, 6), 85, np.int32))
    # order 0: the straight push of 0.5 m through the face-2 centre
    b["x0"][0] = 0.0
    b["goal"][0] = (0.5, 0.0, 0.0)
    b["modes"][0] = 6
    return b


def _max_length_run(b, task, kw):
    import oracle
    import torch
    from paper_2609_21803_amd import native
    ctx = native.Context(max_batch=len(b["nseg"]), max_segments=6, max_intervals=512, task=task,
                         params=native.SolverParams(**kw))
    out = ctx.evaluate(**native.to_device(b))
    torch.cuda.synchronize()
    ctx.check()
    g = {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
    o = oracle.evaluate(f32(b["x0"]), f32(b["goal"]), f32(b["inst"]), b["nseg"], b["modes"], b["knots"],
                        params=oracle.Params(timed=1 if task == 2 else 0, **kw), nmax=512)
    conv = (g["stats"][:, 3] == 1) & (o["stats"][:, 3] == 1)
    rel = np.abs(g["cost"].astype(np.float64) - o["cost"]) / np.maximum(np.abs(o["cost"]), 1e-12)
    print(f"maximum length, task {task} {kw}: both converged {conv.sum()}, status agreement "
          f"{(g['stats'][:, 3] == o['stats'][:, 3]).mean():.3f}, feasible gpu/oracle {g['feasible'].sum()}/"
          f"{o['feasible'].sum()}, max rel cost on converged {rel[conv].max() if conv.any() else 0:.2e}", flush=True)
    assert np.all(g["traj"][:, 511:] == 0) and np.all(g["traj"][:, 510, 4:] == 0)
    return g, o, conv, rel


@pytest.mark.parametrize("task", [0, 2])
def test_maximum_length_sequences_match_oracle(orc, task):
    """Orders at the longest work-space height: 6 segments x 85 intervals = 510 of the 512
    intervals a context can hold, fixed step and optimised timing, default tolerances.  The
    straight push reaches its closed form (d^2 / T, or d^2 / T + w_T T with T at the
    duration bound) within 5e-3: every one of the 510 defects may sit within the stopping
    tolerance (about 1e-6 m) and these slacks add up along the push (the FP64 oracle itself
    lands 2.5e-3 and 1.1e-3 from it).  Where both sides converge, the flags agree and the
    costs within 1e-3: the stopping region (stationarity 1e-4) is wide over 510 stages, and
    the device's FP32 gains and steps end at another point of it than the oracle's FP64
    path (tightened tolerances shrink the gap, see the next test; the oracle's own change
    under a one-ulp goal move is at most 1.2e-6 there).  The statuses agree on most orders."""
    b = _max_length_batch()
    g, o, conv, rel = _max_length_run(b, task, {})
    T = 510 * 0.1 if task == 0 else min(max(0.5 / 0.1, 510 * 0.02), 510 * 0.2)
    Jstar = 0.25 / T + (0.01 * T if task == 2 else 0.0)
    assert g["feasible"][0] == 1 and abs(float(g["cost"][0]) - Jstar) <= 5e-3 * Jstar, (g["cost"][0], Jstar)
    assert conv.sum() >= 1
    assert np.array_equal(g["feasible"][conv], o["feasible"][conv]) and np.all(rel[conv] <= 1e-3)
    assert (g["stats"][:, 3] == o["stats"][:, 3]).mean() >= 0.8


def test_maximum_length_tight_tolerances_match_oracle(orc):
    """The same 510-interval orders (fixed step) with tightened stopping tolerances
    (stationarity 1e-6, feasibility and complementarity 1e-8, refinement-size budget):
    most converge on both sides, the costs agree within 1e-4 and the straight push is
    within 1e-4 of d^2 / T."""
    b = _max_length_batch()
    kw = dict(omega_star=1e-6, eta_star=1e-8, rc_star=1e-8, al_max=40, gn_max=25)
    g, o, conv, rel = _max_length_run(b, 0, kw)
    assert conv.sum() >= 16
    assert np.array_equal(g["feasible"][conv], o["feasible"][conv]) and np.all(rel[conv] <= 1e-4)
    assert abs(float(g["cost"][0]) - 0.25 / 51.0) <= 1e-4 * 0.25 / 51.0
