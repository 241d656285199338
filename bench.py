"""Benchmark of the batched mode-conditioned TO evaluator on one MI355X.

A step is one comet_evaluate over the whole batch of the planar-pushing workload
(64 start/goal pairs x all 1,728 three-segment orders, 8+8+8 intervals = 110,592 TOs,
augmented-Lagrangian outer loop <= 20, Gauss-Newton inner loop <= 10), inputs resident in
HBM.  Prints one JSON line with solves/s, the roofline of the solver kernel and the FP64
CPU oracle timed on a bounded sample of the same workload.

The learned leg trains the proposal / warm-start network on evaluator results (BF16 matrix
cores), times its training step and batched inference against the BF16 matrix-core peak,
and compares the device time to the first feasible plan of the plain and the learned
expansion on held-out instances (pushing, flipping, and pushing with free motion, with the
fixed step and as the paper transcribes it, in the paper's s_max = 1 configuration).

The flipping leg times one round of the bimanual-flipping workload (32,768 orders); the
timed leg runs the headline orders with optimised timing (interval durations as controls).

The scale legs run the pushing expansion at W = 4,096 -> B = 131,072 and the flipping
expansion at 32,768 orders per round under a 200,000-evaluation budget.

    python bench.py [--gpus 1] [--steps 5] [--warmup 1] [--no-cpu] [--no-learned] [--no-flip] [--no-timed]
                    [--no-scale]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per control interval per Gauss-Newton iteration of the pushing task
# (structure-aware count, masked rows excluded): linearisation ~150, block assembly ~450,
# 7x7 Cholesky ~140, gains ~490, value update ~200, forward pass ~60 and ~110 per trial step
# length (8 trials): ~2.4 kflop.  An outer (multiplier) update adds ~40 flop per interval.
FLOP_PER_INTERVAL_GN = 2400.0
FLOP_PER_INTERVAL_AL = 40.0
PEAK_FP32_TFLOPS = 157.3     # MI355X published FP32 vector peak
PEAK_BF16_TFLOPS = 2500.0    # MI355X published dense BF16 matrix-core peak
PEAK_FP64_TFLOPS = 78.6      # MI355X published FP64 vector peak
# The pushing solver's arithmetic is FP64 (primal, residuals, merit sums and the Riccati
# recursion; FP32 only stores gains, steps and multipliers): the instruction-mix counters
# in the committed kernel profiles put 96.5 % of its executed floating-point operations
# in FP64, so its ALU roofline is the FP64 vector peak (256 CUs x 4 SIMDs x 16 lanes x
# 2 flop per FMA x 2.4 GHz = 78.6 TFLOP/s).  Packed FP32 is disabled at compile time.
PUSH_PEAK_BASIS = ("FP64 vector peak: 96.5 % of the kernel's executed floating-point operations are FP64 "
                   "(SQ_INSTS_VALU_{FMA,MUL,ADD}_F{32,64} counters in the kernel's profile); frac_of_fp32_peak "
                   "relates the same rate to the 157.3 TFLOP/s FP32 vector peak")
# Flipping task (17 stage unknowns, 32 row slots), structure-aware work per interval per
# Gauss-Newton iteration: linearisation ~0.3 kflop, block assembly ~0.8, 17 x 17 Cholesky
# ~1.6, the 9 right-hand sides ~5.2, value function ~2.2, forward pass ~0.3, trial steps
# ~1.2: ~10 kflop (FP64).
FLIP_FLOP_PER_INTERVAL_GN = 10000.0
# Pushing with optimised timing (8 stage unknowns, 12 row slots): the same count with the
# duration column and the two bound rows: linearisation ~180, block assembly ~620 (the
# squared row fill grows from 109 to 151 entries), 8x8 Cholesky ~200, gains ~640, value
# update ~230, forward pass ~70 and ~130 per trial step length (8 trials): ~3.0 kflop.
TIMED_FLOP_PER_INTERVAL_GN = 3000.0
# Pushing with free motion (9 stage unknowns, 15 row slots, 14 row arguments): linearisation
# ~250, block assembly ~350 (squared row fill ~200 entries), 9x9 Cholesky ~240, the solves
# for 5 + 1 right-hand sides ~490 each way, value update ~360, forward pass ~90 and ~130 per
# trial step length (8 trials): ~3.3 kflop.
FREE_FLOP_PER_INTERVAL_GN = 3300.0
# Free motion with optimised timing (10 stage unknowns, 17 row slots): the free-motion count
# with the duration column in the five defects and the two bound rows, a 10x10 Cholesky
# (~330) and solves for 5 + 1 right-hand sides on 10 unknowns: ~3.8 kflop.
FREE_TIMED_FLOP_PER_INTERVAL_GN = 3800.0
HBM_PEAK_GBS = 8000.0


KERNEL_SOURCES = ["paper_2609_21803_amd/csrc/evaluator.hip", "paper_2609_21803_amd/csrc/push_solver.inc",
                  "paper_2609_21803_amd/csrc/push_model.h", "paper_2609_21803_amd/csrc/dmath.h"]
PROFILE = os.path.join(ROOT, "profiles", "k_push_solve_push_plain_110592.txt")
PROFILE_TIMED = os.path.join(ROOT, "profiles", "k_push_solve_timed_push_plain_110592.txt")
PROFILE_FREE = os.path.join(ROOT, "profiles", "k_push_solve_free_118080.txt")
PROFILE_FREE_TIMED = os.path.join(ROOT, "profiles", "k_push_solve_free_timed_118080.txt")
FLIP_SOURCES = ["paper_2609_21803_amd/csrc/flip.hip", "paper_2609_21803_amd/csrc/dmath.h"]
PROFILE_FLIP = os.path.join(ROOT, "profiles", "k_flip_solve_flip_32768.txt")


def profiled_traffic(path=PROFILE, sources=KERNEL_SOURCES):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel sources changed after those counters were taken."""
    import hashlib
    if not os.path.exists(path):
        return None
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, s), "rb").read() for s in sources)).hexdigest()
    fields = {}
    for line in open(path):
        if ":" in line:
            k, v = line.split(":", 1)
            fields[k.strip()] = v.strip().split()[0] if v.strip() else ""
    if fields.get("source_sha256") != h:
        return None
    try:
        return float(fields["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(batch, seconds_target=15.0, timed=0):
    """Oracle (FP64, plain C, one sequence per thread over all host threads) on a
    strided sample of the workload; returns solves/s."""
    import oracle
    prm = oracle.Params(timed=timed)
    n_threads = os.cpu_count() or 1
    B = len(batch["nseg"])
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    n = 64 * n_threads
    # calibrate on a small strided sample, then size the timed sample to ~seconds_target
    idx = np.linspace(0, B - 1, n).astype(np.int64)
    sub = {k: v[idx] for k, v in batch.items()}
    t0 = time.perf_counter()
    oracle.evaluate(f32(sub["x0"]), f32(sub["goal"]), f32(sub["inst"]), sub["nseg"], sub["modes"], sub["knots"],
                    params=prm, nthreads=n_threads)
    dt = time.perf_counter() - t0
    n2 = int(min(B, max(n, n * seconds_target / max(dt, 1e-3))))
    idx = np.linspace(0, B - 1, n2).astype(np.int64)
    sub = {k: v[idx] for k, v in batch.items()}
    t0 = time.perf_counter()
    oracle.evaluate(f32(sub["x0"]), f32(sub["goal"]), f32(sub["inst"]), sub["nseg"], sub["modes"], sub["knots"],
                    params=prm, nthreads=n_threads)
    dt = time.perf_counter() - t0
    return dict(value=n2 / dt, unit="solves/s", cores=n_threads, kind="oracle", value_per_core=n2 / dt / n_threads,
                sample=f"{n2} of {B} TOs, evenly strided over the batch, FP64, {n_threads} threads, {dt:.1f} s")


def mlp_flops(B, dims, train):
    """Matrix-core flops of one forward (or forward + backward) pass over B samples."""
    layers = list(zip(dims[:-1], dims[1:]))
    f = sum(2.0 * B * k * n for k, n in layers)                  # forward products
    if train:
        f += sum(2.0 * B * k * n for k, n in layers)             # weight gradients
        f += sum(2.0 * B * k * n for k, n in layers[1:])         # input gradients (not for the input layer)
    return f


def flip_cpu_baseline(batch, seconds_target=10.0):
    """Flip oracle (FP64, plain C, one order per thread over all host threads) on an evenly
    strided sample of the flipping round; returns solves/s."""
    from oracle import flip as F
    n_threads = os.cpu_count() or 1
    B = len(batch["nseg"])
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)

    def run(n):
        idx = np.linspace(0, B - 1, n).astype(np.int64)
        sub = {k: v[idx] for k, v in batch.items()}
        t0 = time.perf_counter()
        F.evaluate(f32(sub["x0"]), f32(sub["goal"]), f32(sub["inst"]), sub["nseg"], sub["modes"], sub["knots"],
                   nthreads=n_threads)
        return time.perf_counter() - t0

    n = 4 * n_threads
    dt = run(n)
    n2 = int(min(B, max(n, n * seconds_target / max(dt, 1e-3))))
    dt = run(n2)
    return dict(value=n2 / dt, unit="solves/s", cores=n_threads, kind="oracle", value_per_core=n2 / dt / n_threads,
                sample=f"{n2} of {B} orders, evenly strided over the round, FP64, {n_threads} threads, {dt:.1f} s")


def flip_leg(native, I, torch, B=32768, cpu=True):
    """One round of the bimanual-flipping workload: B orders (K ~ U{1..6}, 10 intervals per
    segment) on 32 seeded start/goal pairs, one launch timed after one warm-up launch."""
    b = I.flip_batch(3100, B)
    ctx = native.Context(max_batch=B, max_intervals=60, task=native.TASK_FLIP)
    d = native.to_device(b)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = ctx.evaluate(**d)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms = ctx.kernel_ms()
    st = out["stats"].cpu().numpy()
    N = I.n_intervals(b).astype(np.float64)
    flops = float((st[:, 1] * N).sum()) * FLIP_FLOP_PER_INTERVAL_GN
    ach = flops / (kms * 1e-3) / 1e12
    res = {"workload": f"bimanual flipping: {B} orders, K ~ U{{1..6}}, 10 intervals per segment, 32 start/goal pairs "
                       "(goal th ~ U[pi/2, pi], px ~ U[-0.2, 0.2] m), AL<=20 x GN<=10, FP64",
           "value": B / (ms * 1e-3), "unit": "solves/s", "ms": ms, "mean_gn_iterations": float(st[:, 1].mean()),
           "mean_intervals": float(N.mean()), "feasible_fraction": float(out["feasible"].float().mean().item()),
           "roofline": {"bound": "alu", "kernel": "k_flip_solve", "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "kernel_ms": kms, "flop": flops,
                        "traffic": profiled_traffic(PROFILE_FLIP, FLIP_SOURCES)}}
    if cpu:
        res["cpu_baseline"] = flip_cpu_baseline(b)
    return res


def timed_leg(native, I, torch, cpu=True):
    """Pushing with optimised timing (interval durations as controls) on the headline
    workload's orders: one launch after a warm-up launch, then two more for the kernel
    average."""
    b = I.push_plain()
    B, N = len(b["nseg"]), 24
    ctx = native.Context(max_batch=B, max_segments=6, max_intervals=N, task=native.TASK_PUSH_TIMED)
    d = native.to_device(b)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()
    ctx.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = ctx.evaluate(**d)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    kms = [ctx.kernel_ms()]
    for _ in range(2):
        out = ctx.evaluate(**d)
        torch.cuda.synchronize()
        kms.append(ctx.kernel_ms())
    kms = float(np.mean(kms))
    st = out["stats"].cpu().numpy()
    flops = float((st[:, 1].astype(np.float64) * N).sum()) * TIMED_FLOP_PER_INTERVAL_GN + \
        float((st[:, 0].astype(np.float64) * N).sum()) * FLOP_PER_INTERVAL_AL
    ach = flops / (kms * 1e-3) / 1e12
    res = {"workload": "planar pushing with optimised timing (duration of every interval a control, "
                       "0.02 <= h <= 0.2 s, time weight 0.01): the headline's 110,592 orders, 24 intervals, "
                       "AL<=20 x GN<=10",
           "value": B / (ms * 1e-3), "unit": "solves/s", "ms": ms,
           "feasible_fraction": float(out["feasible"].float().mean().item()),
           "mean_gn_iterations": float(st[:, 1].mean()), "mean_al_iterations": float(st[:, 0].mean()),
           "roofline": {"bound": "alu", "kernel": "k_push_solve (timed)", "achieved": ach, "peak": PEAK_FP64_TFLOPS,
                        "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS, "kernel_ms": kms, "flop_per_launch": flops,
                        "traffic": profiled_traffic(PROFILE_TIMED), "peak_basis": PUSH_PEAK_BASIS,
                        "frac_of_fp32_peak": ach / PEAK_FP32_TFLOPS}}
    if cpu:
        res["cpu_baseline"] = cpu_baseline(b, seconds_target=10.0, timed=1)
    return res


def hetero_leg(native, I, torch, B=131072):
    """Heterogeneous batch (K ~ U{1..5}, 5..15 intervals per segment, up to 75 intervals):
    the persistent work queue with the orders in input order, in the default schedule
    (length-sorted queue) and in the autotuner's pick."""
    b = I.push_hetero(seed=2100, B=B)
    ctx = native.Context(max_batch=B, max_segments=6, max_intervals=75)
    d = native.to_device(b)
    out = ctx.evaluate(**d)
    torch.cuda.synchronize()

    def timed_runs():
        ms = []
        for _ in range(2):
            ctx.evaluate(**d)
            torch.cuda.synchronize()
            ms.append(ctx.kernel_ms())
        return ms

    default_ms = timed_runs()
    ctx.set_schedule(0, 0)
    input_order_ms = timed_runs()
    sched, tuned_ms = ctx.autotune(**d, out=out)
    best = []
    for _ in range(2):
        out = ctx.evaluate(**d)
        torch.cuda.synchronize()
        best.append(ctx.kernel_ms())
    st = out["stats"].cpu().numpy()
    N = I.n_intervals(b).astype(np.float64)
    return {"workload": f"pushing, heterogeneous: {B} orders, K ~ U{{1..5}}, 5..15 intervals per segment, "
                        "64 start/goal pairs (seed 2100)",
            "mean_intervals": float(N.mean()), "mean_gn_iterations": float(st[:, 1].mean()),
            "input_order": {"kernel_ms": float(np.mean(input_order_ms)),
                            "solves_per_s": B / (np.mean(input_order_ms) * 1e-3)},
            "default_schedule": {"kernel_ms": float(np.mean(default_ms)), "solves_per_s": B / (np.mean(default_ms) * 1e-3)},
            "autotuned_schedule": {"schedule": sched, "kernel_ms": float(np.mean(best)),
                                   "solves_per_s": B / (np.mean(best) * 1e-3)}}


def free_leg(native, I, torch, seeds=(5300, 5301, 5302, 5303), n_eval_inst=8, cpu=True, planner=True, timed=False):
    """Pushing with free motion: the Sec. III-A language at the paper's segment cap of eight
    (205,632 admissible orders, 14,760 of them of at most six segments), in the planner
    configurations of Sec. IV-A on the device, 50 intervals per order as the paper's
    transcription (split evenly over the segments, the remainder to the first ones): full enumeration
    (every admissible order in one batch), seed only (every order of at most six segments),
    and expansion with s_max = 1 and 3 rounds after that seed (r = 2, batches of up to
    16,384, at most 1,024 best-ranked orders expanded per round); and the ablations'
    uniform sampling and MCTS (pool 1,024) with a budget of 40,960 orders, about what three
    expansion rounds evaluate; refinement of the 256 best feasible orders.  Per goal: orders evaluated, device time of the whole search, time to
    the first feasible order, the plan, and whether it recovers the full enumeration's plan
    cost (within 1e-4).  Then the evaluator alone on every order of at most six segments for
    each of 8 instances (118,080 TOs), one launch timed after a warm-up, with its roofline,
    and the oracle's rate on a strided sample.  planner=False runs only the seed pass that
    lists the orders of at most six segments (two intervals per segment) before the
    evaluator launch.  timed=True: the same with optimised timing (the interval durations
    as controls with bounds, the paper's pushing transcription), the planner with the
    paper's budgets of that transcription (t_exp = 300 and t_ref = 1,500 iterations per
    candidate: at most 30 x 10 and 60 x 25 Gauss-Newton iterations), the evaluator launch
    with 50 intervals per order at the exploration budget of the other tasks."""
    full = 205632
    task = native.TASK_PUSH_FREE_TIMED if timed else native.TASK_PUSH_FREE
    budgets = native.SolverParams(al_max=30, gn_max=10, ref_al_max=60, ref_gn_max=25) if timed else None
    ctx = native.Context(max_batch=full, max_segments=8, max_intervals=80, task=task, params=budgets)
    common = dict(kcap=8, radius=2, knots_per_segment=0, n_total=50, k_ref=256)   # the paper's 50 knots per order
    configs = {"full_enumeration": native.ExpandParams(**common, seed_max_segments=8, rounds=0, frontier_W=1,
                                                         batch_B=full, eval_budget=full),
               "seed_only": native.ExpandParams(**common, seed_max_segments=6, rounds=0, frontier_W=1, batch_B=16384,
                                                eval_budget=16384),
               "expansion_smax1": native.ExpandParams(**common, seed_max_segments=6, rounds=1, frontier_W=1024,
                                                      batch_B=16384, eval_budget=full),
               "expansion_smax3": native.ExpandParams(**common, seed_max_segments=6, rounds=3, frontier_W=1024,
                                                      batch_B=16384, eval_budget=full),
               # the ablations' allocation policies at the budget of three expansion rounds
               "uniform_sampling": native.ExpandParams(**common, seed_max_segments=6, rounds=16, frontier_W=1,
                                                       batch_B=16384, eval_budget=40960,
                                                       policy=native.POLICY_UNIFORM, sample_seed=11,
                                                       sample_draws=32768),
               "mcts_p1024": native.ExpandParams(**common, seed_max_segments=6, rounds=0, frontier_W=1, batch_B=1024,
                                                 eval_budget=40960, policy=native.POLICY_MCTS, sample_seed=11)}
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    rows, seed6 = {k: [] for k in configs}, None
    if not planner:
        x0, goal, inst = I.push_free_pairs(seeds[0], 1)
        native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]),
                      native.ExpandParams(kcap=8, radius=1, knots_per_segment=2, k_ref=1, seed_max_segments=6, rounds=0,
                                          frontier_W=1, batch_B=16384, eval_budget=16384))
        torch.cuda.synchronize()
        seed6 = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
        configs, rows = {}, {}
    for name, prm in configs.items():
        for sd in seeds:
            x0, goal, inst = I.push_free_pairs(sd, 1)
            # one search per goal: its time (HIP events around the launch of the captured loop)
            # does not include graph capture and instantiation
            o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
            torch.cuda.synchronize()
            K = int(o["nseg"].item())
            if seed6 is None and name == "seed_only":
                seed6 = native.expand_trace(ctx)[0].cpu().numpy().view(np.uint64)
            rows[name].append({"seed": sd, "evaluated": st["evaluated"], "rounds": st["rounds_done"],
                               "feasible": st["n_feasible"], "device_ms": st["t_total_ms"],
                               "t_first_feasible_ms": st["t_first_feasible_ms"],
                               "plan": o["modes"].cpu().numpy()[:K].tolist(),
                               "plan_cost": float(o["cost"].item()) if K else None})
    ref = {r["seed"]: r["plan_cost"] for r in rows.get("full_enumeration", [])}
    summary = {}
    for name, rs in rows.items():
        for r in rs:
            J, Jf = r["plan_cost"], ref[r["seed"]]
            r["recovers_full_enumeration"] = bool(J is not None and Jf is not None and abs(J - Jf) <= 1e-4 * abs(Jf))
        summary[name] = {"recovered": f"{sum(r['recovers_full_enumeration'] for r in rs)}/{len(rs)}",
                         "median_evaluated": float(np.median([r["evaluated"] for r in rs])),
                         "median_device_ms": float(np.median([r["device_ms"] for r in rs]))}
    all_keys = seed6
    # the evaluator alone: every admissible order of at most six segments (the seed-only
    # configuration's evaluated set) on each of n_eval_inst instances
    n1 = len(all_keys)
    nseg1 = (all_keys >> np.uint64(60)).astype(np.int32)
    modes1 = np.zeros((n1, 6), np.int32)
    for i in range(6):   # free-motion keys: 4 bits per id below the segment count
        modes1[:, i] = ((all_keys >> np.uint64(56 - 4 * i)) & np.uint64(15)).astype(np.int32)
    modes1[np.arange(6)[None, :] >= nseg1[:, None]] = 0
    x0, goal, inst = I.push_free_pairs(5400, n_eval_inst)
    pair = np.repeat(np.arange(n_eval_inst), n1)
    nseg = np.tile(nseg1, n_eval_inst)
    if timed:   # 50 intervals per order, split evenly, the remainder to the first segments
        j = np.arange(6)[None, :]
        kn = np.where(j < nseg[:, None], 50 // nseg[:, None] + (j < (50 % nseg)[:, None]), 0).astype(np.int32)
    else:
        kn = np.where(np.arange(6)[None, :] < nseg[:, None], 10, 0).astype(np.int32)
    batch = dict(x0=x0[pair], goal=goal[pair], inst=inst[pair], nseg=nseg, modes=np.tile(modes1, (n_eval_inst, 1)),
                 knots=kn)
    n = len(nseg)
    ectx = native.Context(max_batch=n, max_segments=6, max_intervals=60, task=task)
    d = native.to_device(batch)
    ectx.evaluate(**d)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    out = ectx.evaluate(**d)
    e1.record()
    torch.cuda.synchronize()
    ms, kms = e0.elapsed_time(e1), ectx.kernel_ms()
    st = out["stats"].cpu().numpy()
    N = I.n_intervals(batch).astype(np.float64)
    fgn = FREE_TIMED_FLOP_PER_INTERVAL_GN if timed else FREE_FLOP_PER_INTERVAL_GN
    flops = float((st[:, 1] * N).sum()) * fgn + float((st[:, 0] * N).sum()) * FLOP_PER_INTERVAL_AL
    ach = flops / (kms * 1e-3) / 1e12
    res = {"workload": ("pushing with free motion and optimised timing" if timed else "pushing with free motion") +
                       " (16 mode ids, the Sec. III-A language capped at 8 segments: "
                       f"{full} admissible orders, {n1} of <= 6); planner configurations with 50 intervals per order "
                       f"on the goals of seeds {seeds[0]}..{seeds[-1]}; evaluator on all {n1} orders of <= 6 segments x "
                       f"{n_eval_inst} instances (seed 5400), " + ("50 intervals per order" if timed else
                                                                    "10 intervals per segment") +
                       ("; planner budgets t_exp = 300 (30 x 10), t_ref = 1,500 (60 x 25) Gauss-Newton iterations"
                        if timed else ""),
           "planner_summary": summary, "planner": rows,
           "evaluate": {"orders": n, "value": n / (ms * 1e-3), "unit": "solves/s", "ms": ms,
                        "mean_intervals": float(N.mean()), "mean_gn_iterations": float(st[:, 1].mean()),
                        "feasible_fraction": float(out["feasible"].float().mean().item()),
                        "roofline": {"bound": "alu", "kernel": "k_push_solve (free motion" +
                                     (", optimised timing)" if timed else ")"), "achieved": ach,
                                     "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": ach / PEAK_FP64_TFLOPS,
                                     "kernel_ms": kms, "flop_per_launch": flops,
                                     "traffic": profiled_traffic(PROFILE_FREE_TIMED if timed else PROFILE_FREE)}}}
    if cpu:
        res["evaluate"]["cpu_baseline"] = free_cpu_baseline(batch, timed=timed)
    return res


def free_cpu_baseline(batch, seconds_target=10.0, timed=False):
    """Free-motion oracle (FP64, plain C, one order per thread over all host threads) on an
    evenly strided sample of the batch; returns solves/s."""
    from oracle import free as F
    n_threads = os.cpu_count() or 1
    B = len(batch["nseg"])
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)

    def run(n):
        idx = np.linspace(0, B - 1, n).astype(np.int64)
        sub = {k: v[idx] for k, v in batch.items()}
        t0 = time.perf_counter()
        F.evaluate(f32(sub["x0"]), f32(sub["goal"]), f32(sub["inst"]), sub["nseg"], sub["modes"], sub["knots"],
                   nthreads=n_threads, timed=timed)
        return time.perf_counter() - t0

    n = 4 * n_threads
    dt = run(n)
    n2 = int(min(B, max(n, n * seconds_target / max(dt, 1e-3))))
    dt = run(n2)
    return dict(value=n2 / dt, unit="solves/s", cores=n_threads, kind="oracle", value_per_core=n2 / dt / n_threads,
                sample=f"{n2} of {B} orders, evenly strided over the batch, FP64, {n_threads} threads, {dt:.1f} s")


def expand_scale_leg(native, I, torch, seeds=(2000, 2001)):
    """The heterogeneous expansion at its configured scale, in the captured loop on the
    device: orders of 1..5 segments (10 intervals each), seed of all orders of at most two
    segments, two rounds of two-edit neighbourhoods (22,464 orders, then the frontier of the
    W = 4,096 best-ranked orders fills B = 131,072 children); per instance the orders evaluated, the device time of the
    whole loop (expansion, evaluation, refinement) and the orders evaluated per second."""
    W, B = 4096, 131072
    ctx = native.Context(max_batch=B, max_segments=6, max_intervals=50)
    prm = native.ExpandParams(kcap=5, seed_max_segments=2, radius=2, rounds=2, frontier_W=W, knots_per_segment=10,
                              k_ref=16, batch_B=B, eval_budget=400000)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    rows = []
    for sd in seeds:
        x0, goal, inst = I.push_pairs(sd, 1)
        native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)          # capture + warm-up
        torch.cuda.synchronize()
        o, st = native.expand(ctx, t(x0[0]), t(goal[0]), t(inst[0]), prm)
        torch.cuda.synchronize()
        K = int(o["nseg"].item())
        rows.append({"seed": sd, "evaluated": st["evaluated"], "rounds": st["rounds_done"],
                     "feasible": st["n_feasible"], "device_ms": st["t_total_ms"],
                     "orders_per_s": st["evaluated"] / (st["t_total_ms"] * 1e-3),
                     "t_first_feasible_ms": st["t_first_feasible_ms"], "plan": o["modes"].cpu().numpy()[:K].tolist(),
                     "plan_cost": float(o["cost"].item())})
    return {"workload": "pushing expansion: K <= 5, 10 intervals per segment, seed = all 156 orders of <= 2 segments, "
                        f"2 rounds, frontier W = {W}, batch B = {B}, r = 2, K_ref = 16 (goals of seeds 2000..)",
            "instances": rows}


def flip_expand_scale_leg(native, I, torch, n=2):
    """The flipping expansion at its configured scale: goals th ~ U[pi/2, pi], px ~ U[-0.2,
    0.2] m, orders of up to six segments (10 intervals each), 32,768 orders per round, an
    evaluation budget of 200,000, frontier W = 4,096; plans found (none is a result too),
    orders evaluated and device time per round."""
    B, W = 32768, 4096
    ctx = native.Context(max_batch=B, max_segments=6, max_intervals=60, task=native.TASK_FLIP)
    prm = native.ExpandParams(kcap=6, seed_max_segments=1, radius=1, rounds=6, frontier_W=W, knots_per_segment=10,
                              k_ref=16, batch_B=B, eval_budget=200000)
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()
    x0, goal, inst = I.flip_pairs(3000, n)
    rows = []
    for i in range(n):
        o, st = native.expand(ctx, t(x0[i]), t(goal[i]), t(inst[i]), prm)
        torch.cuda.synchronize()
        K = int(o["nseg"].item())
        rows.append({"goal": [float(goal[i, 0]), float(goal[i, 1])], "evaluated": st["evaluated"],
                     "rounds": st["rounds_done"], "feasible": st["n_feasible"], "device_ms": st["t_total_ms"],
                     "ms_per_round": st["t_total_ms"] / max(1, st["rounds_done"]),
                     "t_first_feasible_ms": st["t_first_feasible_ms"], "plan": o["modes"].cpu().numpy()[:K].tolist(),
                     "plan_cost": float(o["cost"].item()) if K else None})
    return {"workload": f"flipping expansion: goals th ~ U[pi/2, pi] (seed 3000), K <= 6, 10 intervals per segment, "
                        f"B = {B} per round, budget 200,000, W = {W}, r = 1",
            "plans_found": sum(1 for r in rows if r["plan"]), "instances": rows}


def learned_leg(native, I, torch):
    """Train the network on evaluator results, time training and inference, and compare the
    time to the first feasible plan of the plain and the learned expansion."""
    from paper_2609_21803_amd import learned
    t0 = time.perf_counter()
    data = learned.generate(2097152, seed=4000)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    mlp = native.MLP(max_batch=131072, seed=1)
    dims = [mlp.in_dim] + [mlp.hidden] * mlp.layers + [mlp.out_dim]
    steps, batch = 1500, 8192
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    # time the bare training steps on one resident minibatch, then train on the data
    idx = torch.arange(batch, device="cuda")
    mb = [data[k].index_select(0, idx).contiguous() for k in ("X", "y_feas", "y_cost", "y_traj", "mask")]
    for _ in range(3):
        mlp.train_step(*mb, lr=0.0)
    e0.record()
    for _ in range(50):
        mlp.train_step(*mb, lr=0.0)
    e1.record()
    torch.cuda.synchronize()
    step_ms = e0.elapsed_time(e1) / 50
    mlp.set_params(native.MLP(max_batch=16, seed=1).get_params())       # fresh weights and optimiser state
    t0 = time.perf_counter()
    log = learned.train(mlp, data, steps=steps, batch=batch, lr=1e-3, log_every=steps - 1)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    Bf = 131072
    xf = data["X"][:Bf].contiguous()
    mlp.forward(xf)
    e0.record()
    for _ in range(10):
        mlp.forward(xf)
    e1.record()
    torch.cuda.synchronize()
    fwd_ms = e0.elapsed_time(e1) / 10
    prm = native.ExpandParams(kcap=3, seed_max_segments=2, radius=1, rounds=2, frontier_W=4096, knots_per_segment=8,
                              k_ref=64, batch_B=16384, eval_budget=20000, learned_warm=1)
    ctx = native.Context(max_batch=16384, max_segments=6, max_intervals=24)
    x0, goal, inst = I.push_pairs(9100, 8)
    rows = learned.compare(ctx, mlp, prm, list(zip(x0, goal, inst)), trace=True)
    # D6: feasibility ranking of the evaluated orders, network logit vs the plain planner's
    # evaluation order (earlier = ranked better), against the evaluator's flags
    auc_net, auc_plain = [], []
    for r, a, g, m in zip(rows, x0, goal, inst):
        k, J, v = r["plain"].pop("trace")
        feas = v <= 1e-5
        auc_net.append(learned.feasibility_auc(mlp, k, feas, a, g, m, 8))
        auc_plain.append(learned.auc(-np.arange(len(v), dtype=np.float64), feas))
    held = I.push_hetero(seed=4900, B=65536)
    wctx = native.Context(max_batch=65536, max_segments=6, max_intervals=75)
    savings = learned.warm_start_savings(wctx, mlp, held)
    tp = [r["plain"]["t_first_ms"] for r in rows]
    tl = [r["learned"]["t_first_ms"] for r in rows]
    same = sum(r["plain"]["modes"] == r["learned"]["modes"] and
               abs(r["plain"]["cost"] - r["learned"]["cost"]) <= 1e-4 * max(abs(r["plain"]["cost"]), 1e-12)
               for r in rows)
    tr_fl = mlp_flops(batch, dims, True)
    fw_fl = mlp_flops(Bf, dims, False)
    tr_tf = tr_fl / (step_ms * 1e-3) / 1e12
    return {
        "ttfp_ms_plain_median": float(np.median(tp)), "ttfp_ms_learned_median": float(np.median(tl)),
        "ttfp_ratio_median": float(np.median(np.array(tl) / np.array(tp))),
        "same_returned_plan": f"{same}/{len(rows)}",
        "first_feasible_index_median": {"plain": float(np.median([r["plain"]["first_index"] for r in rows])),
                                        "learned": float(np.median([r["learned"]["first_index"] for r in rows]))},
        "instances": "8 held-out pushing start/goal pairs (seed 9100), K<=3, 8 intervals per segment, "
                     "2 rounds, batch 16,384, budget 20,000",
        "feasibility_auc": {"network_median": float(np.nanmedian(auc_net)),
                            "plain_order_median": float(np.nanmedian(auc_plain)),
                            "per_instance_network": auc_net, "per_instance_plain_order": auc_plain,
                            "over": "every order the plain expansion evaluated on each held-out instance"},
        "warm_start_gn": {**savings, "batch": "65,536 held-out ragged orders (seed 4900), K ~ U{1..5}, "
                                              "5..15 intervals per segment"},
        "training": {"samples": int(data["X"].shape[0]), "steps": steps, "batch": batch, "gen_s": t_gen,
                     "train_s": t_train, "final_loss": log[-1][1]},
        "roofline": {"bound": "mfma", "kernel": "train step (k_gemm x 14 + loss, reductions, AdamW)",
                     "achieved": tr_tf, "peak": PEAK_BF16_TFLOPS, "unit": "TFLOP/s", "frac": tr_tf / PEAK_BF16_TFLOPS,
                     "ms": step_ms, "flop": tr_fl},
        "inference": {"batch": Bf, "ms": fwd_ms, "achieved": fw_fl / (fwd_ms * 1e-3) / 1e12, "peak": PEAK_BF16_TFLOPS,
                      "unit": "TFLOP/s"},
    }


def learned_flip_leg(native, I, torch):
    """The learned proposal on flipping: train a network on flipping evaluator results and
    compare the plain and the learned expansion of one batch of all admissible one- and
    two-segment orders on held-out pivot-reachable goals."""
    from paper_2609_21803_amd import learned
    t0 = time.perf_counter()
    ctx = native.Context(max_batch=32768, max_segments=6, max_intervals=20, task=native.TASK_FLIP)
    data = learned.generate_flip(96, seed=5000, ctx=ctx)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    mlp = native.MLP(max_batch=8192, seed=1)
    t0 = time.perf_counter()
    log = learned.train(mlp, data, steps=800, batch=8192, lr=1e-3, log_every=799)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    prm = native.ExpandParams(kcap=2, seed_max_segments=2, radius=1, rounds=0, frontier_W=8, knots_per_segment=10,
                              k_ref=16, batch_B=8192, eval_budget=8192, learned_warm=1)
    ctx2 = native.Context(max_batch=8192, max_segments=6, max_intervals=20, task=native.TASK_FLIP)
    rows = learned.compare(ctx2, mlp, prm, list(zip(*I.flip_pivot_pairs(9400, 8))))
    tp = np.array([r["plain"]["t_first_ms"] for r in rows])
    tl = np.array([r["learned"]["t_first_ms"] for r in rows])
    ok = (tp > 0) & (tl > 0)
    same_cost = sum(abs(r["plain"]["cost"] - r["learned"]["cost"]) <= 1e-4 * max(abs(r["plain"]["cost"]), 1e-12)
                    for r in rows)
    return {
        "ttfp_ms_plain_median": float(np.median(tp[ok])) if ok.any() else None,
        "ttfp_ms_learned_median": float(np.median(tl[ok])) if ok.any() else None,
        "ttfp_ratio_median": float(np.median(tl[ok] / tp[ok])) if ok.any() else None,
        "same_returned_cost": f"{same_cost}/{len(rows)}",
        "identical_returned_orders": f"{sum(r['plain']['modes'] == r['learned']['modes'] for r in rows)}/{len(rows)}",
        "first_feasible_index_median": {"plain": float(np.median([r["plain"]["first_index"] for r in rows])),
                                        "learned": float(np.median([r["learned"]["first_index"] for r in rows]))},
        "instances": "8 held-out pivot-reachable flipping goals (seed 9400, th ~ U[0.9, 1.5]), one batch of the "
                     "8,192 first admissible orders of 1-2 segments, 10 intervals per segment, refinement of 16",
        "training": {"samples": int(data["X"].shape[0]), "feasible_fraction": float(data["y_feas"].mean()),
                     "steps": 800, "batch": 8192, "gen_s": t_gen, "train_s": t_train, "final_loss": log[-1][1]},
    }


def learned_free_leg(native, I, torch, timed=False):
    """The learned proposal on pushing with free motion: train a network on the evaluator's
    results of uniformly sampled admissible orders (cap 8, 50 intervals per order) and
    compare the plain and the learned expansion in the paper's s_max = 1 configuration on
    the free leg's four goals (held out from training).  timed=True: the paper's
    transcription (optimised timing) with its budgets (30 x 10 and 60 x 25 Gauss-Newton
    iterations), for the training data as for the searches."""
    from paper_2609_21803_amd import learned
    task = native.TASK_PUSH_FREE_TIMED if timed else native.TASK_PUSH_FREE
    budgets = native.SolverParams(al_max=30, gn_max=10, ref_al_max=60, ref_gn_max=25) if timed else None
    t0 = time.perf_counter()
    gen = native.Context(max_batch=16384, max_segments=8, max_intervals=50, task=task, params=budgets)
    data = learned.generate_free(16, 16384, seed=6000, ctx=gen, kcap=8, n_total=50)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    in_dim, out_dim = native.mlp_dims(task)
    mlp = native.MLP(max_batch=16384, seed=1, in_dim=in_dim, out_dim=out_dim)
    t0 = time.perf_counter()
    log = learned.train(mlp, data, steps=800, batch=8192, lr=1e-3, log_every=799)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    prm = native.ExpandParams(kcap=8, radius=2, knots_per_segment=0, n_total=50, k_ref=256, seed_max_segments=6,
                              rounds=1, frontier_W=1024, batch_B=16384, eval_budget=205632, learned_warm=1)
    ctx = native.Context(max_batch=16384, max_segments=8, max_intervals=50, task=task, params=budgets)
    pairs = [tuple(a[0] for a in I.push_free_pairs(sd, 1)) for sd in range(5300, 5304)]
    rows = learned.compare(ctx, mlp, prm, pairs, trace=True)
    auc_net, auc_plain = [], []
    for r, (a, g, m) in zip(rows, pairs):
        k, J, v = r["plain"].pop("trace")
        feas = v <= 1e-5
        auc_net.append(learned.feasibility_auc(mlp, k, feas, a, g, m, 0, task=task, n_total=50))
        auc_plain.append(learned.auc(-np.arange(len(v), dtype=np.float64), feas))
    tp = np.array([r["plain"]["t_first_ms"] for r in rows])
    tl = np.array([r["learned"]["t_first_ms"] for r in rows])
    ok = (tp > 0) & (tl > 0)
    same_cost = sum(abs(r["plain"]["cost"] - r["learned"]["cost"]) <= 1e-4 * max(abs(r["plain"]["cost"]), 1e-12)
                    for r in rows)
    return {
        "ttfp_ms_plain_median": float(np.median(tp[ok])) if ok.any() else None,
        "ttfp_ms_learned_median": float(np.median(tl[ok])) if ok.any() else None,
        "ttfp_ratio_median": float(np.median(tl[ok] / tp[ok])) if ok.any() else None,
        "search_ms_median": {"plain": float(np.median([r["plain"]["t_total_ms"] for r in rows])),
                             "learned": float(np.median([r["learned"]["t_total_ms"] for r in rows]))},
        "same_returned_cost": f"{same_cost}/{len(rows)}",
        "learned_cost_minus_plain": [r["learned"]["cost"] - r["plain"]["cost"] for r in rows],
        "first_feasible_index_median": {"plain": float(np.median([r["plain"]["first_index"] for r in rows])),
                                        "learned": float(np.median([r["learned"]["first_index"] for r in rows]))},
        "feasibility_auc": {"network_median": float(np.nanmedian(auc_net)),
                            "plain_order_median": float(np.nanmedian(auc_plain)),
                            "over": "every order the plain expansion evaluated on each goal"},
        "instances": "the free leg's goals (seeds 5300-5303), cap 8, seed <= 6 segments, one round of two-edit "
                     "neighbours (W = 1,024, batches of 16,384), 50 intervals per order, refinement of 256" +
                     ("; optimised timing, budgets 30 x 10 and 60 x 25 Gauss-Newton iterations" if timed else ""),
        "training": {"samples": int(data["X"].shape[0]), "feasible_fraction": float(data["y_feas"].mean()),
                     "sampling": "16 goals (seed 6000), 16,384 distinct orders each from the uniform sampler",
                     "steps": 800, "batch": 8192, "gen_s": t_gen, "train_s": t_train, "final_loss": log[-1][1]},
    }


def policy_leg(native, I, torch):
    """Allocation policies on the same evaluator at equal evaluation budgets: Alg. 1's
    expansion vs uniform sampling without replacement (the baseline of Sec. IV-B), time to the
    first feasible plan, plans found and returned cost."""
    t = lambda a: torch.as_tensor(np.asarray(a, np.float32)).cuda()

    def run(ctx, pairs, prm):
        rows = []
        for x0, goal, inst in pairs:
            o, st = native.expand(ctx, t(x0), t(goal), t(inst), prm)
            torch.cuda.synchronize()
            rows.append((int(o["nseg"].item()), float(o["cost"].item()), st))
        return rows

    def summary(rows):
        found = [r for r in rows if r[0] > 0]
        tf = [r[2]["t_first_feasible_ms"] for r in rows if r[2]["t_first_feasible_ms"] > 0]
        return {"plans_found": f"{len(found)}/{len(rows)}",
                "ttfp_ms_median": float(np.median(tf)) if tf else None,
                "first_feasible_index_median": float(np.median([r[2]["first_feasible_index"] for r in rows
                                                               if r[2]["first_feasible_index"] > 0] or [0])),
                "feasible_evaluated_median": float(np.median([r[2]["n_feasible"] for r in rows])),
                "evaluated_median": float(np.median([r[2]["evaluated"] for r in rows])),
                "cost": [r[1] if r[0] > 0 else None for r in rows]}

    out = {}
    # flipping: 8 pivot-reachable goals, two-segment cap, budget 2,400
    ctx = native.Context(max_batch=2048, max_segments=6, max_intervals=20, task=native.TASK_FLIP)
    pairs = list(zip(*I.flip_pivot_pairs(9400, 8)))
    common = dict(kcap=2, knots_per_segment=10, k_ref=16, batch_B=2048, eval_budget=2400)
    e = run(ctx, pairs, native.ExpandParams(**common, seed_max_segments=1, radius=1, rounds=1, frontier_W=8))
    u = run(ctx, pairs, native.ExpandParams(**common, rounds=1, policy=native.POLICY_UNIFORM, sample_seed=1,
                                            sample_draws=65536))
    m = run(ctx, pairs, native.ExpandParams(**{**common, "batch_B": 256}, policy=native.POLICY_MCTS, sample_seed=1))
    out["flip"] = {"instances": "8 pivot-reachable flipping goals (seed 9400), K <= 2, 10 intervals per segment, "
                                "batch 2,048 (MCTS pool 256), budget 2,400 evaluations, refinement of 16",
                   "expansion": summary(e), "uniform": summary(u), "mcts_P256": summary(m)}
    # pushing: 8 start/goal pairs, four-segment cap (22,620 orders), budget 8,000
    ctx = native.Context(max_batch=4096, max_segments=6, max_intervals=24)
    pairs = list(zip(*I.push_pairs(9100, 8)))
    common = dict(kcap=4, knots_per_segment=6, k_ref=64, batch_B=4096, eval_budget=8000)
    e = run(ctx, pairs, native.ExpandParams(**common, seed_max_segments=2, radius=1, rounds=2, frontier_W=4096))
    u = run(ctx, pairs, native.ExpandParams(**common, rounds=2, policy=native.POLICY_UNIFORM, sample_seed=1,
                                            sample_draws=131072))
    m = run(ctx, pairs, native.ExpandParams(**{**common, "batch_B": 1024}, policy=native.POLICY_MCTS, sample_seed=1))
    out["push"] = {"instances": "8 pushing start/goal pairs (seed 9100), K <= 4 (22,620 orders), 6 intervals per "
                                "segment, batch 4,096 (MCTS pool 1,024), budget 8,000 evaluations, refinement of 64",
                   "expansion": summary(e), "uniform": summary(u), "mcts_P1024": summary(m)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-proposal leg")
    ap.add_argument("--no-flip", action="store_true", help="skip the flipping leg")
    ap.add_argument("--no-hetero", action="store_true", help="skip the heterogeneous-batch leg")
    ap.add_argument("--no-policies", action="store_true", help="skip the allocation-policy comparison")
    ap.add_argument("--no-timed", action="store_true", help="skip the optimised-timing pushing leg")
    ap.add_argument("--no-scale", action="store_true", help="skip the expansion legs at the configured scale")
    ap.add_argument("--no-free", action="store_true", help="skip the free-motion pushing leg")
    ap.add_argument("--no-free-timed", action="store_true", help="skip the free-motion leg with optimised timing")
    ap.add_argument("--no-free-planner", action="store_true",
                    help="free-motion leg: the evaluator launch only, not the four planner configurations")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run one 256 MiB device-to-device copy (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the evaluator runs on a single MI355X "
              "(multi-GPU sharding is a design note, not built).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2609_21803_amd import instances as I
    from paper_2609_21803_amd import native

    torch.cuda.set_device(0)
    peaks = native.probe_peaks()        # the device's measured rates, beside the published peaks
    batch = I.push_plain()
    B = len(batch["nseg"])
    N = 24
    ctx = native.Context(max_batch=B, max_segments=6, max_intervals=N)
    d = native.to_device(batch)
    out = dict(cost=torch.empty(B, device="cuda"), viol=torch.empty(B, device="cuda"),
               feasible=torch.empty(B, dtype=torch.uint8, device="cuda"),
               traj=torch.empty((B, N + 1, 7), device="cuda"), stats=torch.empty((B, 4), dtype=torch.int32, device="cuda"))
    for _ in range(args.warmup):
        ctx.evaluate(**d, **out)
    torch.cuda.synchronize()
    ctx.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    kern_ms = []
    torch.cuda.synchronize()
    e0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.evaluate(**d, **out)
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / max(args.steps, 1)
    kern_ms.append(ctx.kernel_ms())          # kernel of the last step, HIP events in the library
    # one more step with per-launch kernel timing for the roofline average
    for _ in range(2):
        ctx.evaluate(**d, **out)
        torch.cuda.synchronize()
        kern_ms.append(ctx.kernel_ms())
    if args.copy_probe:
        src = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
    stats = out["stats"].cpu().numpy()
    feas = out["feasible"].cpu().numpy()
    gn_units = float((stats[:, 1].astype(np.float64) * N).sum())
    al_units = float((stats[:, 0].astype(np.float64) * N).sum())
    flops = gn_units * FLOP_PER_INTERVAL_GN + al_units * FLOP_PER_INTERVAL_AL
    kms = float(np.mean(kern_ms))
    achieved = flops / (kms * 1e-3) / 1e12
    solves_per_s = B / (ms * 1e-3)
    res = {
        "metric": "mode-TO solves/s at viol<=1e-5",
        "value": solves_per_s,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",   # FP64 arithmetic (96.5 % of executed flops), FP32 storage of gains, steps, multipliers
        "data": "synthetic",
        "config": {"workload": "planar pushing: 64 seeded start/goal pairs x all 1,728 three-segment contact-mode "
                               "orders, 8+8+8 intervals (110,592 TOs), AL<=20 x GN<=10",
                   "batch": B, "intervals": N, "parallelism": "single GPU"},
        "feasible_fraction": float(feas.mean()),
        "feasible_solves_per_s": float(feas.sum()) / (ms * 1e-3),
        "mean_gn_iterations": float(stats[:, 1].mean()),
        "mean_al_iterations": float(stats[:, 0].mean()),
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": profiled_traffic(),
                     "kernel": "k_push_solve", "kernel_ms": kms, "flop_per_launch": flops,
                     "peak_basis": PUSH_PEAK_BASIS, "frac_of_fp32_peak": achieved / PEAK_FP32_TFLOPS,
                     "hbm_gbs": (profiled_traffic() / (kms * 1e-3) / 1e9) if profiled_traffic() else None},
        "gn_histogram": {"bin_edges": list(range(0, 221, 20)),
                         "counts": np.histogram(stats[:, 1], bins=list(range(0, 221, 20)))[0].tolist()},
        "al_histogram": {"al_iterations": list(range(1, 21)),
                         "counts": np.bincount(np.clip(stats[:, 0], 0, 20), minlength=21)[1:].tolist()},
        "peaks_measured": {**peaks, "note": "microbenchmarks on this device (non-packed FP32 FMA chains, FP64 FMA "
                                            "chains, register-resident BF16 matrix-core products, 1 GiB copy); "
                                            "published: FP32 157.3, FP64 78.6, dense BF16 2500 TFLOP/s, "
                                            "HBM 8000 GB/s"},
        "wall_s_timed": wall,
    }
    print(f"[bench] pushing: {ms:.2f} ms/step", file=sys.stderr, flush=True)
    legs = [("timed", not args.no_timed, lambda: timed_leg(native, I, torch, cpu=not args.no_cpu)),
            ("hetero", not args.no_hetero, lambda: hetero_leg(native, I, torch)),
            ("flip", not args.no_flip, lambda: flip_leg(native, I, torch, cpu=not args.no_cpu)),
            ("policies", not args.no_policies, lambda: policy_leg(native, I, torch)),
            ("expand_scale", not args.no_scale, lambda: expand_scale_leg(native, I, torch)),
            ("flip_expand_scale", not args.no_scale, lambda: flip_expand_scale_leg(native, I, torch)),
            ("free", not args.no_free, lambda: free_leg(native, I, torch, cpu=not args.no_cpu,
                                                        planner=not args.no_free_planner)),
            ("free_timed", not args.no_free_timed, lambda: free_leg(native, I, torch, cpu=not args.no_cpu,
                                                                    planner=not args.no_free_planner, timed=True)),
            ("learned", not args.no_learned, lambda: learned_leg(native, I, torch)),
            ("learned_flip", not args.no_learned, lambda: learned_flip_leg(native, I, torch)),
            ("learned_free", not args.no_learned and not args.no_free,
             lambda: learned_free_leg(native, I, torch)),
            ("learned_free_timed", not args.no_learned and not args.no_free_timed,
             lambda: learned_free_leg(native, I, torch, timed=True)),
            ("cpu_baseline", not args.no_cpu, lambda: cpu_baseline(batch))]
    for name, on, run in legs:
        if on:
            t = time.perf_counter()
            res[name] = run()
            print(f"[bench] {name} leg done in {time.perf_counter() - t:.1f} s", file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
