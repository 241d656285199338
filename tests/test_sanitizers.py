"""CPU sanitizer runs of the host code: the FP64 oracles (threaded evaluation and the
greedy expansion; for free motion, in both of its builds, the seed and a batch step) under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer, and the library's host MCTS search (mcts_tree.h) under the same, each on
a small workload.  The sanitized builds must run clean (any report makes the process exit
non-zero) and give the results of the plain builds bit for bit; the host MCTS search
must select the oracle's orders, batch after batch, for a synthetic evaluator.

CPU only: the GPU kernels are not built with sanitizers (host code only).
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = os.path.join(HERE, "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=23",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1:exitcode=24", TSAN_OPTIONS="halt_on_error=1:exitcode=25")
MODES = {"asan": ["-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"],
         "tsan": ["-fsanitize=thread"]}


def _build_oracle(tmp, task, mode):
    exe = os.path.join(tmp, f"oracle_{task}_{mode}")
    defs = {"free_timed": ["-DFREE", "-DFREE_TIMED"], "push_timed": ["-DPUSH", "-DPUSH_TIMED"]}.get(
        task, [f"-D{task.upper()}"])
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-std=gnu11", "-pthread",
           *defs, *MODES[mode], "-o", exe, os.path.join(SAN, "oracle_driver.c"), "-lm"]
    subprocess.check_call(cmd)
    return exe


def _write(path, b, nthreads, expand, nmax):
    B = len(b["nseg"])
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    with open(path, "wb") as f:
        np.array([B], np.int64).tofile(f)
        np.array([6, nmax, nthreads, expand], np.int32).tofile(f)
        for k in ("x0", "goal", "inst"):
            np.ascontiguousarray(f32(b[k])).tofile(f)
        for k in ("nseg", "modes", "knots"):
            np.ascontiguousarray(b[k], np.int32).tofile(f)


def _read_free(path, B):
    raw = open(path, "rb").read()
    o = 8 * B + 8 * B + B + 16 * B
    out = _read(path, B, 0)
    n = int(np.frombuffer(raw, np.int64, 1, o)[0]); o += 8
    out["seed"] = np.frombuffer(raw, np.uint64, n, o); o += 8 * n
    m = int(np.frombuffer(raw, np.int64, 1, o)[0]); o += 8
    out["batch"] = np.frombuffer(raw, np.uint64, m, o)
    return out


@pytest.mark.parametrize("mode", ["asan", "tsan"])
@pytest.mark.parametrize("timed", [False, True])
def test_free_oracle_runs_clean_under_sanitizers(tmp_path, timed, mode):
    """The free-motion oracle (both builds): threaded evaluation of admissible orders of up
    to four segments, the seed enumeration and one batch-construction step, bit for bit
    the plain build's results."""
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    from oracle import free as F
    exe = _build_oracle(str(tmp_path), "free_timed" if timed else "free", mode)
    keys = F.seed(4)
    rng = np.random.default_rng(41 + timed)
    pick = rng.choice(len(keys), 40, replace=False)
    x0, goal, inst = I.push_free_pairs(8100 + timed, 4)
    orders = [F.key_modes(int(keys[p])) for p in pick]
    kn = [[3] * len(o) for o in orders]
    b = I.orders_batch(x0, goal, inst, np.arange(40) % 4, orders, kn)
    nmax = 12
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write(inp, b, nthreads=4, expand=1, nmax=nmax)
    r = subprocess.run([exe, inp, out], env=ENV, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    got = _read_free(out, 40)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    ref = F.evaluate(f32(b["x0"]), f32(b["goal"]), f32(b["inst"]), b["nseg"], b["modes"], b["knots"], nmax=nmax,
                     timed=timed)
    for k in ("cost", "viol", "feasible", "stats"):
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    assert np.array_equal(got["seed"], keys)
    merit = (np.arange(len(keys)) * 7919 % 1000) / 1000.0
    assert np.array_equal(got["batch"], F.expand_next(keys, merit, 6, 2, 16, 4096))
    assert len(got["batch"]) > 0


def _read(path, B, expand):
    raw = open(path, "rb").read()
    o = 0
    cost = np.frombuffer(raw, np.float64, B, o); o += 8 * B
    viol = np.frombuffer(raw, np.float64, B, o); o += 8 * B
    feas = np.frombuffer(raw, np.uint8, B, o); o += B
    stats = np.frombuffer(raw, np.int32, 4 * B, o).reshape(B, 4); o += 16 * B
    out = dict(cost=cost, viol=viol, feasible=feas, stats=stats)
    if expand:
        out["key"] = int(np.frombuffer(raw, np.uint64, 1, o)[0]); o += 8
        out["J"], out["v"] = np.frombuffer(raw, np.float64, 2, o); o += 16
        out["ctr"] = np.frombuffer(raw, np.int64, 4, o)
    return out


@pytest.mark.parametrize("mode", ["asan", "tsan"])
@pytest.mark.parametrize("task", ["push", "push_timed", "flip"])
def test_oracle_runs_clean_under_sanitizers(orc, tmp_path, task, mode):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = _build_oracle(str(tmp_path), task, mode)
    if task.startswith("push"):
        b = I.subset(I.push_tiny(), np.arange(0, 1152, 9))
        nmax = 10
    else:
        b = I.flip_tiny(B=48)
        nmax = 15
    inp, out = str(tmp_path / "in.bin"), str(tmp_path / "out.bin")
    _write(inp, b, nthreads=4, expand=1, nmax=nmax)
    r = subprocess.run([exe, inp, out], env=ENV, capture_output=True, text=True, timeout=900)
    assert r.returncode == 0, r.stderr[-4000:]
    got = _read(out, len(b["nseg"]), 1)
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    if task.startswith("push"):
        prm = orc.Params(timed=int(task == "push_timed"))
        ref = orc.evaluate(f32(b["x0"]), f32(b["goal"]), f32(b["inst"]), b["nseg"], b["modes"], b["knots"], nmax=nmax,
                           params=prm)
        ep = orc.Expand(kcap=2, seed_max_segments=1, radius=2, rounds=1, frontier_W=8, knots_per_segment=5, k_ref=4,
                        n_total=0, batch_B=300, eval_budget=900)
        e = orc.expand(f32(b["x0"])[0], f32(b["goal"])[0], f32(b["inst"])[0, 0], ep, params=prm)
        ekey, eJ, ectr = e["best_key"], e["best_cost"], [e["evaluated"], e["rounds"], e["n_feasible"],
                                                          e["first_feasible"]]
    else:
        from oracle import flip as F
        ref = F.evaluate(f32(b["x0"]), f32(b["goal"]), f32(b["inst"]), b["nseg"], b["modes"], b["knots"], nmax=nmax)
        ep = orc.Expand(kcap=2, seed_max_segments=1, radius=2, rounds=1, frontier_W=8, knots_per_segment=5, k_ref=4,
                        n_total=0, batch_B=300, eval_budget=900)
        ekey, eJ, ev, ectr, *_ = F.expand(f32(b["x0"])[0], f32(b["goal"])[0], float(f32(b["inst"])[0, 0]), ep)
        ectr = list(ectr)
    for k in ("cost", "viol", "feasible", "stats"):
        assert np.array_equal(got[k], ref[k], equal_nan=True), k
    assert got["key"] == ekey and (got["J"] == eJ or (np.isnan(got["J"]) and np.isnan(eJ)))
    assert list(got["ctr"]) == list(ectr)


def _fmix(h):
    m = (1 << 64) - 1
    h ^= h >> 33
    h = (h * 0xff51afd7ed558ccd) & m
    h ^= h >> 33
    h = (h * 0xc4ceb9fe1a85ec53) & m
    h ^= h >> 33
    return h


def _synthetic(keys, refine):
    J, v = [], []
    for k in keys:
        h = _fmix(int(k))
        J.append(0.1 + (h % 10007) / 10007.0)
        v.append(0.0 if (h >> 20) % 3 == 0 else ((h >> 32) % 1000) * 1e-5)
    return np.array(J), np.array(v)


@pytest.mark.parametrize("mode", ["asan", "tsan"])
def test_host_mcts_search_runs_clean_and_matches_oracle(tmp_path, mode):
    """The library's host MCTS search, built alone for the CPU with sanitizers, evaluates the
    same orders in the same order as the oracle's search for one synthetic evaluator."""
    from oracle import mcts as T
    exe = str(tmp_path / f"mcts_{mode}")
    cmd = [HIPCC, "--offload-host-only", "-O1", "-g", "-std=c++17"]
    for flag in MODES[mode]:
        cmd += ["-Xarch_host", flag]
    cmd += ["-o", exe, os.path.join(SAN, "mcts_driver.hip")]
    subprocess.check_call(cmd)
    for task, kcap, P, budget, seed in [(0, 3, 64, 900, 7), (0, 4, 200, 1500, 2), (1, 2, 128, 700, 3)]:
        r = subprocess.run([exe, str(task), str(kcap), str(P), str(budget), str(seed)], env=ENV, capture_output=True,
                           text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        lines = r.stdout.split()
        got = [int(x) for x in r.stdout.splitlines() if not x.startswith("batches")]
        _, _, _, keys, _, _, nb, _ = T.mcts_search(task, None, None, None, kcap, P, budget, seed, 5, 4,
                                                   evaluate=_synthetic)
        assert got == [int(k) for k in keys], (task, len(got), len(keys))
        assert int(lines[-1]) == nb
