"""Whole benchmark launches against the oracles, sequence by sequence under the parity rule
of tests/parity.py: the flipping round (32,768 orders, up to 60 intervals) and the timed
pushing launch (110,592 orders, 24 intervals).  The oracles take about 2.5 and 2 minutes on
16 threads, so this is a script, run by hand on a GPU machine:
python tests/full_parity_flip_timed.py [flip|timed]."""
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
sys.path.insert(0, HERE)
import numpy as np
import torch

import oracle
import parity
from paper_2609_21803_amd import instances as I
from paper_2609_21803_amd import native

f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)


def chunked(run, b, n_chunks=16):
    n, parts, t0 = len(b["nseg"]), [], time.time()
    step = (n + n_chunks - 1) // n_chunks
    for c0 in range(0, n, step):
        parts.append(run(I.subset(b, np.arange(c0, min(n, c0 + step)))))
        print(f"  oracle {min(n, c0 + step)}/{n} after {time.time() - t0:.0f} s", flush=True)
    return {k: np.concatenate([p[k] for p in parts]) for k in ("cost", "viol", "feasible", "stats")}


def flip():
    from oracle import flip as F
    b = I.flip_batch(3100, 32768)
    ctx = native.Context(max_batch=32768, max_intervals=60, task=native.TASK_FLIP)
    print("step: flip launch", flush=True)
    out = ctx.evaluate(**native.to_device(b), want_traj=False)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    ev = lambda s, **kw: F.evaluate(f32(s["x0"]), f32(s["goal"]), f32(s["inst"]), s["nseg"], s["modes"], s["knots"],
                                    nmax=60, **kw)
    o = chunked(ev, b)
    # the flipping evaluator is FP64 throughout: input draws only
    parity.check(g, o, b, lambda s, rows, r32: ev(s), "flip, all 32,768")


def timed():
    b = I.push_plain()
    ctx = native.Context(max_batch=len(b["nseg"]), max_segments=6, max_intervals=24, task=native.TASK_PUSH_TIMED)
    print("step: timed launch", flush=True)
    out = ctx.evaluate(**native.to_device(b), want_traj=False)
    torch.cuda.synchronize()
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    ev = lambda s, r32=0: oracle.evaluate(f32(s["x0"]), f32(s["goal"]), f32(s["inst"]), s["nseg"], s["modes"],
                                          s["knots"], params=oracle.Params(timed=1, round32=r32), nmax=24)
    o = chunked(ev, b)
    parity.check(g, o, b, lambda s, rows, r32: ev(s, r32), "timed, all 110,592", round32=1 | 2 | 4 | 8, allow=2e-3)


if __name__ == "__main__":
    which = sys.argv[1:] or ["flip", "timed"]
    for w in which:
        {"flip": flip, "timed": timed}[w]()
    print("done", flush=True)
