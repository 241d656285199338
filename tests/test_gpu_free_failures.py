"""The solver's failure paths on the free-motion tasks (fixed step and optimised timing),
forced by its parameters on both sides: no retry after a failed factorisation, a damping
cap of 1e-6, one outer iteration, an indefinite start (rho0 = -1: the first factorisation
of every solve fails) and the indefinite start without retries (every factorisation fails,
every step is rejected).  These are normal-exit solves.  Asserted: per-sequence parity with
the FP64 oracle under the rule of tests/parity.py on every admissible order of at most two
segments on four instances, the feasible flag equal to v <= eps_feas, and the status and
failure counts the forced path implies (Sec. III-C: a factorisation that fails after the
retries rejects the step)."""
import numpy as np
import pytest

import parity
from paper_2609_21803_amd import instances as I

pytestmark = pytest.mark.gpu

ROUND32 = 1 | 2 | 4 | 8
EPS = 1e-5
KW = [dict(chol_retries=0), dict(rho_max=1e-6), dict(al_max=1), dict(rho0=-1.0), dict(rho0=-1.0, chol_retries=0)]


def f32(a):
    return np.asarray(a, np.float32).astype(np.float64)


@pytest.mark.parametrize("kw", KW)
@pytest.mark.parametrize("timed", [False, True])
def test_free_forced_failure_paths_match_oracle(timed, kw):
    import torch
    import oracle
    from oracle import free as F
    from paper_2609_21803_amd import native
    task = native.TASK_PUSH_FREE_TIMED if timed else native.TASK_PUSH_FREE
    orders = [F.key_modes(int(k)) for k in F.seed(2)]
    x0, goal, inst = I.push_free_pairs(5100 + timed, 4)
    pair = np.repeat(np.arange(4), len(orders))
    b = I.orders_batch(x0, goal, inst, pair, orders * 4, [[10] * len(o) for o in orders] * 4)
    nmax = 20
    ctx = native.Context(max_batch=len(pair), max_segments=6, max_intervals=nmax, task=task,
                         params=native.SolverParams(**kw))
    out = ctx.evaluate(**native.to_device(b))
    torch.cuda.synchronize()
    ctx.check()
    g = {k: v.cpu().numpy() for k, v in out.items() if v is not None}

    def run_oracle(batch, params):
        return F.evaluate(f32(batch["x0"]), f32(batch["goal"]), f32(batch["inst"]), batch["nseg"], batch["modes"],
                          batch["knots"], params=params, nmax=nmax, timed=timed)

    o = run_oracle(b, oracle.Params(**kw))

    def solve(sub, rows, r32):
        return run_oracle(sub, oracle.Params(**kw, round32=r32))
    parity.check(g, o, b, solve, f"free{' timed' if timed else ''} forced {kw}", round32=ROUND32,
                 allow=2e-3 if timed else 1e-3)
    assert np.array_equal(g["feasible"] == 1, g["viol"] <= EPS)
    assert set(np.unique(g["stats"][:, 3])) <= {0, 1, 2}
    if kw.get("al_max") == 1:
        assert np.all(g["stats"][:, 0] == 1)
    if kw.get("rho0") == -1.0:
        assert np.all(g["stats"][:, 2] >= 1)
        if kw.get("chol_retries") == 0:
            assert np.array_equal(g["stats"], o["stats"]) and np.all(g["feasible"] == 0)
