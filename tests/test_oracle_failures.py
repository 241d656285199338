"""Failure injection on the FP64 oracle (CPU): the solver's failure paths forced by its
parameters, each a normal-exit solve (Sec. III-C: a failed Cholesky factorisation raises
the damping, exhausted retries reject the step; budget exhaustion alone does not
establish feasibility).

* rho0 = -1: the first factorisation of every solve fails (S - I is indefinite), the
  retry raises the damping to its floor and the solve goes on;
* rho0 = -1 with chol_retries = 0: every factorisation fails and every step is rejected;
* chol_retries = 0 alone, rho_max = 1e-6 (the damping cannot grow past a tiny value),
  al_max = 1 (one outer iteration, most solves end at the budget).

Checked on the two-segment workload: every result is finite or flagged (status 2 with a
NaN cost), statuses are valid, the feasible flag is exactly v <= eps_feas whatever the
status, iteration counters respect the budget, and the forced paths are taken.
"""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

EPS = 1e-5


def _run(orc, **kw):
    b = I.subset(I.push_tiny(), np.arange(0, 1152, 3))
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    r = orc.evaluate(f32(b["x0"]), f32(b["goal"]), f32(b["inst"]), b["nseg"], b["modes"], b["knots"],
                     params=orc.Params(**kw), nmax=10)
    return b, r


def _common(r, al_max=20, gn_max=10):
    st = r["stats"]
    assert set(np.unique(st[:, 3])) <= {0, 1, 2}
    ok = st[:, 3] != 2
    assert np.all(np.isfinite(r["cost"][ok])) and np.all(np.isfinite(r["viol"][ok]))
    assert np.all(np.isnan(r["cost"][~ok]))
    assert np.array_equal(r["feasible"] == 1, r["viol"] <= EPS)
    assert np.all(st[:, 0] <= al_max) and np.all(st[:, 1] <= al_max * gn_max)
    assert np.all(r["feasible"][st[:, 3] == 1] == 1)     # converged implies feasible here


@pytest.mark.parametrize("kw", [dict(chol_retries=0), dict(rho_max=1e-6), dict(al_max=1), dict(rho0=-1.0),
                                dict(rho0=-1.0, chol_retries=0), dict(chol_retries=0, rho_max=1e-6, al_max=2)])
def test_forced_failure_paths_end_normally(orc, kw):
    b, r = _run(orc, **kw)
    _common(r, al_max=kw.get("al_max", 20))
    _, base = _run(orc)
    print(kw, "feasible", r["feasible"].sum(), "of", len(r["feasible"]), "(default", base["feasible"].sum(), ")",
          "statuses", np.bincount(r["stats"][:, 3], minlength=3), "Cholesky failures", r["stats"][:, 2].sum())
    if kw.get("al_max") == 1:
        assert np.all(r["stats"][:, 0] == 1)
        # budget exhaustion alone does not establish feasibility: some solves stop at the
        # budget infeasible, and no budget-limited solve is flagged feasible above eps
        assert np.any((r["stats"][:, 3] == 0) & (r["feasible"] == 0))
        assert r["feasible"].sum() < base["feasible"].sum()


def test_indefinite_start_is_caught_by_the_factorisation(orc):
    """rho0 = -1 makes S = G - I indefinite: the positive-definiteness test of the Cholesky
    factorisation fails on the first iteration of every solve.  With retries the damping
    goes to its floor and the solves proceed (feasible orders found); without, every step is
    rejected, each Gauss-Newton iteration counts one failure, and no solve leaves its start."""
    _, a = _run(orc, rho0=-1.0)
    assert np.all(a["stats"][:, 2] >= 1) and a["feasible"].sum() > 0
    _, z = _run(orc, rho0=-1.0, chol_retries=0)
    assert np.array_equal(z["stats"][:, 2], z["stats"][:, 1])
    assert np.all(z["stats"][:, 3] == 0) and np.all(z["stats"][:, 0] == 20)
    b = I.subset(I.push_tiny(), np.arange(0, 1152, 3))
    f32 = lambda a_: np.asarray(a_, np.float32).astype(np.float64)
    # the returned trajectory is the schedule-derived start
    for i in range(0, len(z["cost"]), 37):
        K = int(b["nseg"][i])
        seq = orc.Seq(b["modes"][i, :K], b["knots"][i, :K], x0=f32(b["x0"])[i], goal=f32(b["goal"])[i],
                      mu=float(f32(b["inst"])[i, 0]))
        J0, v0 = seq.score(seq.initial())
        assert z["cost"][i] == J0 and z["viol"][i] == v0


def test_no_retry_rejects_instead_of_damping(orc):
    """With retries, a failed factorisation is retried at raised damping; without, the step
    is rejected: the retry-free solves count no more Cholesky failures per iteration than
    one, and their results differ only where a factorisation failed."""
    _, a = _run(orc, chol_retries=0)
    _, d = _run(orc)
    fa = a["stats"][:, 2]
    assert np.all(fa <= a["stats"][:, 1])                 # at most one failure per Gauss-Newton iteration
    same = (fa == 0) & (d["stats"][:, 2] == 0)
    assert np.array_equal(a["cost"][same], d["cost"][same], equal_nan=True)
    assert np.array_equal(a["stats"][same], d["stats"][same])


def test_damping_cap_changes_only_solves_that_reach_it(orc):
    """rho_max = 1e8 (the default) against 1e-6: solves whose damping never needed to grow
    beyond 1e-6 give the same result bit for bit; the cap only changes the others."""
    _, a = _run(orc, rho_max=1e-6)
    _, d = _run(orc)
    same = np.array_equal(a["cost"], d["cost"], equal_nan=True)
    diff = (~np.isclose(a["cost"], d["cost"], rtol=0, atol=0, equal_nan=True)).sum()
    print("solves changed by the damping cap:", diff, "of", len(a["cost"]))
    assert not same and diff < len(a["cost"])
