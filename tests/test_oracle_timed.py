"""Pins of the optimised-timing pushing oracle (interval durations as controls, Sec. III-C
"Shared representation across contact modes"; the pushing configuration of Sec. IV-A runs
with an optimised time step and a duration bound).

The timed problem adds the duration h_k of each interval as a fourth control, the bound
rows h_min <= h_k <= h_max, and charges h_k (effort + w_T).  What pins it, beyond its own
formulas: the fixed-step model (already pinned) at h = dt, central differences, a dense
linear solve of the Gauss-Newton system, and closed-form optima of the straight push in
the three regimes of the duration bound (interior, upper bound active, lower bound active).
"""
import itertools

import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

DT, H_MIN, H_MAX, W_T = 0.1, 0.02, 0.2, 0.01
FMAX = 0.5 * 1.0 * 9.81
TIGHT = dict(al_max=80, gn_max=40, eta_star=1e-12, omega_star=1e-11, rc_star=1e-12, mu_min=1e-8)


def _timed_v(v11, h):
    """(x_k, u_k[3], x_{k+1}) -> (x_k, u_k[3], h, x_{k+1})."""
    return np.concatenate([v11[:7], [h], v11[7:]])


@pytest.mark.parametrize("face,slip,smask", list(itertools.product(range(4), range(3), (0, 1))))
def test_timed_rows_reduce_to_fixed_rows_at_the_fixed_step(orc, face, slip, smask):
    """At h = dt every fixed-step row (pinned separately) is reproduced, column for column;
    the defects are affine in h (explicit Euler), so c(2 dt) - c(dt) = dt * dc/dh exactly
    up to rounding; the two duration rows are h - h_max and h_min - h."""
    rng = np.random.default_rng(7 + 6 * face + 2 * slip + smask)
    for _ in range(4):
        v = rng.normal(size=11) * np.array([0.2, 0.2, 2, 0.04, 2, 1, 0.1, 0.2, 0.2, 2, 0.04])
        c0, J0, en0 = orc.push_rows(face, slip, smask, 0.37, v)
        c1, J1, en1 = orc.push_rows(face, slip, smask, 0.37, _timed_v(v, DT), timed=1)
        assert np.array_equal(c1[:10], c0) and np.array_equal(en1[:10], en0)
        cols = [0, 1, 2, 3, 4, 5, 6, 8, 9, 10, 11]
        assert np.array_equal(J1[:10][:, cols], J0)
        c2, _, _ = orc.push_rows(face, slip, smask, 0.37, _timed_v(v, 2 * DT), timed=1)
        assert np.allclose(c2[:4] - c1[:4], DT * J1[:4, 7], rtol=1e-12, atol=1e-15)
        assert en1[10] == 1 and en1[11] == 1
        assert c1[10] == DT - H_MAX and c1[11] == H_MIN - DT
        assert J1[10, 7] == 1 and J1[11, 7] == -1 and np.count_nonzero(J1[10:]) == 2


@pytest.mark.parametrize("face,slip", list(itertools.product(range(4), range(3))))
def test_timed_row_jacobians_match_central_differences(orc, face, slip):
    rng = np.random.default_rng(300 + 3 * face + slip)
    for _ in range(4):
        v = rng.normal(size=12) * np.array([0.2, 0.2, 2, 0.04, 2, 1, 0.1, 0.03, 0.2, 0.2, 2, 0.04])
        v[7] = abs(v[7]) + 0.05
        c, J, en = orc.push_rows(face, slip, 1, 0.37, v, timed=1)
        Jfd = np.zeros_like(J)
        for j in range(12):
            h = 1e-6 * max(1.0, abs(v[j]))
            vp, vm = v.copy(), v.copy()
            vp[j] += h
            vm[j] -= h
            Jfd[:, j] = (orc.push_rows(face, slip, 1, 0.37, vp, timed=1)[0]
                         - orc.push_rows(face, slip, 1, 0.37, vm, timed=1)[0]) / (2 * h)
        assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-8), np.abs(J - Jfd).max()


def test_timed_cost_value_gradient_and_hessian_model(orc):
    """Cost h (effort + w_T) = (h / dt) (fixed-step cost) + w_T h; its gradient matches
    central differences; the Hessian model is the exact force/velocity block (central
    differences of the gradient) and has no duration entries."""
    rng = np.random.default_rng(5)
    for _ in range(6):
        u3 = rng.normal(size=3) * np.array([2.0, 1.0, 0.1])
        h = 0.03 + 0.15 * rng.random()
        J0, _, _ = orc.push_cost(u3)
        u = np.append(u3, h)
        J, g, H = orc.push_cost(u, timed=1)
        assert np.isclose(J, h / DT * J0 + W_T * h, rtol=1e-14)
        gfd = np.zeros(4)
        Hfd = np.zeros((4, 4))
        for j in range(4):
            e = np.zeros(4)
            e[j] = 1e-6
            gfd[j] = (orc.push_cost(u + e, timed=1)[0] - orc.push_cost(u - e, timed=1)[0]) / 2e-6
            Hfd[:, j] = (orc.push_cost(u + e, timed=1)[1] - orc.push_cost(u - e, timed=1)[1]) / 2e-6
        assert np.allclose(g, gfd, rtol=1e-7, atol=1e-10)
        assert np.allclose(H[:3, :3], Hfd[:3, :3], rtol=1e-6, atol=1e-10)
        assert np.all(H[3] == 0) and np.all(H[:, 3] == 0)
        assert np.all(np.linalg.eigvalsh(H[:3, :3]) > 0)


def test_timed_row_scales(orc):
    """Rows that do not involve h keep the fixed-step scales; the duration rows (type 12)
    have Jacobian-row norm 1 at every sample point, so their median is 1; the defects gain
    the h column, so their scales can only grow."""
    s0, s1 = orc.scales(0), orc.scales(1)
    assert np.array_equal(s1[4:12], s0[4:12])
    assert s1[12] == 1.0 and s0[12] == 1.0
    assert np.all(s1[:4] >= s0[:4])


def _random_timed_point(orc, seed, modes=(6, 1, 11), knots=(3, 4, 2)):
    rng = np.random.default_rng(seed)
    S = orc.Seq(modes, knots, goal=(0.12, -0.05, 0.8), mu=0.41, timed=1)
    z = S.initial() + 0.01 * rng.normal(size=S.N * 8)
    lam = 0.1 * rng.normal(size=S.N * 5)
    nu = np.abs(0.1 * rng.normal(size=S.N * 7))
    lamT = 0.1 * rng.normal(size=3)
    return S, z, lam, nu, lamT


@pytest.mark.parametrize("seed", [0, 1])
def test_timed_merit_gradient_matches_central_differences(orc, seed):
    S, z, lam, nu, lamT = _random_timed_point(orc, seed)
    _, g = S.merit(z, lam, nu, lamT, 0.05)
    gfd = np.zeros_like(g)
    for i in range(len(z)):
        zp, zm = z.copy(), z.copy()
        zp[i] += 1e-6
        zm[i] -= 1e-6
        gfd[i] = (S.merit(zp, lam, nu, lamT, 0.05)[0] - S.merit(zm, lam, nu, lamT, 0.05)[0]) / 2e-6
    assert np.allclose(g, gfd, rtol=1e-5, atol=1e-7), np.abs(g - gfd).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_timed_riccati_step_equals_dense_kkt_solve(orc, seed):
    """The backward Riccati recursion over the 8 stage unknowns gives the step of the dense
    system (H + rho I) dz = -g, with H = sum over active rows of a a^T / mu plus the cost
    Hessian model (force/velocity block by differences of the cost gradient)."""
    S, z, lam, nu, lamT = _random_timed_point(orc, seed)
    mu_al, rho, N, W = 0.03, 1e-3, S.N, 8
    _, g = S.merit(z, lam, nu, lamT, mu_al)
    c, J, en, cT, JT = S.blocks(z)
    H = np.zeros((W * N, W * N))
    for k in range(N):
        cols = ([(k - 1) * W + 4 + i for i in range(4)] if k > 0 else [None] * 4) + [k * W + i for i in range(W)]
        for r in range(12):
            if not en[k, r]:
                continue
            if r >= 5 and not (nu[k * 7 + r - 5] + c[k, r] / mu_al > 0):
                continue
            a = np.zeros(W * N)
            for j, col in enumerate(cols):
                if col is not None:
                    a[col] += J[k, r, j]
            H += np.outer(a, a) / mu_al
        u = z[k * W:k * W + 4]
        for j in range(3):
            e = np.zeros(4)
            e[j] = 1e-6
            H[k * W:k * W + 3, k * W + j] += ((orc.push_cost(u + e, 1)[1] - orc.push_cost(u - e, 1)[1]) / 2e-6)[:3]
    for r in range(3):
        a = np.zeros(W * N)
        a[(N - 1) * W + 4:(N - 1) * W + 8] = JT[r]
        H += np.outer(a, a) / mu_al
    dz_dense = np.linalg.solve(H + rho * np.eye(len(z)), -g)
    dz = S.step(z, lam, nu, lamT, mu_al, rho)
    assert dz is not None
    assert np.linalg.norm(dz - dz_dense) <= 1e-6 * np.linalg.norm(dz_dense)


def _straight(orc, d, N, params):
    modes = np.zeros((1, 6), np.int32)
    knots = np.zeros((1, 6), np.int32)
    modes[0, 0], knots[0, 0] = 6, N
    return orc.evaluate(np.zeros((1, 4)), np.array([[d, 0.0, 0.0]]), np.array([[0.4]]), np.array([1]), modes, knots,
                        params=params)


@pytest.mark.parametrize("d,N", [(0.2, 20), (0.3, 24), (0.12, 10), (0.5, 10), (0.01, 24)])
def test_timed_straight_push_closed_forms(orc, d, N):
    """Goal (d, 0, 0) pushed through the centre of the face opposite to the motion: the
    slider moves at v = v_ref F_n / f_max, so with T = sum h the cost is
    sum h (v^2 + w_T) >= d^2 / T + w_T T (Cauchy-Schwarz), minimised at T* = d / sqrt(w_T)
    with J* = 2 d sqrt(w_T) when N h_min <= T* <= N h_max, and at the active bound otherwise
    (every h at that bound, constant force)."""
    T = d / np.sqrt(W_T)
    T = min(max(T, N * H_MIN), N * H_MAX)
    Jstar = d * d / T + W_T * T
    r = _straight(orc, d, N, orc.Params(timed=1, **TIGHT))
    assert r["feasible"][0] == 1 and r["stats"][0, 3] == 1
    assert abs(r["cost"][0] - Jstar) <= 1e-7 * Jstar, (r["cost"][0], Jstar)
    h = r["traj"][0, :N, 7]
    assert abs(h.sum() - T) <= 1e-6 * T
    assert np.all(h >= H_MIN - 1e-7) and np.all(h <= H_MAX + 1e-7)
    if T in (N * H_MIN, N * H_MAX):
        assert np.allclose(h, T / N, rtol=1e-6)
    assert np.allclose(r["traj"][0, :N, 4], FMAX * d / T, rtol=1e-5)
    # the exploration budget and tolerances reach it within 1e-3
    r2 = _straight(orc, d, N, orc.Params(timed=1))
    assert r2["feasible"][0] == 1 and abs(r2["cost"][0] - Jstar) <= 1e-3 * Jstar


def test_timed_zero_motion_goal_costs_the_shortest_duration(orc):
    """Goal = start: zero force and zero slip satisfy every row of every order, and the
    time charge is least with every interval at h_min: J = w_T N h_min."""
    b = I._batch(np.zeros((1, 4)), np.zeros((1, 3)), np.array([[0.35]]), I.all_orders(1), (6,))
    r = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"], params=orc.Params(timed=1))
    assert np.all(r["feasible"] == 1)
    assert np.allclose(r["cost"], W_T * 6 * H_MIN, rtol=1e-4)
    assert np.allclose(r["traj"][:, :6, 7], H_MIN, atol=1e-6)


def test_fixed_step_plans_rescore_as_timed_plans_and_timed_plans_respect_the_bounds(orc):
    """A fixed-step plan with h = dt inserted is a point of the timed problem: its timed
    score is J_fixed + w_T N dt with the same violation (the duration rows are inactive at
    dt).  Every feasible timed plan keeps its durations in [h_min, h_max], and rescoring
    its trajectory reproduces the cost and violation the solve returned."""
    N = 12
    b = I._batch(np.zeros((1, 4)), np.array([[0.15, 0.03, 0.2]]), np.array([[0.45]]), I.all_orders(2)[::7], (6, 6))
    rf = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"])
    rt = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"], params=orc.Params(timed=1))
    assert rf["feasible"].sum() >= 4 and rt["feasible"].sum() >= 4

    def seq(i):
        return orc.Seq(b["modes"][i, :2], b["knots"][i, :2], goal=b["goal"][i], mu=float(b["inst"][i, 0]), timed=1)

    for i in np.where(rf["feasible"] == 1)[0]:
        z = np.zeros(N * 8)
        for k in range(N):
            z[k * 8:k * 8 + 3] = rf["traj"][i, k, 4:7]
            z[k * 8 + 3] = DT
            z[k * 8 + 4:k * 8 + 8] = rf["traj"][i, k + 1, 0:4]
        J, v = seq(i).score(z)
        assert abs(J - (rf["cost"][i] + W_T * N * DT)) <= 1e-12 and v == rf["viol"][i]
    for i in np.where(rt["feasible"] == 1)[0]:
        h = rt["traj"][i, :N, 7]
        assert np.all(h >= H_MIN - 1e-5) and np.all(h <= H_MAX + 1e-5)
        z = np.zeros(N * 8)
        for k in range(N):
            z[k * 8:k * 8 + 4] = rt["traj"][i, k, 4:8]
            z[k * 8 + 4:k * 8 + 8] = rt["traj"][i, k + 1, 0:4]
        J, v = seq(i).score(z)
        assert abs(J - rt["cost"][i]) <= 1e-12 * max(1.0, abs(J)) and v == rt["viol"][i]


@pytest.mark.parametrize("modes,knots,goal", [((6, 7), (4, 4), (0.1, 0.0, 0.2)), ((6,), (10,), (0.15, 0.02, 0.1))])
def test_timed_converged_solve_is_a_kkt_point_for_slsqp(orc, modes, knots, goal):
    """An independent NLP solver (scipy SLSQP) started at the timed oracle's solution finds
    no better feasible point of the same transcription (Eq. 2 with the durations as
    controls) nearby.  The tight solve ends feasible at its iteration budget rather than at
    the 1e-11 stationarity test: spreading the elapsed time differently over intervals that
    move at the same speed leaves the cost unchanged, and that flat direction slows the
    last digits of the stationarity measure."""
    from scipy.optimize import minimize
    N = sum(knots)
    S = orc.Seq(list(modes), list(knots), goal=goal, mu=0.4, timed=1)
    ma = np.zeros((1, 6), np.int32)
    ka = np.zeros((1, 6), np.int32)
    ma[0, :len(modes)] = modes
    ka[0, :len(knots)] = knots
    r = orc.evaluate(np.zeros((1, 4)), np.array([goal]), np.array([[0.4]]), np.array([len(modes)]), ma, ka,
                     params=orc.Params(timed=1, **TIGHT))
    print("oracle", r["cost"][0], r["viol"][0], r["stats"][0])
    assert r["feasible"][0] == 1
    z0 = np.zeros(N * 8)
    for k in range(N):
        z0[k * 8:k * 8 + 4] = r["traj"][0, k, 4:8]
        z0[k * 8 + 4:k * 8 + 8] = r["traj"][0, k + 1, 0:4]

    def eqs(z):
        c, J, en, cT, JT = S.blocks(z)
        return np.concatenate([c[:, :5][en[:, :5] == 1], cT])

    def ineqs(z):
        c, J, en, cT, JT = S.blocks(z)
        return -c[:, 5:][en[:, 5:] == 1]

    obj = lambda z: S.score(z)[0]
    res = minimize(obj, z0, method="SLSQP", constraints=[dict(type="eq", fun=eqs), dict(type="ineq", fun=ineqs)],
                   options=dict(ftol=1e-14, maxiter=200))
    Jr, vr = S.score(res.x)
    print("slsqp", Jr, vr, res.message)
    assert abs(r["cost"][0] - obj(z0)) < 1e-12
    assert not (vr <= 1e-8 and Jr < r["cost"][0] - 1e-6), (Jr, r["cost"][0])
