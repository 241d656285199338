"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test names the passage it rests on (paper section / equation / algorithm) or the
mathematical fact it uses: central finite differences, a dense linear solve, closed
forms, symmetry of the square slider, brute force, and an independent NLP solver.
"""
import itertools

import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

DT = 0.1
A_SIDE = 0.1
FMAX = 0.5 * 1.0 * 9.81


def traj_to_z(traj, N):
    """ABI trajectory rows (x_k, u_k) -> the oracle's (u_k, x_{k+1}) primal layout."""
    z = np.zeros(N * 7)
    for k in range(N):
        z[k * 7:k * 7 + 3] = traj[k, 4:7]
        z[k * 7 + 3:k * 7 + 7] = traj[k + 1, 0:4]
    return z


# ---------------------------------------------------------------------------------
# Model: derivatives and the quasi-static law
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("face,slip,smask", list(itertools.product(range(4), range(3), (0, 1))))
def test_row_jacobians_match_central_differences(orc, face, slip, smask):
    """Analytic row Jacobians (Sec. III-C, A_k) against central differences, h = 1e-6."""
    rng = np.random.default_rng(100 + 6 * face + 2 * slip + smask)
    for _ in range(5):
        v = rng.normal(size=11) * np.array([0.2, 0.2, 2, 0.04, 2, 1, 0.1, 0.2, 0.2, 2, 0.04])
        c, J, en = orc.push_rows(face, slip, smask, 0.37, v)
        Jfd = np.zeros_like(J)
        for j in range(11):
            h = 1e-6 * max(1.0, abs(v[j]))
            vp, vm = v.copy(), v.copy()
            vp[j] += h
            vm[j] -= h
            Jfd[:, j] = (orc.push_rows(face, slip, smask, 0.37, vp)[0] - orc.push_rows(face, slip, smask, 0.37, vm)[0]) / (2 * h)
        assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-8), (face, slip, np.abs(J - Jfd).max())
        # masked rows have zero residual and derivative (fixed-row masking, Sec. III-C)
        assert np.all(c[en == 0] == 0) and np.all(J[en == 0] == 0)
        assert en[3] == smask and en[7] == (1 if slip == 0 else 0)


def test_limit_surface_radius_is_mean_distance_over_square():
    """c_ls = mean distance from the centre over a uniform-pressure square of side a
    (the ellipsoidal limit surface of the slider); checked by 2-D quadrature."""
    n = 2000
    g = (np.arange(n) + 0.5) / n - 0.5
    X, Y = np.meshgrid(g * A_SIDE, g * A_SIDE)
    mean_r = np.sqrt(X ** 2 + Y ** 2).mean()
    closed = A_SIDE * (np.sqrt(2) + np.log(1 + np.sqrt(2))) / 6
    assert abs(mean_r - closed) < 1e-7


def test_one_euler_step_matches_contact_wrench_formulation(orc):
    """One explicit-Euler step of the quasi-static law written through the contact
    Jacobian: wrench = (F, p x F) with p = (a/2) n + s t, twist = (v_ref/f_max)
    diag(1, 1, 1/c_ls^2) wrench, world velocity = R(theta) twist_xy."""
    cls = A_SIDE * (np.sqrt(2) + np.log(1 + np.sqrt(2))) / 6
    rng = np.random.default_rng(7)
    for face in range(4):
        ang = face * np.pi / 2
        n = np.array([np.cos(ang), np.sin(ang)])
        t = np.array([-np.sin(ang), np.cos(ang)])
        x = np.array([0.05, -0.02, 0.7, 0.013])
        u = np.array([1.3, -0.4, 0.02])
        p = 0.5 * A_SIDE * n + x[3] * t
        F = -u[0] * n + u[1] * t
        wrench = np.array([F[0], F[1], np.cross(np.append(p, 0.0), np.append(F, 0.0))[2]])
        tw = (1.0 / FMAX) * wrench * np.array([1, 1, 1 / cls ** 2])
        R = np.array([[np.cos(x[2]), -np.sin(x[2])], [np.sin(x[2]), np.cos(x[2])]])
        vw = R @ tw[:2]
        x1 = np.array([x[0] + DT * vw[0], x[1] + DT * vw[1], x[2] + DT * tw[2], x[3] + DT * u[2]])
        v = np.concatenate([x, u, x1])
        c, _, _ = orc.push_rows(face, 0, 1, 0.4, v)
        assert np.allclose(c[:4], 0, atol=1e-14), c[:4]


def test_row_scales_closed_form_entries(orc):
    """Median Jacobian-row norms (Sec. IV-A, constraint scaling) for the row types whose
    norm is the same at every sample point: bounds and terminal rows 1, slide row
    sqrt(1+mu^2) at mu=0.4, s-defect sqrt(2+dt^2), theta-defect at F_n = 0.05 f_max."""
    s = orc.scales()
    cls2 = (A_SIDE * (np.sqrt(2) + np.log(1 + np.sqrt(2))) / 6) ** 2
    k1 = 1 / FMAX
    dth = np.sqrt(2 + (DT * k1 * 0.05 * FMAX / cls2) ** 2 + (DT * k1 * 0.5 * A_SIDE / cls2) ** 2)
    expect = {2: dth, 3: np.sqrt(2 + DT ** 2), 4: 1.0, 5: np.sqrt(1.16), 6: 1.0, 7: np.sqrt(1.16), 8: 1.0,
              9: 1.0, 10: 1.0, 11: 1.0}
    for t, e in expect.items():
        assert abs(s[t] - e) < 1e-12, (t, s[t], e)
    assert 1.414 < s[0] < 1.416 and abs(s[0] - s[1]) < 1e-12


# ---------------------------------------------------------------------------------
# One Gauss-Newton step: structured Riccati == dense solve; gradient == d(merit)
# ---------------------------------------------------------------------------------
def _random_point(orc, seed, modes=(6, 1, 11), knots=(3, 4, 2)):
    rng = np.random.default_rng(seed)
    S = orc.Seq(modes, knots, goal=(0.12, -0.05, 0.8), mu=0.41)
    z = S.initial() + 0.01 * rng.normal(size=S.N * 7)
    lam = 0.1 * rng.normal(size=S.N * 5)
    nu = np.abs(0.1 * rng.normal(size=S.N * 5))
    lamT = 0.1 * rng.normal(size=3)
    return S, z, lam, nu, lamT


def _dense_gn(S, z, lam, nu, lamT, mu_al, orc):
    """Dense GN matrix H + rho I (without rho) and active set, built from the oracle's
    per-stage scaled rows, with the cost Hessian taken by differences of the gradient
    with all constraint terms switched off (mu -> inf)."""
    N = S.N
    c, J, en, cT, JT = S.blocks(z)
    H = np.zeros((7 * N, 7 * N))
    for k in range(N):
        cols = ([(k - 1) * 7 + 3 + i for i in range(4)] if k > 0 else [None] * 4) + [k * 7 + i for i in range(7)]
        for r in range(10):
            if not en[k, r]:
                continue
            if r < 5:
                active = True
            else:
                active = nu[k * 5 + r - 5] + c[k, r] / mu_al > 0
            if not active:
                continue
            a = np.zeros(7 * N)
            for j, col in enumerate(cols):
                if col is not None:
                    a[col] += J[k, r, j]
            H += np.outer(a, a) / mu_al
    for r in range(3):
        a = np.zeros(7 * N)
        a[(N - 1) * 7 + 3:(N - 1) * 7 + 7] = JT[r]
        H += np.outer(a, a) / mu_al
    zero = np.zeros_like(lam)
    for i in range(7 * N):
        h = 1e-4
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        gp = S.merit(zp, zero, zero, np.zeros(3), 1e300)[1]
        gm = S.merit(zm, zero, zero, np.zeros(3), 1e300)[1]
        H[:, i] += (gp - gm) / (2 * h)
    return H


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_riccati_step_equals_dense_kkt_solve(orc, seed):
    """Backward Riccati recursion with Cholesky (Sec. III-C, S_k) gives the same step as
    numpy.linalg.solve on the assembled block-tridiagonal system (H + rho I) dz = -g."""
    S, z, lam, nu, lamT = _random_point(orc, seed)
    mu_al, rho = 0.03, 1e-3
    _, g = S.merit(z, lam, nu, lamT, mu_al)
    H = _dense_gn(S, z, lam, nu, lamT, mu_al, orc)
    dz_dense = np.linalg.solve(H + rho * np.eye(len(z)), -g)
    dz = S.step(z, lam, nu, lamT, mu_al, rho)
    assert dz is not None
    assert np.linalg.norm(dz - dz_dense) <= 1e-8 * np.linalg.norm(dz_dense)


@pytest.mark.parametrize("seed", [3, 4])
def test_merit_gradient_matches_central_differences(orc, seed):
    """Gradient of the augmented-Lagrangian merit against central differences."""
    S, z, lam, nu, lamT = _random_point(orc, seed)
    mu_al = 0.05
    _, g = S.merit(z, lam, nu, lamT, mu_al)
    gfd = np.zeros_like(g)
    for i in range(len(z)):
        h = 1e-6
        zp, zm = z.copy(), z.copy()
        zp[i] += h
        zm[i] -= h
        gfd[i] = (S.merit(zp, lam, nu, lamT, mu_al)[0] - S.merit(zm, lam, nu, lamT, mu_al)[0]) / (2 * h)
    assert np.allclose(g, gfd, rtol=1e-5, atol=1e-7), np.abs(g - gfd).max()


def test_merit_reduces_to_objective_at_feasible_point(orc):
    """At a point satisfying every row with strictly inactive inequalities and zero
    multipliers the merit equals the objective J of Eq. (2); a pure equality violation
    c adds c^2/(2 mu) (penalty) on top."""
    S = orc.Seq([6], [4], goal=(0.0, 0.0, 0.0), mu=0.4)
    z = np.zeros(S.N * 7)
    z[0::7] = 1e-3          # tiny pushing force on a resting slider violates the defects
    lam, nu, lamT = S.duals()
    J, _ = S.score(np.zeros(S.N * 7))
    phi0, _ = S.merit(np.zeros(S.N * 7), lam, nu, lamT, 0.1)
    assert J == 0.0 and phi0 == 0.0


# ---------------------------------------------------------------------------------
# Whole solves: closed form, zero motion, symmetry, segment merging, KKT by SLSQP
# ---------------------------------------------------------------------------------
TIGHT = dict(al_max=80, gn_max=40, eta_star=1e-12, omega_star=1e-11, rc_star=1e-12, mu_min=1e-8)


@pytest.mark.parametrize("d,modes,knots", [(0.2, [6], [10]), (-0.15, [0], [12]), (0.25, [6, 6], [5, 5])])
def test_straight_sticking_push_reaches_closed_form(orc, d, modes, knots):
    """Goal (d, 0, 0) pushed through the centre of the face opposite to the motion:
    by Cauchy-Schwarz the discrete optimum is J* = d^2 / (v_ref^2 T), T = N dt, reached by
    a constant normal force f_max |d| / (v_ref T)."""
    N = sum(knots)
    T = N * DT
    B = 1
    modes_a = np.zeros((B, 6), np.int32)
    knots_a = np.zeros((B, 6), np.int32)
    modes_a[0, :len(modes)] = modes
    knots_a[0, :len(knots)] = knots
    r = orc.evaluate(np.zeros((1, 4)), np.array([[d, 0, 0]]), np.array([[0.4]]), np.array([len(modes)]),
                     modes_a, knots_a, params=orc.Params(**TIGHT))
    Jstar = d ** 2 / T
    assert r["feasible"][0] == 1
    assert abs(r["cost"][0] - Jstar) <= 1e-8 * Jstar, (r["cost"][0], Jstar)
    fn = r["traj"][0, :N, 4]
    assert np.allclose(fn, FMAX * abs(d) / T, rtol=1e-6)
    # with the default (exploration) tolerances the same solve is within 1e-4
    r2 = orc.evaluate(np.zeros((1, 4)), np.array([[d, 0, 0]]), np.array([[0.4]]), np.array([len(modes)]),
                      modes_a, knots_a)
    assert r2["feasible"][0] == 1 and abs(r2["cost"][0] - Jstar) <= 1e-4 * Jstar


def test_closed_form_is_a_lower_bound_for_every_order(orc):
    """Every feasible order on goal (d, 0, 0) costs at least d^2/(v_ref^2 T) (same bound)."""
    b = I._batch(np.zeros((1, 4)), np.array([[0.2, 0.0, 0.0]]), np.array([[0.4]]), I.all_orders(2), (5, 5))
    r = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"])
    f = r["feasible"] == 1
    assert f.sum() > 10
    # the violation tolerance relaxes the bound to (d - v)^2 / T
    lb = (0.2 - r["viol"][f]) ** 2 / 1.0
    assert np.all(r["cost"][f] >= lb - 1e-9)
    # the straight push (face 2 stick twice, id 6) attains it
    k = np.where((b["modes"][:, 0] == 6) & (b["modes"][:, 1] == 6))[0][0]
    assert abs(r["cost"][k] - 0.04) <= 1e-4 * 0.04


def test_zero_motion_goal_is_feasible_at_zero_cost_for_every_order(orc):
    """Goal = start: zero force and zero slip satisfy every row of every order, J = 0."""
    b = I._batch(np.zeros((1, 4)), np.zeros((1, 3)), np.array([[0.35]]), I.all_orders(2), (5, 5))
    r = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"])
    assert np.all(r["feasible"] == 1)
    assert np.all(r["cost"] <= 1e-6)


def _sym_batch(goal, mu, face_map, slip_map):
    orders = I.all_orders(2)
    mapped = np.vectorize(lambda m: 3 * face_map[m // 3] + slip_map[m % 3])(orders)
    b0 = I._batch(np.zeros((1, 4)), np.array([goal]), np.array([[mu]]), orders, (5, 5))
    return b0, mapped


@pytest.mark.parametrize("seed", [0, 1])
def test_square_symmetry_rotation_and_mirror(orc, seed):
    """The square slider is invariant under its symmetry group: rotating the goal by
    +90 deg about the start and relabelling face j -> j+1, or mirroring y -> -y with
    face j -> -j and slide+ <-> slide-, maps each order's NLP onto another's."""
    x0, goal, inst = I.push_pairs(seed, 1)
    g, mu = goal[0], inst[0, 0]
    base = I._batch(x0, goal, inst, I.all_orders(2), (5, 5))
    r0 = orc.evaluate(base["x0"], base["goal"], base["inst"], base["nseg"], base["modes"], base["knots"])
    for goal2, fmap, smap in [((-g[1], g[0], g[2]), [1, 2, 3, 0], [0, 1, 2]),
                              ((g[0], -g[1], -g[2]), [0, 3, 2, 1], [0, 2, 1])]:
        orders = I.all_orders(2)
        mapped = np.vectorize(lambda m: 3 * fmap[m // 3] + smap[m % 3])(orders)
        b2 = I._batch(x0, np.array([goal2]), inst, mapped, (5, 5))
        r2 = orc.evaluate(b2["x0"], b2["goal"], b2["inst"], b2["nseg"], b2["modes"], b2["knots"])
        margin = (r0["viol"] <= 1e-6) | (r0["viol"] >= 1e-5 + 1e-3)
        assert np.array_equal(r0["feasible"][margin], r2["feasible"][margin])
        both = (r0["feasible"] == 1) & (r2["feasible"] == 1)
        rel = np.abs(r0["cost"][both] - r2["cost"][both]) / np.maximum(np.abs(r0["cost"][both]), 1e-12)
        assert rel.max(initial=0) <= 1e-8, rel.max()


def test_duplicate_segments_merge_into_one(orc):
    """(A, A, B) with (n1, n2, n3) intervals is the same NLP as (A, B) with (n1+n2, n3):
    the boundary between two equal modes masks no row (Sec. III-C fixed rows)."""
    x0, goal, inst = I.push_pairs(3, 4)
    modes3 = np.zeros((4, 6), np.int32)
    knots3 = np.zeros((4, 6), np.int32)
    modes2 = np.zeros((4, 6), np.int32)
    knots2 = np.zeros((4, 6), np.int32)
    for i, (a, bb) in enumerate([(6, 1), (4, 10), (0, 8), (11, 2)]):
        modes3[i, :3] = (a, a, bb)
        knots3[i, :3] = (3, 2, 5)
        modes2[i, :2] = (a, bb)
        knots2[i, :2] = (5, 5)
    r3 = orc.evaluate(x0, goal, inst, np.full(4, 3), modes3, knots3)
    r2 = orc.evaluate(x0, goal, inst, np.full(4, 2), modes2, knots2)
    assert np.array_equal(r3["cost"], r2["cost"]) and np.array_equal(r3["viol"], r2["viol"])
    assert np.array_equal(r3["traj"], r2["traj"])


def test_converged_solve_is_a_kkt_point_for_slsqp(orc):
    """An independent NLP solver (scipy SLSQP) started at the oracle's converged point
    finds no better feasible point of the same transcription (Eq. 2)."""
    from scipy.optimize import minimize
    S = orc.Seq([6, 7], [3, 3], goal=(0.1, 0.0, 0.2), mu=0.4)
    modes = np.zeros((1, 6), np.int32)
    knots = np.zeros((1, 6), np.int32)
    modes[0, :2] = (6, 7)
    knots[0, :2] = (3, 3)
    r = orc.evaluate(np.zeros((1, 4)), np.array([[0.1, 0.0, 0.2]]), np.array([[0.4]]), np.array([2]), modes,
                     knots, params=orc.Params(**TIGHT))
    assert r["feasible"][0] == 1 and r["stats"][0, 3] == 1
    z0 = traj_to_z(r["traj"][0], S.N)

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
    assert abs(r["cost"][0] - obj(z0)) < 1e-12
    assert not (vr <= 1e-8 and Jr < r["cost"][0] - 1e-6), (Jr, r["cost"][0])


def test_invalid_inputs_score_as_infeasible(orc):
    """Out-of-range mode ids and non-finite inputs give cost NaN, violation +inf."""
    x0 = np.zeros((3, 4))
    goal = np.array([[0.1, 0, 0], [np.nan, 0, 0], [0.1, 0, 0]])
    inst = np.array([[0.4], [0.4], [0.4]])
    modes = np.zeros((3, 6), np.int32)
    knots = np.zeros((3, 6), np.int32)
    modes[:, 0] = (6, 6, 12)
    knots[:, 0] = 5
    r = orc.evaluate(x0, goal, inst, np.ones(3, np.int32), modes, knots)
    assert r["feasible"][0] == 1
    assert np.isnan(r["cost"][1]) and np.isinf(r["viol"][1]) and r["feasible"][1] == 0
    assert np.isnan(r["cost"][2]) and np.isinf(r["viol"][2]) and r["feasible"][2] == 0


def test_warm_start_at_a_kkt_point_stays_there(orc):
    """A solve started from a converged point with the tight warm-start penalty returns that
    point: the straight sticking push (closed-form optimum d^2 / (v_ref^2 T)) warm-started at
    its own solution keeps the closed-form cost, and a warm start does not cost more
    Gauss-Newton iterations than the schedule-derived start on converged orders."""
    d, N = 0.05, 10
    x0 = np.zeros((1, 4))
    goal = np.array([[d, 0.0, 0.0]])
    inst = np.array([[0.4]])
    modes = np.zeros((1, 6), np.int32)
    knots = np.zeros((1, 6), np.int32)
    modes[0, 0], knots[0, 0] = 6, N
    tight = orc.Params(**TIGHT)
    r = orc.evaluate(x0, goal, inst, np.ones(1, np.int32), modes, knots, params=tight)
    rw = orc.evaluate(x0, goal, inst, np.ones(1, np.int32), modes, knots, warm=r["traj"], params=tight)
    closed = d * d / (N * DT)
    assert rw["feasible"][0] == 1 and rw["stats"][0, 3] == 1
    assert abs(rw["cost"][0] - closed) <= 1e-8 * closed
    assert rw["stats"][0, 1] < r["stats"][0, 1]
    b = I.subset(I.push_tiny(), np.arange(0, 1152, 9))
    p = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"])
    w = orc.evaluate(b["x0"], b["goal"], b["inst"], b["nseg"], b["modes"], b["knots"], warm=p["traj"])
    conv = (p["stats"][:, 3] == 1) & (w["stats"][:, 3] == 1)
    assert conv.sum() >= 20
    assert w["stats"][conv, 1].mean() < p["stats"][conv, 1].mean()
    both = conv & (p["feasible"] == 1) & (w["feasible"] == 1)
    rel = np.abs(w["cost"][both] - p["cost"][both]) / np.maximum(np.abs(p["cost"][both]), 1e-12)
    assert np.median(rel) < 1e-4 and np.quantile(rel, 0.9) < 1e-3   # same optimum, default tolerances
