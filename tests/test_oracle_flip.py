"""Pins of the FP64 flip oracle against facts that do not come from the oracle itself:
central finite differences, an independent world-frame wrench balance, the static box at
rest, mirror symmetry of the box, a dense linear solve, and a brute-force count of the
mode language."""
import itertools

import numpy as np
import pytest

from oracle import flip as F

fid, fg = F.mode_id, F.finger
MG = 0.5 * 9.81
W, H = 0.2, 0.1


def pivot_goal_px(th, px0=0.0):
    """centre x after pivoting from rest (centre px0) about the bottom-left corner to th"""
    c = np.array([-W / 2, -H / 2])
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    return px0 - W / 2 - (R @ c)[0]


# orders used by several pins: face-supported, sliding and pivoting, one and two fingers
ORDERS = [
    ([fid(fg(0, 1), 0, 0), fid(fg(0, 0), 0, 3)], [4, 5]),
    ([fid(0, 0, 0), fid(fg(0, 0), fg(1, 0), 3)], [3, 4]),
    ([fid(fg(2, 0), 0, 1)], [5]),
    ([fid(fg(2, 2), fg(1, 1), 2)], [4]),
    ([fid(fg(1, 0), fg(2, 0), 4)], [5]),
    ([fid(0, fg(0, 0), 3), fid(fg(1, 1), 0, 0)], [3, 3]),
]


def _rand_args(rng):
    v = rng.normal(size=F.NV) * 0.3
    v[[2, F.NV - 6]] = rng.uniform(-0.5, 2.0, 2)   # angles
    return v


@pytest.mark.parametrize("oi", range(len(ORDERS)))
def test_complex_step_jacobian_matches_central_differences(oi):
    """Every row's complex-step Jacobian equals central differences of the real rows."""
    m, kn = ORDERS[oi]
    S = F.Seq(m, kn, goal=(0.1, 1.0), mu_g=0.66)
    rng = np.random.default_rng(oi)
    for k in (0, S.N - 1):
        v = _rand_args(rng)
        c, J, en = S.rows(k, v)
        c_real, en2 = S.rows(k, v, complex_step=False)
        assert np.array_equal(en, en2)
        assert np.allclose(c, c_real, rtol=1e-14, atol=1e-14)
        h = 1e-6
        Jfd = np.zeros_like(J)
        for j in range(F.NV):
            e = np.zeros(F.NV)
            e[j] = h
            Jfd[:, j] = (S.rows(k, v + e, complex_step=False)[0] - S.rows(k, v - e, complex_step=False)[0]) / (2 * h)
        assert np.allclose(J, Jfd, rtol=1e-6, atol=1e-7), np.abs(J - Jfd).max()


def _world_wrench(face_codes, v):
    """Independent world-frame statics: contact points and forces rotated into the world,
    table reaction from the force balance, moments by 2-D cross products."""
    th = v[2]
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    ctr = v[0:2]
    pts, frc = [], []
    for i, code in enumerate(face_codes):
        if code == 0:
            continue
        face = (code - 1) // 3
        ang = face * np.pi / 2
        n = np.array([np.cos(ang), np.sin(ang)])
        t = np.array([-np.sin(ang), np.cos(ang)])
        h = W / 2 if face % 2 == 0 else H / 2
        s = v[6 + i]
        fn, ft = v[F.NX + 3 + 3 * i], v[F.NX + 4 + 3 * i]
        pts.append(ctr + R @ (h * n + s * t))
        frc.append(R @ (-fn * n + ft * t))
    r = -sum(frc, np.zeros(2)) + np.array([0.0, MG])
    cross = lambda a, b: a[0] * b[1] - a[1] * b[0]
    return ctr, R, pts, frc, r, cross


@pytest.mark.parametrize("seed", range(4))
def test_pivot_and_support_rows_match_world_frame_statics(seed):
    """The pivot moment row equals the world-frame moment balance about the corner; the
    centre-of-pressure rows equal the support-face bound on -(moment about the centre)/r_y
    (Sec. IV-B: quasi-static wrench balance with the table reaction eliminated)."""
    rng = np.random.default_rng(10 + seed)
    f1, f2 = fg(0, 0), fg(1, 1)
    for g, dirn in ((3, 1.0), (4, -1.0)):
        S = F.Seq([fid(f1, f2, g)], [3])
        v = _rand_args(rng)
        c, _, en = S.rows(0, v)
        ctr, R, pts, frc, r, cross = _world_wrench((f1, f2), v)
        cb = np.array([-dirn * W / 2, -H / 2])           # bottom-left / bottom-right corner of face 3
        corner = ctr + R @ cb
        mom = sum(cross(p - corner, f) for p, f in zip(pts, frc)) + cross(ctr - corner, np.array([0.0, -MG]))
        assert np.isclose(c[14], mom / (MG * W), rtol=1e-12, atol=1e-12)
        assert np.isclose(c[27], -r[1] / MG, rtol=1e-12, atol=1e-12)
        mu_g = S.mu_g
        assert np.isclose(c[30], (r[0] - mu_g * r[1]) / MG, atol=1e-12)
        # corner no-slip and height rows
        x1 = v[F.NX + F.NU:]
        R1 = np.array([[np.cos(x1[2]), -np.sin(x1[2])], [np.sin(x1[2]), np.cos(x1[2])]])
        c1 = x1[0:2] + R1 @ cb
        assert np.isclose(c[12], c1[0] - corner[0], atol=1e-12) and np.isclose(c[13], c1[1], atol=1e-12)
    S = F.Seq([fid(f1, f2, 0)], [3])
    v = _rand_args(rng)
    c, _, en = S.rows(0, v)
    ctr, R, pts, frc, r, cross = _world_wrench((f1, f2), v)
    tau_ctr = sum(cross(p - ctr, f) for p, f in zip(pts, frc))
    # support face 3 horizontal: centre of pressure at ctr + (d, -H/2) with tau + d r_y + (H/2) r_x = 0
    assert np.isclose(c[28], (tau_ctr + H / 2 * r[0] - W / 2 * r[1]) / (MG * W), atol=1e-12)
    assert np.isclose(c[29], (-tau_ctr - H / 2 * r[0] - W / 2 * r[1]) / (MG * W), atol=1e-12)


def test_box_at_rest_is_feasible_at_zero_cost():
    """Goal = start, fingers free, table stick: the box at rest is the optimum (J = 0)."""
    r = F.evaluate(F.X0[None], np.array([[0.0, 0.0]]), np.array([0.7]), np.array([2]),
                   np.array([[fid(0, 0, 0), fid(fg(0, 0), 0, 0), 0, 0, 0, 0]]), np.array([[4, 4, 0, 0, 0, 0]]))
    assert r["feasible"][0] == 1 and r["stats"][0, 3] == 1
    assert abs(r["cost"][0]) < 1e-8   # stopping tolerance: optimum J = 0


def _mirror_id(mid):
    f1, f2, g = mid // 65, (mid // 5) % 13, mid % 5

    def mf(code):
        if code == 0:
            return 0
        face, slip = (code - 1) // 3, (code - 1) % 3
        face = {0: 2, 2: 0}.get(face, face)
        slip = {1: 2, 2: 1}.get(slip, slip)
        return 1 + 3 * face + slip
    return fid(mf(f1), mf(f2), {1: 2, 2: 1, 3: 4, 4: 3}.get(g, g))


def test_mirror_symmetry_of_the_box():
    """Reflecting the plane x -> -x maps faces 0 <-> 2, slide+ <-> slide-, pivot left <->
    right and the goal (px, th) -> (-px, -th): the same NLP, hence the same cost,
    violation and flag (exact up to rounding)."""
    rng = np.random.default_rng(5)
    orders = [
        ([fid(fg(0, 1), 0, 0), fid(fg(0, 0), 0, 3)], [10, 10], (pivot_goal_px(1.2), 1.2)),
        ([fid(0, 0, 0), fid(fg(0, 0), fg(1, 0), 3)], [10, 10], (pivot_goal_px(1.0), 1.0)),
        ([fid(fg(2, 0), 0, 1)], [8], (0.05, 0.0)),
        ([fid(fg(2, 1), fg(1, 2), 0), fid(fg(2, 0), 0, 1)], [5, 6], (0.03, 0.0)),
    ]
    for m, kn, goal in orders:
        mu = rng.uniform(0.62, 0.78)
        K = len(m)
        mm = np.zeros((2, 6), np.int32)
        kk = np.zeros((2, 6), np.int32)
        mm[0, :K] = m
        mm[1, :K] = [_mirror_id(x) for x in m]
        kk[:, :K] = kn
        r = F.evaluate(np.stack([F.X0, F.X0]), np.array([goal, (-goal[0], -goal[1])]), np.array([mu, mu]),
                       np.array([K, K]), mm, kk)
        assert r["feasible"][0] == r["feasible"][1]
        assert np.isclose(r["cost"][0], r["cost"][1], rtol=1e-7, atol=1e-12), r["cost"]
        assert np.isclose(r["viol"][0], r["viol"][1], rtol=1e-5, atol=1e-12), r["viol"]
        T0, T1 = r["traj"][0], r["traj"][1]
        sign = np.array([-1, 1, -1, -1, 1, -1, -1, -1, -1, 1, -1, 1, -1, -1, 1, -1, -1])
        assert np.allclose(T1, T0 * sign, atol=1e-6)


def test_feasible_flips_satisfy_the_physics():
    """Converged feasible pivots: dynamics, finger cones and unilateral contacts hold when
    recomputed from the returned trajectory."""
    cases = [([fid(fg(0, 1), 0, 0), fid(fg(0, 0), 0, 3)], [10, 10], (pivot_goal_px(1.2), 1.2)),
             ([fid(0, 0, 0), fid(fg(0, 0), fg(1, 0), 3)], [10, 10], (pivot_goal_px(1.2), 1.2))]
    for m, kn, goal in cases:
        K = len(m)
        mm = np.zeros((1, 6), np.int32)
        kk = np.zeros((1, 6), np.int32)
        mm[0, :K], kk[0, :K] = m, kn
        r = F.evaluate(F.X0[None], np.array([goal]), np.array([0.7]), np.array([K]), mm, kk)
        assert r["feasible"][0] == 1 and r["stats"][0, 3] == 1
        T = r["traj"][0]
        N = sum(kn)
        dt = 0.1
        x, u = T[:N + 1, :8], T[:N, 8:]
        rates = np.stack([x[:N, 3], x[:N, 4], x[:N, 5], u[:, 0], u[:, 1], u[:, 2], u[:, 5], u[:, 8]], 1)
        assert np.abs(x[1:] - x[:N] - dt * rates).max() < 1e-5
        assert abs(x[N, 0] - goal[0]) < 1e-5 and abs(x[N, 2] - goal[1]) < 1e-5
        assert (u[:, 3] > -1e-5 * MG).all() and (np.abs(u[:, 4]) <= 0.5 * u[:, 3] + 1e-5 * MG).all()
        # table reaction stays in its cone with r_y >= 0 (from the world-frame statics)
        for k in range(N):
            v = np.concatenate([x[k], u[k], x[k + 1]])
            codes = (m[0] // 65, (m[0] // 5) % 13) if k < kn[0] else (m[-1] // 65, (m[-1] // 5) % 13)
            *_, rr, _ = _world_wrench(codes, v)
            assert rr[1] > -1e-5 * MG and abs(rr[0]) <= 0.7 * rr[1] + 1e-5 * MG


@pytest.mark.parametrize("oi", [0, 1, 3])
def test_gauss_newton_step_equals_dense_kkt_solve(oi):
    """The Riccati recursion returns the solution of the dense system (H + rho I) dz = -g,
    H = cost Hessian + (1/mu) sum over equality and active inequality rows of a a^T, built
    here from the rows' Jacobians without any recursion."""
    m, kn = ORDERS[oi]
    S = F.Seq(m, kn, goal=(0.05, 0.8), mu_g=0.7)
    rng = np.random.default_rng(oi)
    z = S.initial() + rng.normal(size=S.N * F.NW) * 0.01
    lam = rng.normal(size=S.N * F.NE) * 0.1
    nu = np.abs(rng.normal(size=S.N * F.NI)) * 0.1
    lamT = rng.normal(size=F.NT) * 0.1
    mu, rho = 0.05, 1e-3
    phi, g, dz = S.merit_grad_step(z, lam, nu, lamT, mu, rho)
    n = S.N * F.NW
    Hd = np.zeros((n, n))
    dt, mg2 = 0.1, MG * MG
    wu = np.array([1e-2, 1e-2, 1e-2, 1 / mg2, 1 / mg2, 1e-2, 1 / mg2, 1 / mg2, 1e-2])
    for k in range(S.N):
        idx = np.arange(k * F.NW, k * F.NW + F.NU)
        Hd[idx, idx] += 2 * dt * wu
        c, J, en = S.rows(k, S.args(z, k))
        cols = list(range((k - 1) * F.NW + F.NU, k * F.NW)) if k > 0 else []
        var = np.array(cols + list(range(k * F.NW, (k + 1) * F.NW)))
        Jv = J[:, F.NV - len(var):]
        for r in range(F.NR):
            if not en[r]:
                continue
            if r >= F.NE and nu[k * F.NI + r - F.NE] + c[r] / mu <= 0:
                continue
            Hd[np.ix_(var, var)] += np.outer(Jv[r], Jv[r]) / mu
    xN = np.arange((S.N - 1) * F.NW + F.NU, S.N * F.NW)
    for j in (0, 2, 3, 4, 5):
        Hd[xN[j], xN[j]] += 1 / mu
    ref = np.linalg.solve(Hd + rho * np.eye(n), -g)
    assert dz is not None
    assert np.allclose(dz, ref, rtol=1e-6, atol=1e-9 * np.abs(ref).max())


def test_merit_gradient_matches_central_differences():
    m, kn = ORDERS[0]
    S = F.Seq(m, kn, goal=(0.05, 0.8), mu_g=0.7)
    rng = np.random.default_rng(3)
    z = S.initial() + rng.normal(size=S.N * F.NW) * 0.01
    lam = rng.normal(size=S.N * F.NE) * 0.1
    nu = np.abs(rng.normal(size=S.N * F.NI)) * 0.1
    lamT = rng.normal(size=F.NT) * 0.1
    _, g, _ = S.merit_grad_step(z, lam, nu, lamT, 0.05, 1e-3)
    h = 1e-6
    for j in rng.choice(S.N * F.NW, 40, replace=False):
        e = np.zeros_like(z)
        e[j] = h
        fp = S.merit_grad_step(z + e, lam, nu, lamT, 0.05, 1e-3)[0]
        fm = S.merit_grad_step(z - e, lam, nu, lamT, 0.05, 1e-3)[0]
        assert np.isclose(g[j], (fp - fm) / (2 * h), rtol=1e-5, atol=1e-7)


# ---------------------------------------------------------------------------------
# The mode language: an independent set-based reimplementation of the rules
# ---------------------------------------------------------------------------------
def _faces(mid):
    f1, f2, g = mid // 65, (mid // 5) % 13, mid % 5
    return [None if f == 0 else (f - 1) // 3 for f in (f1, f2)], g


def _admissible_py(seq):
    support, prev_g, prev_faces = 3, None, [None, None]
    for j, mid in enumerate(seq):
        if j and seq[j - 1] == mid:
            return False
        faces, g = _faces(mid)
        if g >= 3 and prev_g is not None and prev_g >= 3 and g != prev_g:
            return False
        if g <= 2 and prev_g is not None and prev_g >= 3:
            support = (support - (1 if prev_g == 3 else -1)) % 4
        touching = {f for f in faces if f is not None}
        if faces[0] is not None and faces[0] == faces[1]:
            return False
        if g >= 3 and not touching:
            return False
        forbidden = {support}
        if g >= 3:
            forbidden.add((support - (1 if g == 3 else -1)) % 4)
        if touching & forbidden:
            return False
        for i in range(2):
            if faces[i] is not None and prev_faces[i] is not None and faces[i] != prev_faces[i]:
                return False
        prev_faces, prev_g = faces, g
    return True


def test_language_single_segment_count_and_brute_force():
    """One-segment orders from the rest pose: 3 x (10^2 - 27) face-supported + 2 x 30
    pivots = 279; two-segment orders agree with the set-based brute force."""
    ones = [m for m in range(F.N_MODES) if F.admissible([m])]
    assert len(ones) == 3 * (100 - 27) + 2 * 30 == 279
    assert ones == [m for m in range(F.N_MODES) if _admissible_py([m])]
    rng = np.random.default_rng(0)
    pairs = [(a, b) for a, b in itertools.product(ones, repeat=2)]
    sample = [pairs[i] for i in rng.choice(len(pairs), 4000, replace=False)]
    for a, b in sample:
        assert F.admissible([a, b]) == _admissible_py([a, b]), (a, b)
    for _ in range(3000):
        K = int(rng.integers(3, 7))
        seq = [int(x) for x in rng.integers(0, F.N_MODES, K)]
        seq[0] = ones[int(rng.integers(len(ones)))]
        assert F.admissible(seq) == _admissible_py(seq)


def test_invalid_orders_score_as_infeasible():
    """Out-of-range ids and a pivot run that changes direction (its corner is undefined)."""
    mm = np.zeros((3, 6), np.int32)
    kk = np.zeros((3, 6), np.int32)
    mm[0, 0] = 845
    mm[1, :2] = (fid(fg(0, 0), 0, 3), fid(fg(1, 0), 0, 4))
    mm[2, 0] = fid(0, 0, 0)
    kk[:, :2] = 3
    r = F.evaluate(np.stack([F.X0] * 3), np.zeros((3, 2)), np.full(3, 0.7), np.array([1, 2, 1]), mm, kk)
    assert np.isnan(r["cost"][0]) and np.isnan(r["cost"][1]) and r["stats"][1, 3] == 3
    assert r["feasible"][2] == 1


# ---------------------------------------------------------------------------------
# Expansion over the flip language (Alg. 1)
# ---------------------------------------------------------------------------------
def _neigh1_py(modes, kcap, M=F.N_MODES):
    """one-edit list in enumeration order (substitutions, deletions, insertions)"""
    K, out = len(modes), []
    for i in range(K):
        for idx in range(M):
            if idx != modes[i]:
                out.append(modes[:i] + [idx] + modes[i + 1:])
    if K > 1:
        for i in range(K):
            out.append(modes[:i] + modes[i + 1:])
    if K < kcap:
        for i in range(K + 1):
            for idx in range(M):
                out.append(modes[:i] + [idx] + modes[i:])
    return out


def _neigh_py(modes, kcap, radius):
    """r-edit list (Sec. III-B): the one-edit list, then, for r = 2, the one-edit lists of
    its admissible entries in order (every intermediate order stays admissible)"""
    l1 = _neigh1_py(modes, kcap)
    if radius < 2:
        return l1
    out = list(l1)
    for q in l1:
        if _admissible_py(q):
            out += _neigh1_py(q, kcap)
    return out


def _expand_next_py(V, merit, kcap, W, room, radius=1):
    order = sorted(range(len(V)), key=lambda i: (merit[i], F.key_make(V[i])))
    seen = {tuple(v) for v in V}
    out = []
    for i in order[:W]:
        for nb in _neigh_py(list(V[i]), kcap, radius):
            if len(out) >= room:
                return out
            t = tuple(nb)
            if t in seen:
                continue
            seen.add(t)
            if _admissible_py(nb):
                out.append(nb)
    return out


def test_seed_is_the_admissible_single_segments_in_key_order():
    s = F.seed(1)
    assert [F.key_modes(int(k)) for k in s] == [[m] for m in range(F.N_MODES) if _admissible_py([m])]


@pytest.mark.parametrize("kcap,W,room,seed,radius", [(2, 3, 500, 0, 1), (3, 8, 4000, 1, 1), (2, 50, 100000, 2, 1),
                                                     (2, 2, 100000, 3, 2), (3, 1, 30000, 4, 2)])
def test_batch_construction_matches_brute_force(kcap, W, room, seed, radius):
    """One batch-construction step: rank by (merit, key), traverse W parents, admit unseen
    admissible one-edit neighbours in enumeration order (independent set-based code)."""
    rng = np.random.default_rng(seed)
    pool = [F.key_modes(int(k)) for k in F.seed(1)]
    V = [pool[i] for i in rng.choice(len(pool), 60, replace=False)]
    V += [V[i] + pool[int(rng.integers(len(pool)))] for i in range(10)]
    V = [v for v in V if _admissible_py(v)]
    merit = rng.choice([0.5, 1.0, 2.0, np.inf], len(V))
    keys = np.array([F.key_make(v) for v in V], np.uint64)
    got = F.expand_next(keys, merit, kcap, radius, W, room)
    ref = _expand_next_py(V, list(merit), kcap, W, room, radius)
    assert [F.key_modes(int(k)) for k in got] == ref


def test_expansion_over_the_whole_single_segment_space_returns_the_enumeration_argmin():
    """With K_cap = 1 the seed is the whole admissible space: the returned plan is the
    refined argmin over all 279 orders, computed here by direct evaluation."""
    goal = (0.04, 0.0)
    ep = oracle_expand_params(kcap=1, seed_max_segments=1, rounds=0, frontier_W=1, knots_per_segment=8, k_ref=4,
                              batch_B=1000, eval_budget=1000)
    bk, bJ, bv, cnt, ek, eJ, ev = F.expand(F.X0, goal, 0.7, ep)
    assert cnt[0] == 279
    ones = [m for m in range(F.N_MODES) if _admissible_py([m])]
    B = len(ones)
    r = F.evaluate(np.tile(F.X0, (B, 1)), np.tile(goal, (B, 1)), np.full(B, 0.7), np.ones(B, np.int32),
                   np.array([[m, 0, 0, 0, 0, 0] for m in ones]), np.array([[8, 0, 0, 0, 0, 0]] * B))
    assert np.array_equal(eJ, r["cost"]) and np.array_equal(ev, r["viol"])
    feas = np.where(r["feasible"] == 1)[0]
    assert len(feas) >= 1 and cnt[2] == len(feas)
    best4 = sorted(feas, key=lambda i: (r["cost"][i], ones[i]))[:4]
    import oracle
    rr = F.evaluate(np.tile(F.X0, (len(best4), 1)), np.tile(goal, (len(best4), 1)), np.full(len(best4), 0.7),
                    np.ones(len(best4), np.int32), np.array([[ones[i], 0, 0, 0, 0, 0] for i in best4]),
                    np.array([[8, 0, 0, 0, 0, 0]] * len(best4)), params=oracle.Params(**oracle.REFINE))
    ok = [j for j in range(len(best4)) if rr["feasible"][j]]
    j = min(ok, key=lambda j: (rr["cost"][j], ones[best4[j]]))
    assert F.key_modes(int(bk)) == [ones[best4[j]]] and bJ == rr["cost"][j]


def oracle_expand_params(**kw):
    import oracle
    e = oracle.Expand()
    for k, v in kw.items():
        setattr(e, k, v)
    return e
