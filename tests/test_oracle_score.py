"""Pins of the oracle's scoring and ranking against independent restatements.

* Eq. (4): the physical-unit objective and violation of a trajectory, recomputed here in
  NumPy from the quasi-static pushing law written through the contact wrench (no row
  scaling: the reported violation is in the units of each row).
* Eq. (5): the merit M = J + mu max(v - eps, 0) with NaN ranked as +inf, and the pushing
  batch-construction step of Alg. 1 (rank the evaluated orders by increasing merit, ties by
  key; traverse at most W of them; admit unseen one-edit neighbours in enumeration order),
  recomputed by set-based Python and compared with the oracle's step and with the batches
  of a whole oracle expansion.
* The network's pushing input encoding against vectors written out by hand.
"""
import numpy as np
import pytest

from paper_2609_21803_amd import instances as I

DT, A_SIDE, FMAX, VREF = 0.1, 0.1, 0.5 * 1.0 * 9.81, 1.0
CLS = A_SIDE * (np.sqrt(2) + np.log(1 + np.sqrt(2))) / 6
EPS = 1e-5


# ---------------------------------------------------------------------------------
# Eq. (4) in NumPy
# ---------------------------------------------------------------------------------
def _face_frame(face):
    ang = face * np.pi / 2
    return np.array([np.cos(ang), np.sin(ang)]), np.array([-np.sin(ang), np.cos(ang)])


def _euler(x, u, face):
    """x_{k+1} of the quasi-static law: contact force F = -F_n n + F_t t applied at
    p = (a/2) n + s t, wrench (F, p x F), body twist (v_ref / f_max) diag(1, 1, 1/c_ls^2)
    times the wrench, rotated into the world; the contact coordinate moves with v_s."""
    n, t = _face_frame(face)
    p = 0.5 * A_SIDE * n + x[3] * t
    F = -u[0] * n + u[1] * t
    tau = p[0] * F[1] - p[1] * F[0]
    tw = (VREF / FMAX) * np.array([F[0], F[1], tau / CLS ** 2])
    c, s = np.cos(x[2]), np.sin(x[2])
    return np.array([x[0] + DT * (c * tw[0] - s * tw[1]), x[1] + DT * (s * tw[0] + c * tw[1]),
                     x[2] + DT * tw[2], x[3] + DT * u[2]])


def _score_np(x0, goal, mu, modes, knots, X, U):
    """Objective sum dt ((F_n^2 + F_t^2) / f_max^2 + (v_s / v_ref)^2) and the largest
    violation of any enabled row in physical units: defects (the contact-coordinate defect
    dropped on the last interval of a segment followed by another face), the mode row
    (stick: v_s = 0; slide+-: F_t = +-mu F_n), F_n >= 0, the cone (stick) or slip sign
    (slide), |s_{k+1}| <= a/2, and the terminal pose."""
    J, v = 0.0, 0.0
    k = 0
    for j, (m, n) in enumerate(zip(modes, knots)):
        face, slip = m // 3, m % 3
        nxt = modes[j + 1] if j + 1 < len(modes) else m
        for i in range(n):
            x, u, x1 = X[k], U[k], X[k + 1]
            J += DT * ((u[0] ** 2 + u[1] ** 2) / FMAX ** 2 + (u[2] / VREF) ** 2)
            d = x1 - _euler(x, u, face)
            if i == n - 1 and nxt // 3 != face:
                d = d[:3]
            v = max(v, np.abs(d).max())
            sg = (0.0, 1.0, -1.0)[slip]
            v = max(v, abs(u[2]) if slip == 0 else abs(u[1] - sg * mu * u[0]))
            ineq = [-u[0], x1[3] - A_SIDE / 2, -x1[3] - A_SIDE / 2]
            ineq += [u[1] - mu * u[0], -u[1] - mu * u[0]] if slip == 0 else [-sg * u[2]]
            v = max(v, max(0.0, max(ineq)))
            k += 1
    v = max(v, np.abs(X[-1][:3] - goal).max())
    return J, v


def _rollout(x0, modes, knots, U):
    X = [np.asarray(x0, np.float64)]
    k = 0
    for m, n in zip(modes, knots):
        for _ in range(n):
            X.append(_euler(X[-1], U[k], m // 3))
            k += 1
    return np.array(X)


def _to_z(X, U):
    N = len(U)
    z = np.zeros(N * 7)
    for k in range(N):
        z[k * 7:k * 7 + 3] = U[k]
        z[k * 7 + 3:k * 7 + 7] = X[k + 1]
    return z


def _consistent_case(modes, knots, mu, rng):
    """Controls that satisfy every mode row, rolled out exactly: zero defects and mode
    rows; the terminal goal is the rolled-out pose (so only planted violations remain)."""
    U = []
    for m, n in zip(modes, knots):
        slip = m % 3
        for _ in range(n):
            fn = rng.uniform(0.5, 2.0)
            if slip == 0:
                U.append([fn, rng.uniform(-0.5, 0.5) * mu * fn, 0.0])
            else:
                sg = 1.0 if slip == 1 else -1.0
                U.append([fn, sg * mu * fn, sg * rng.uniform(0.0, 0.05)])
    U = np.array(U)
    X = _rollout(np.zeros(4), modes, knots, U)
    return X, U


def _oracle_score(orc, modes, knots, goal, mu, X, U):
    s = orc.Seq(modes, knots, x0=(0, 0, 0, 0), goal=goal, mu=mu)
    return s.score(_to_z(X, U))


PLANTS = ["x-defect", "theta-defect", "cone", "face", "terminal", "slip-sign", "masked-s"]


@pytest.mark.parametrize("plant", PLANTS)
def test_score_equals_numpy_violation_with_planted_maximum(orc, plant):
    """One violation planted in an otherwise consistent trajectory decides v-hat; the
    oracle reports it in physical units (an x-defect of 0.02 is 0.02, not 0.02 over the
    row scale sqrt(2) of the defect rows), and the objective is the NumPy sum."""
    rng = np.random.default_rng(900 + PLANTS.index(plant))
    mu = 0.4
    modes, knots = [0, 8, 4], [4, 3, 5]          # stick on face 0, slide- on face 2, slide+ on face 1
    X, U = _consistent_case(modes, knots, mu, rng)
    U2 = U.copy()
    goal = X[-1, :3].copy()
    expect = None
    if plant == "x-defect":
        X[5, 0] += 0.02
        expect = 0.02
    elif plant == "theta-defect":
        X[2, 2] -= 0.03
        expect = 0.03
    elif plant == "cone":
        U2[1, 1] = U2[1, 0] * mu + 0.3              # stick interval: F_t beyond mu F_n by 0.3
        X = _rollout(np.zeros(4), modes, knots, U2)
        goal = X[-1, :3].copy()
        expect = 0.3
    elif plant == "face":
        X[3, 3] = A_SIDE / 2 + 0.011
        expect = None                               # also moves the neighbouring s-defects
    elif plant == "terminal":
        goal = goal + np.array([0.0, -0.04, 0.0])
        expect = 0.04
    elif plant == "slip-sign":
        U2[5, 2] = 0.07                             # slide- interval: v_s must be <= 0
        X = _rollout(np.zeros(4), modes, knots, U2)
        goal = X[-1, :3].copy()
        expect = 0.07
    elif plant == "masked-s":
        # the last interval of segment 0 precedes a face change: its s-defect is not a
        # row, so a jump of the contact coordinate there is free
        X[4, 3] += 0.03
        Xr = _rollout(X[4], modes[1:], knots[1:], U2[4:])
        X[4:] = Xr
        goal = X[-1, :3].copy()
        expect = 0.0
    Jn, vn = _score_np(np.zeros(4), goal, mu, modes, knots, X, U2)
    Jo, vo = _oracle_score(orc, modes, knots, goal, mu, X, U2)
    if expect is not None:
        assert abs(vn - expect) <= 1e-12, (vn, expect)
    assert abs(vo - vn) <= 1e-15 + 1e-14 * vn, (plant, vo, vn)
    assert abs(Jo - Jn) <= 1e-14 * Jn, (Jo, Jn)


def test_score_equals_numpy_on_random_trajectories(orc):
    """Generic trajectories (every row violated by some amount), all 12 ids."""
    rng = np.random.default_rng(44)
    for it in range(60):
        K = int(rng.integers(1, 4))
        modes = [int(m) for m in rng.integers(0, 12, K)]
        knots = [int(n) for n in rng.integers(1, 5, K)]
        N = sum(knots)
        mu = rng.uniform(0.3, 0.5)
        U = rng.normal(size=(N, 3)) * np.array([1.0, 0.5, 0.05])
        X = np.concatenate([np.zeros((1, 4)), rng.normal(size=(N, 4)) * np.array([0.1, 0.1, 0.5, 0.03])])
        goal = rng.normal(size=3) * 0.2
        Jn, vn = _score_np(np.zeros(4), goal, mu, modes, knots, X, U)
        Jo, vo = _oracle_score(orc, modes, knots, goal, mu, X, U)
        assert abs(vo - vn) <= 1e-15 + 1e-14 * vn, (it, vo, vn)
        assert abs(Jo - Jn) <= 1e-14 * Jn


def test_converged_solves_report_their_numpy_score(orc):
    """The score of returned trajectories (tiny workload) recomputed from the trajectory
    rows in NumPy: cost and violation agree, so a feasible flag is v-hat <= 1e-5 of Eq. (4)."""
    b = I.subset(I.push_tiny(), np.arange(0, 1152, 37))
    f32 = lambda a: np.asarray(a, np.float32).astype(np.float64)
    r = orc.evaluate(f32(b["x0"]), f32(b["goal"]), f32(b["inst"]), b["nseg"], b["modes"], b["knots"], nmax=10)
    for i in range(len(b["nseg"])):
        K = int(b["nseg"][i])
        modes, knots = [int(m) for m in b["modes"][i, :K]], [int(n) for n in b["knots"][i, :K]]
        T = r["traj"][i]
        Jn, vn = _score_np(np.zeros(4), f32(b["goal"])[i], float(f32(b["inst"])[i, 0]), modes, knots,
                           T[:, :4], T[:-1, 4:7])
        assert abs(r["cost"][i] - Jn) <= 1e-12 * max(Jn, 1e-12) and abs(r["viol"][i] - vn) <= 1e-15 + 1e-12 * vn
        assert r["feasible"][i] == (vn <= EPS)


# ---------------------------------------------------------------------------------
# Eq. (5) and the pushing batch-construction step of Alg. 1
# ---------------------------------------------------------------------------------
def _merit_py(J, v, eps=EPS, mu=100.0):
    if np.isnan(J) or np.isnan(v):
        return np.inf
    M = J + mu * max(v - eps, 0.0)
    return np.inf if np.isnan(M) else M


def test_merit_is_equation_5(orc):
    """M = J + 100 max(v - eps, 0): a feasible order ranks by its cost alone, an infeasible
    one pays 100 per unit of violation beyond eps; NaN and +inf rank last."""
    cases = [(0.3, 0.0), (0.3, 1e-5), (0.3, 2e-5), (0.3, 0.01), (2.0, 1.0), (0.0, np.inf), (np.inf, 0.0),
             (np.nan, 0.0), (0.2, np.nan), (-0.1, 0.5), (np.inf, np.inf)]
    for J, v in cases:
        assert orc.merit(J, v) == _merit_py(J, v), (J, v)
    assert orc.merit(0.3, 0.01) == 0.3 + 100 * (0.01 - 1e-5)
    assert orc.merit(0.3, 1e-6) == 0.3


def _key(m):
    k = len(m) << 60
    for i, x in enumerate(m):
        k |= int(x) << (50 - 10 * i)
    return k


def _edit1_list(m, M, kcap):
    """one-edit orders in enumeration order: substitutions (position, then id), deletions
    (position), insertions (position, then id); duplicates kept (first occurrence wins
    later)"""
    K, out = len(m), []
    for i in range(K):
        for a in range(M):
            if a != m[i]:
                out.append(m[:i] + (a,) + m[i + 1:])
    if K > 1:
        for i in range(K):
            out.append(m[:i] + m[i + 1:])
    if K < kcap:
        for i in range(K + 1):
            for a in range(M):
                out.append(m[:i] + (a,) + m[i:])
    return out


def _next_batch_py(V, J, v, kcap, W, room, M=12):
    """Rank V by (Eq. 5 merit, key) increasing, traverse at most W, admit unseen one-edit
    neighbours in enumeration order until room orders are admitted."""
    merit = [_merit_py(a, b) for a, b in zip(J, v)]
    order = sorted(range(len(V)), key=lambda i: (merit[i], _key(V[i])))
    seen = set(V)
    out = []
    for i in order[:W]:
        for nb in _edit1_list(V[i], M, kcap):
            if len(out) >= room:
                return out
            if nb in seen:
                continue
            seen.add(nb)
            out.append(nb)
    return out


@pytest.mark.parametrize("kcap,W,room,seed", [(3, 4, 300, 0), (3, 40, 5000, 1), (2, 200, 100000, 2),
                                              (4, 7, 1000, 3)])
def test_pushing_batch_step_matches_python_twin(orc, kcap, W, room, seed):
    """oracle.expand_next on the oracle's own Eq. (5) merits equals the set-based twin,
    with ties in merit (broken by key), NaN and +inf costs and violations."""
    rng = np.random.default_rng(seed)
    V = sorted({tuple(int(x) for x in rng.integers(0, 12, int(rng.integers(1, kcap + 1)))) for _ in range(80)})
    n = len(V)
    J = rng.choice([0.1, 0.25, 0.5, 1.0, np.inf, np.nan], n, p=[0.3, 0.2, 0.2, 0.1, 0.1, 0.1])
    v = rng.choice([0.0, 5e-6, 1e-3, 0.01, np.inf, np.nan], n, p=[0.3, 0.2, 0.2, 0.1, 0.1, 0.1])
    keys = np.array([_key(m) for m in V], np.uint64)
    merit = np.array([orc.merit(a, b) for a, b in zip(J, v)])
    got = orc.expand_next(keys, merit, n_modes=12, kcap=kcap, radius=1, frontier_W=W, room=room)
    ref = _next_batch_py(V, J, v, kcap, W, room)
    assert [tuple(orc.key_modes(int(k))) for k in got] == ref
    # the ranking direction: reversing the merits changes the batch unless W covers V
    if W < n and len(ref) == room:
        rev = orc.expand_next(keys, -np.where(np.isinf(merit), 1e300, merit), 12, kcap, 1, W, room)
        assert [tuple(orc.key_modes(int(k))) for k in rev] != ref


def test_whole_expansion_batches_equal_python_twin(orc):
    """Every batch of a whole oracle expansion equals the twin's batch built from the
    oracle's own (J, v) of the orders evaluated before it (seed: all orders of at most
    seed_max_segments segments in key order)."""
    x0, goal, inst = I.push_pairs(77, 1)
    ep = orc.Expand(kcap=3, seed_max_segments=1, radius=1, rounds=3, frontier_W=6, knots_per_segment=4, k_ref=4,
                    batch_B=150, eval_budget=100000)
    r = orc.expand(x0[0], goal[0], inst[0, 0], ep, eval_cap=100000)
    keys = [tuple(orc.key_modes(k)) for k in r["eval_keys"]]
    J, v = list(r["eval_cost"]), list(r["eval_viol"])
    seed = [(m,) for m in range(12)]
    assert keys[:12] == seed
    pos = 12
    while pos < len(keys):
        nb = _next_batch_py(keys[:pos], J[:pos], v[:pos], ep.kcap, ep.frontier_W, ep.batch_B)
        assert keys[pos:pos + len(nb)] == nb
        pos += len(nb)
    assert r["rounds"] == ep.rounds + 1


# ---------------------------------------------------------------------------------
# Network input encoding (pushing)
# ---------------------------------------------------------------------------------
def test_encode_push_hand_written_vectors():
    """Layout: 16 pose entries (start x, y, cos, sin; goal x, y, cos, sin; goal - start
    x, y, angle; friction; four zeros), then six slots of 64: one-hot id (12), intervals / 15,
    presence flag, zeros; absent segments all zero."""
    from oracle.mlp import encode_push
    x0 = np.array([[0.0, 0.0, 0.0, 0.0], [0.1, -0.2, np.pi, 0.0]])
    goal = np.array([[0.25, -0.125, 0.0], [0.5, 0.0, 0.0]])
    inst = np.array([[0.375], [0.5]])
    nseg = np.array([3, 1], np.int32)
    modes = np.array([[7, 0, 11, 0, 0, 0], [4, 0, 0, 0, 0, 0]], np.int32)
    knots = np.array([[8, 5, 15, 0, 0, 0], [3, 0, 0, 0, 0, 0]], np.int32)
    X = encode_push(x0, goal, inst, nseg, modes, knots)
    E = np.zeros((2, 416))
    E[0, [2, 6]] = 1.0                         # cos 0 of start and goal
    E[0, 4], E[0, 5] = 0.25, -0.125
    E[0, 8], E[0, 9] = 0.25, -0.125
    E[0, 11] = 0.375
    E[0, 16 + 7], E[0, 16 + 12], E[0, 16 + 13] = 1.0, 8 / 15, 1.0
    E[0, 80 + 0], E[0, 80 + 12], E[0, 80 + 13] = 1.0, 5 / 15, 1.0
    E[0, 144 + 11], E[0, 144 + 12], E[0, 144 + 13] = 1.0, 1.0, 1.0
    E[1, 0], E[1, 1], E[1, 2], E[1, 3] = 0.1, -0.2, -1.0, 0.0
    E[1, 4], E[1, 5], E[1, 6], E[1, 7] = 0.5, 0.0, 1.0, 0.0
    E[1, 8], E[1, 9], E[1, 10] = 0.4, 0.2, -np.pi
    E[1, 11] = 0.5
    E[1, 16 + 4], E[1, 16 + 12], E[1, 16 + 13] = 1.0, 3 / 15, 1.0
    assert X.shape == (2, 416)
    assert np.allclose(X, E, rtol=0, atol=2e-7), np.argwhere(~np.isclose(X, E, rtol=0, atol=2e-7))
