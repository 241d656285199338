"""Pins of the free-motion pushing oracle (the admissible language of Sec. III-A: modes are
contact events or free motion, a contact changes faces only through free motion).

The model adds the pusher position to the state and its velocity to the controls.  What
pins it, beyond its own formulas: the fixed-step pushing model (pinned separately), which
it must reproduce row for row on a face; central differences; a dense solve of the
Gauss-Newton system; closed-form optima (goal = start; a free approach followed by a
straight push); and the language by brute force from an independent transcription of its
rules.  The paper's printed counts of its box language (601 orders of at most six
segments, 6,297 of at most eight) belong to the benchmark's transition system, which the
paper does not state in full: they are printed beside this language's counts, parity
unpinned.
"""
import itertools

import numpy as np
import pytest

from oracle import free as F

DT, HALF = 0.1, 0.05
NORMAL = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0], [0.0, -1.0]])
TIGHT = dict(al_max=80, gn_max=40, eta_star=1e-12, omega_star=1e-11, rc_star=1e-12, mu_min=1e-8)


@pytest.fixture(scope="module")
def orc():
    import oracle
    F.build()
    return oracle


def _free_v(v11, face):
    """pushing v = (x, y, th, s, Fn, Ft, vs, x1, y1, th1, s1) -> free-motion v with the pusher
    on the face: p = (a/2) n + s t, v_p = vs t"""
    n = NORMAL[face]
    t = np.array([-n[1], n[0]])
    p, p1, vp = HALF * n + v11[3] * t, HALF * n + v11[10] * t, v11[6] * t
    return np.concatenate([v11[:3], p, v11[4:6], vp, v11[7:10], p1]), t


@pytest.mark.parametrize("face,slip", list(itertools.product(range(4), range(3))))
def test_contact_rows_reduce_to_the_pushing_rows_on_the_face(orc, face, slip):
    """With the pusher on face j at coordinate s (p = (a/2) n + s t) and moving along it
    (v = v_s t), every contact row equals the fixed-step pushing row it generalises, and
    the Jacobian composed with d v_free / d v_push equals the pushing Jacobian."""
    rng = np.random.default_rng(11 + 3 * face + slip)
    m = F.contact(face, slip)
    for _ in range(4):
        v = rng.normal(size=11) * np.array([0.2, 0.2, 2, 0.04, 2, 1, 0.1, 0.2, 0.2, 2, 0.04])
        cp, Jp, enp = orc.push_rows(face, slip, 1, 0.37, v)
        vf, t = _free_v(v, face)
        c, J, en, _ = F.rows(m, 0.37, vf)
        # free slot -> pushing slot (the defects 3, 4 project on t; slots 5, 6 vanish)
        pairs = [(0, 0), (1, 1), (2, 2), (7, 4), (8, 5), (9, 6), (10, 7), (11, 8), (12, 9)]
        for a, b in pairs:
            assert en[a] == enp[b], (a, b)
            if en[a]:
                assert abs(c[a] - cp[b]) <= 1e-14 * max(1.0, abs(cp[b])), (a, b, c[a], cp[b])
        assert abs(t[0] * c[3] + t[1] * c[4] - cp[3]) <= 1e-15
        assert abs(c[5]) <= 1e-17 and abs(c[6]) <= 1e-17
        assert abs(c[13] - (v[3] - HALF)) <= 1e-16 and abs(c[14] - (-v[3] - HALF)) <= 1e-16
        # chain rule: columns of the pushing v in terms of the free v
        D = np.zeros((14, 11))
        for i in range(3):
            D[i, i] = 1.0
            D[9 + i, 7 + i] = 1.0
        D[3:5, 3] = t
        D[5, 4] = D[6, 5] = 1.0
        D[7:9, 6] = t
        D[12:14, 10] = t
        JD = J @ D
        for a, b in pairs:
            if en[a]:
                assert np.allclose(JD[a], Jp[b], atol=1e-13), (a, b)
        assert np.allclose(t[0] * JD[3] + t[1] * JD[4], Jp[3], atol=1e-15)


@pytest.mark.parametrize("mode", range(16))
def test_row_jacobians_match_central_differences(orc, mode):
    rng = np.random.default_rng(400 + mode)
    scale = np.array([0.2, 0.2, 2, 0.06, 0.06, 2, 1, 0.1, 0.1, 0.2, 0.2, 2, 0.06, 0.06])
    for _ in range(4):
        v = rng.normal(size=14) * scale
        c, J, en, _ = F.rows(mode, 0.37, v)
        Jfd = np.zeros_like(J)
        for j in range(14):
            h = 1e-6 * max(1.0, abs(v[j]))
            vp, vm = v.copy(), v.copy()
            vp[j] += h
            vm[j] -= h
            Jfd[:, j] = (F.rows(mode, 0.37, vp)[0] - F.rows(mode, 0.37, vm)[0]) / (2 * h)
        on = en.astype(bool)
        assert np.allclose(J[on], Jfd[on], rtol=1e-6, atol=1e-8)
        assert not np.any(J[~on]) and not np.any(c[~on])


def test_free_rows_and_the_row_sets(orc):
    """Free motion in front of face j: zero force, no penetration at both knots, no contact
    rows; the enabled rows of every mode."""
    v = np.array([0.1, -0.2, 0.3, 0.07, 0.01, 0.4, -0.2, 0.3, 0.1, 0.12, -0.2, 0.3, 0.1, 0.01])
    for j in range(4):
        c, _, en, _ = F.rows(F.free(j), 0.4, v)
        n = NORMAL[j]
        assert list(np.nonzero(en)[0]) == [0, 1, 2, 3, 4, 5, 6, 8, 9]
        assert c[5] == v[5] and c[6] == v[6]
        assert abs(c[8] - (HALF - n @ v[3:5])) <= 1e-16 and abs(c[9] - (HALF - n @ v[12:14])) <= 1e-16
    for m in range(12):
        en = F.rows(m, 0.4, v)[2]
        want = set(range(15)) - ({10} if m % 3 else set())
        assert set(np.nonzero(en)[0]) == want


def test_cost_and_scales(orc):
    u = np.array([1.3, -0.4, 0.2, -0.7])
    fm = 0.5 * 9.81
    J, g = F.cost(u)
    assert abs(J - DT * ((u[0] ** 2 + u[1] ** 2) / fm ** 2 + u[2] ** 2 + u[3] ** 2)) <= 1e-16
    assert np.allclose(g, DT * 2 * np.array([u[0] / fm ** 2, u[1] / fm ** 2, u[2], u[3]]), rtol=1e-15)
    s = F.scales()
    # unit rows (positions, velocities and forces with unit coefficients) and the cone rows
    for t in (5, 6, 8, 9, 11, 12, 13, 14, 15):
        assert s[t] == 1.0, t
    assert abs(s[7] - np.sqrt(1 + 0.4 ** 2)) <= 1e-15 and abs(s[10] - np.sqrt(1 + 0.4 ** 2)) <= 1e-15
    assert abs(s[3] - np.sqrt(2 + DT ** 2)) <= 1e-15 and abs(s[4] - np.sqrt(2 + DT ** 2)) <= 1e-15
    assert np.all(s[:3] > 1.0)


def _random_point(seed, modes=(15, 9, 15, 12, 0), knots=(3, 2, 3, 2, 2)):
    rng = np.random.default_rng(seed)
    S = F.Seq(modes, knots, goal=(0.08, 0.05, 0.4), mu=0.41)
    z = S.initial() + 0.005 * rng.normal(size=S.N * F.NW)
    lam = 0.1 * rng.normal(size=S.N * F.NE)
    nu = np.abs(0.1 * rng.normal(size=S.N * F.NI))
    lamT = 0.1 * rng.normal(size=3)
    return S, z, lam, nu, lamT


@pytest.mark.parametrize("seed", [0, 1])
def test_merit_gradient_matches_central_differences(orc, seed):
    S, z, lam, nu, lamT = _random_point(seed)
    phi, g, _, _ = S.merit_grad_step(z, lam, nu, lamT, 0.05, 1e-3)
    gfd = np.zeros_like(g)
    for i in range(len(z)):
        zp, zm = z.copy(), z.copy()
        zp[i] += 1e-6
        zm[i] -= 1e-6
        gfd[i] = (S.merit_grad_step(zp, lam, nu, lamT, 0.05, 1e-3)[0] -
                  S.merit_grad_step(zm, lam, nu, lamT, 0.05, 1e-3)[0]) / 2e-6
    assert np.allclose(g, gfd, rtol=1e-5, atol=1e-7), np.abs(g - gfd).max()


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_riccati_step_equals_dense_kkt_solve(orc, seed):
    """The backward Riccati recursion over the 9 stage unknowns gives the step of the dense
    system (H + rho I) dz = -g, with H = sum over active (scaled) rows of a a^T / mu plus the
    cost Hessian."""
    S, z, lam, nu, lamT = _random_point(seed)
    mu_al, rho, N, W, X, U = 0.03, 1e-3, S.N, F.NW, F.NX, F.NU
    _, g, dz, ok = S.merit_grad_step(z, lam, nu, lamT, mu_al, rho)
    assert ok
    sc = F.scales()
    H = np.zeros((W * N, W * N))
    for k in range(N):
        c, J, en, ty = F.rows(S.mode_of(k), S.mu, S.args(z, k))
        cols = ([(k - 1) * W + U + i for i in range(X)] if k > 0 else [None] * X) + [k * W + i for i in range(W)]
        for r in range(F.NR):
            if not en[r]:
                continue
            cs, a_row = c[r] / sc[ty[r]], J[r] / sc[ty[r]]
            if r >= F.NE and not (nu[k * F.NI + r - F.NE] + cs / mu_al > 0):
                continue
            a = np.zeros(W * N)
            for j, col in enumerate(cols):
                if col is not None:
                    a[col] += a_row[j]
            H += np.outer(a, a) / mu_al
        H[k * W:k * W + 2, k * W:k * W + 2] += np.eye(2) * DT * 2 / (0.5 * 9.81) ** 2
        H[k * W + 2:k * W + 4, k * W + 2:k * W + 4] += np.eye(2) * DT * 2
    for r in range(3):
        a = np.zeros(W * N)
        a[(N - 1) * W + U + r] = 1.0 / sc[14 if r < 2 else 15]
        H += np.outer(a, a) / mu_al
    dz_dense = np.linalg.solve(H + rho * np.eye(len(z)), -g)
    assert np.linalg.norm(dz - dz_dense) <= 1e-6 * np.linalg.norm(dz_dense)


def _solve(orc, modes, knots, goal, x0, params):
    m = np.zeros((1, 6), np.int32)
    k = np.zeros((1, 6), np.int32)
    m[0, :len(modes)], k[0, :len(knots)] = modes, knots
    return F.evaluate(np.array([x0]), np.array([goal]), np.array([0.4]), np.array([len(modes)]), m, k, params)


@pytest.mark.parametrize("j", range(4))
def test_goal_at_start_costs_nothing(orc, j):
    """Goal = start and free motion only: zero force and zero velocity satisfy every row, so
    the optimum is J = 0 with the pusher where it started."""
    x0 = np.array([0.0, 0.0, 0.0, *(0.08 * NORMAL[j])])
    r = _solve(orc, [F.free(j)], [8], (0.0, 0.0, 0.0), x0, orc.Params(**TIGHT))
    assert r["feasible"][0] == 1 and r["cost"][0] <= 1e-12
    assert np.allclose(r["traj"][0, 8, 3:5], x0[3:], atol=1e-7)


@pytest.mark.parametrize("d,N1,N2", [(0.05, 6, 10), (0.12, 10, 12), (0.02, 4, 6)])
def test_free_approach_then_straight_push_closed_form(orc, d, N1, N2):
    """Pusher 3 cm in front of face 2 (normal -x), goal (d, 0, 0), order [free in front of
    face 2, stick on face 2]: the free segment brings the pusher to the face centre with a
    constant velocity (least sum dt |v|^2 for a 3 cm move in N1 steps: 0.03^2 / (N1 dt)),
    the slider does not move; then a push through the face centre moves the slider d with
    a constant force (d^2 / (N2 dt), the fixed-step straight push).  J* is the sum."""
    x0 = np.array([0.0, 0.0, 0.0, -0.08, 0.0])
    Jstar = 0.03 ** 2 / (N1 * DT) + d ** 2 / (N2 * DT)
    r = _solve(orc, [F.free(2), F.contact(2, 0)], [N1, N2], (d, 0.0, 0.0), x0, orc.Params(**TIGHT))
    assert r["feasible"][0] == 1 and r["stats"][0, 3] == 1
    assert abs(r["cost"][0] - Jstar) <= 1e-7 * Jstar, (r["cost"][0], Jstar)
    T = r["traj"][0]
    assert np.allclose(T[N1, 3:5], [-HALF, 0.0], atol=1e-6)          # at the face centre
    assert np.allclose(T[:N1 + 1, :3], 0.0, atol=1e-7)                # slider still
    assert np.allclose(T[:N1, 7], 0.03 / (N1 * DT), rtol=1e-5)        # constant approach speed
    r2 = _solve(orc, [F.free(2), F.contact(2, 0)], [N1, N2], (d, 0.0, 0.0), x0, orc.Params())
    assert r2["feasible"][0] == 1 and abs(r2["cost"][0] - Jstar) <= 1e-3 * Jstar


def test_contact_first_needs_the_pusher_on_the_face(orc):
    """The start knot of a contact segment must lie on its face: from 3 cm in front of the
    face a contact-first order cannot be feasible, from the face centre it is."""
    goal = (0.0, 0.05, 0.0)
    far = _solve(orc, [F.contact(3, 0)], [10], goal, np.array([0, 0, 0, 0, -0.08]), orc.Params())
    on = _solve(orc, [F.contact(3, 0)], [10], goal, np.array([0, 0, 0, 0, -0.05]), orc.Params())
    assert far["feasible"][0] == 0 and far["viol"][0] >= 0.029
    assert on["feasible"][0] == 1


# ---------------------------------------------------------------------------------------
# The language, by brute force from an independent transcription of its rules.
# ---------------------------------------------------------------------------------------
def _is_contact(m):
    return m < 12


def _face(m):
    return m // 3 if m < 12 else m - 12


def _step_ok(a, b):
    if a == b:
        return False
    if _is_contact(a) or _is_contact(b):
        return _face(a) == _face(b)          # same face: slip change, leave to or enter from its region
    return (_face(a) - _face(b)) % 4 in (1, 3)


def _admissible(order):
    return all(_step_ok(a, b) for a, b in zip(order, order[1:]))


def _all_admissible(kmax):
    out = []
    for K in range(1, kmax + 1):
        out += [o for o in itertools.product(range(16), repeat=K) if _admissible(o)]
    return out


def test_language_by_brute_force(orc):
    orders = _all_admissible(4)
    got = [F.key_modes(int(k)) for k in F.seed(4)]
    assert [list(o) for o in orders] == got          # same set, in key order
    for o in itertools.product(range(16), repeat=3):
        assert F.admissible(o) == _admissible(o)
    counts = [len(F.seed(K)) for K in range(1, 9)]          # orders of 1..K segments
    # the same counts by the transfer matrix of the rules
    A = np.array([[1 if _step_ok(a, b) else 0 for b in range(16)] for a in range(16)], dtype=object)
    v, tot = np.ones(16, dtype=object), []
    for _ in range(8):
        tot.append(int(v.sum()))
        v = v.dot(A)
    cum = np.cumsum(tot)
    assert list(cum) == counts
    # the seed of eight segments: strictly increasing keys, each admissible by the rules
    # above, as many as the transfer matrix counts -- so it is the whole language, in key order
    s8 = [int(k) for k in F.seed(8)]
    assert all(a < b for a, b in zip(s8, s8[1:]))
    assert all(_admissible(tuple(F.key_modes(k))) for k in s8[::7] + s8[-200:])
    print(f"free-motion language: {cum[5]} orders of <= 6 segments, {cum[7]} of <= 8 "
          f"(the paper's box benchmark: 601 / 6,297 -- parity unpinned: its transition rules are not stated)")


def test_keys_order_by_length_then_ids():
    """Keys of up to eight segments (4 bits per id) round-trip, and comparing keys compares
    the segment count first, then the ids lexicographically."""
    rng = np.random.default_rng(11)
    orders = [tuple(int(x) for x in rng.integers(0, 16, rng.integers(1, 9))) for _ in range(3000)]
    orders += [(15,) * 8, (0,), (15,), (0, 0), (15,) * 7]
    for o in orders:
        assert tuple(F.key_modes(F.key_make(o))) == o
    by_key = sorted(orders, key=F.key_make)
    assert by_key == sorted(orders, key=lambda o: (len(o), o))


def _neigh1(order, kcap):
    K = len(order)
    out = []
    for i in range(K):
        for m in range(16):
            if m != order[i]:
                out.append(order[:i] + (m,) + order[i + 1:])
    if K > 1:
        for i in range(K):
            out.append(order[:i] + order[i + 1:])
    if K < kcap:
        for i in range(K + 1):
            for m in range(16):
                out.append(order[:i] + (m,) + order[i:])
    return out


def _neigh(order, kcap, r):
    """first occurrence in list order, the order itself excluded, admissible only; r = 2 only
    through admissible one-edit intermediates (Sec. III-B)"""
    seen, out = {order}, []
    l1 = _neigh1(order, kcap)
    for o in l1:
        if o not in seen:
            seen.add(o)
            if _admissible(o):
                out.append(o)
    if r >= 2:
        for o in l1:
            if not _admissible(o):
                continue
            for o2 in _neigh1(o, kcap):
                if o2 not in seen:
                    seen.add(o2)
                    if _admissible(o2):
                        out.append(o2)
    return out


@pytest.mark.parametrize("order,r,kcap", [((15,), 1, 6), ((15, 9), 2, 6), ((12, 0, 1, 12), 2, 6), ((15, 9, 15, 12), 1, 6),
                                          ((13, 12, 15, 9, 10), 2, 6), ((14, 6, 14, 15, 9, 15, 12), 2, 8),
                                          ((14, 6, 7, 14, 13, 4, 3, 13), 2, 8), ((12, 13), 2, 8)])
def test_neighbourhoods_by_brute_force(orc, order, r, kcap):
    want = [F.key_make(o) for o in _neigh(order, kcap, r)]
    got = [int(k) for k in F.neighbours(F.key_make(order), kcap, r)]
    assert got == want


@pytest.mark.parametrize("W,room,r", [(4, 50, 1), (16, 400, 2), (1000, 10 ** 6, 1)])
def test_expand_next_matches_a_set_based_twin(orc, W, room, r):
    """One batch step of Alg. 1: rank by (merit, key), NaN as +inf; the first `room` unseen
    admissible neighbours of the W best, in traversal order."""
    rng = np.random.default_rng(W + room)
    seedk = [int(k) for k in F.seed(2)]
    keys = [seedk[i] for i in rng.choice(len(seedk), 40, replace=False)]
    merit = rng.uniform(0, 1, 40)
    merit[rng.choice(40, 5, replace=False)] = np.nan
    merit[3] = merit[4]                                   # a tie, decided by the key
    got = [int(k) for k in F.expand_next(np.array(keys, np.uint64), merit, 8, r, W, room)]
    rank = sorted(range(40), key=lambda i: (np.inf if np.isnan(merit[i]) else merit[i], keys[i]))
    seen, want = set(keys), []
    for i in rank[:W]:
        for o in _neigh(tuple(F.key_modes(keys[i])), 8, r):
            k = F.key_make(o)
            if len(want) < room and k not in seen:
                seen.add(k)
                want.append(k)
    assert got == want


def test_free_unranking_lists_the_language_in_key_order(orc):
    """The sampler's unranking (the t-th admissible order of K segments) enumerates exactly
    the seed's orders of K segments, in key order: all of them for K <= 5, a strided sample
    and both ends for K = 6..8; free-motion draws have uniform segment counts."""
    from oracle import sample as S
    counts = S.free_counts()
    s8 = [int(k) for k in F.seed(8)]
    by_len = {K: [k for k in s8 if k >> 60 == K] for K in range(1, 9)}
    for K in range(1, 9):
        ref = by_len[K]
        ts = range(len(ref)) if K <= 5 else sorted(set(list(range(0, len(ref), 997)) + [0, len(ref) - 1]))
        for t in ts:
            assert F.key_make(S.free_unrank(K, t, counts)) == ref[t], (K, t)
    d = S.free_draws(7, 0, 4000, 8)
    assert all(F.admissible(m) for m in d)
    hist = np.bincount([len(m) for m in d], minlength=9)[1:]
    assert hist.min() > 400 and hist.max() < 600
