"""Pins for the FP64 oracle: each test checks it against something other than
itself (closed forms, independent optimisers, LP, brute force, theorems of
the paper), chosen so that a dropped term, a wrong sign or index or a
transposed operand fails at least one of them."""
import numpy as np
import pytest
from scipy import optimize

from oracle import uot_oracle as O

RNG = np.random.default_rng(1234)


def _rand_problem(rng, N, M, d=2, mass_q=1.3):
    x = rng.uniform(0, 1, (N, d))
    y = rng.uniform(0, 1, (M, d))
    p = rng.uniform(0.3, 1.5, N)
    q = rng.uniform(0.3, 1.5, M)
    q *= mass_q * p.sum() / q.sum() * (M / N) / (M / N)
    dx = rng.uniform(0.5, 1.5, N)
    dx /= dx.sum()
    dy = rng.uniform(0.5, 1.5, M)
    dy /= dy.sum()
    return x, y, p, q, dx, dy


# ---------------------------------------------------------------------------
# P11: every Table proximalexplicit row against brute-force minimisation of
# F(t) + eps KLbar(t | e^{-u/eps} s) over t >= 0 (definition of prox^KL).
# ---------------------------------------------------------------------------
def _kl_bar(t, z):
    if t == 0:
        return z
    return t * np.log(t / z) - t + z


def _brute_prox(F, s_eff, p, eps):
    """argmin_t f(t) + eps KLbar(t|s_eff), searched in log t (ternary search on
    a convex function of t, restricted to the domain of f)."""
    if F.kind == "eq":
        return p
    lo, hi = np.log(s_eff) - 80, np.log(s_eff) + 80
    if F.kind == "rg":
        lo = max(lo, np.log(F.alpha * p)) if F.alpha > 0 else lo
        hi = min(hi, np.log(F.beta * p)) if np.isfinite(F.beta) else hi

    def f(t):
        if F.kind == "kl":
            fv = F.lam * _kl_bar(t, p)
        elif F.kind == "tv":
            fv = F.lam * abs(t - p)
        else:
            fv = 0.0
        return fv + eps * _kl_bar(t, s_eff)

    # the objective is convex in t; golden-section in t on [e^lo, e^hi] split at
    # the kink points to keep it unimodal on each piece
    pts = sorted({np.exp(lo), np.exp(hi)} | ({p} if np.exp(lo) < p < np.exp(hi) else set()))
    best_t, best_v = None, np.inf
    for a, b in zip(pts[:-1], pts[1:]):
        r = optimize.minimize_scalar(lambda lt: f(np.exp(lt)), bounds=(np.log(a), np.log(b)),
                                     method="bounded", options=dict(xatol=1e-13, maxiter=2000))
        for cand in (np.exp(r.x), a, b):
            v = f(cand)
            if v < best_v:
                best_t, best_v = cand, v
    return best_t


@pytest.mark.parametrize("F", [O.EQ, O.KL(0.3), O.KL(2.0), O.TV(0.05), O.TV(0.4),
                               O.RG(0.7, 1.2), O.RG(0.0, 5.0), O.RG(0.5, np.inf)])
def test_proxdiv_rows_match_bruteforce_prox(F):
    rng = np.random.default_rng(7)
    for _ in range(25):
        s = np.exp(rng.uniform(-3, 3))
        p = np.exp(rng.uniform(-3, 3))
        eps = np.exp(rng.uniform(np.log(0.05), np.log(1.0)))
        ubar = rng.uniform(-0.2, 0.2)
        s_eff = np.exp(-ubar / eps) * s
        t = _brute_prox(F, s_eff, p, eps)
        got = O.proxdiv_log(F, np.array([np.log(p)]), np.array([np.log(s)]), ubar, eps)[0]
        assert got == pytest.approx(np.log(t / s), abs=2e-6), (F, s, p, eps, ubar)
        # the scaling-domain table gives the same number
        sc = O.proxdiv_scaling(F, np.array([p]), np.array([s]), ubar, eps)[0]
        assert np.log(sc) == pytest.approx(got, abs=1e-10)


def test_proxdiv_zero_density_cases():
    """Prop. UOTprox case p(x)=0, s(x)>0: eps log(s*/s) + phi'_inf = 0, i.e.
    s* = s e^{-phi'_inf/eps}: a = 0 for KL / = / RG (phi'_inf = inf) and
    a = e^{-lam/eps} for lam TV (phi'_inf = lam)."""
    lp = np.array([-np.inf])
    ls = np.array([0.3])
    eps = 0.1
    for F in (O.EQ, O.KL(1.0), O.RG(0.5, 2.0)):
        assert O.proxdiv_log(F, lp, ls, 0.0, eps)[0] == -np.inf
    assert O.proxdiv_log(O.TV(0.2), lp, ls, 0.0, eps)[0] == pytest.approx(-0.2 / eps)


# ---------------------------------------------------------------------------
# P1: one point (N = M = 1, dx = dy = 1), KL/KL: stationarity of
# lam1 KL(r|p) + lam2 KL(r|q) + eps KL(r|e^{-c/eps}) gives a closed form.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam1,lam2,p,q,c,eps", [
    (1.0, 1.0, 1.0, 1.5, 0.3, 0.05),
    (0.1, 2.0, 0.2, 3.0, 1.0, 0.2),
    (5.0, 0.5, 2.0, 0.7, 0.0, 0.01),
])
def test_one_point_closed_form(lam1, lam2, p, q, c, eps):
    r = np.exp((lam1 * np.log(p) + lam2 * np.log(q) - c) / (lam1 + lam2 + eps))
    u_star = -lam1 * np.log(r / p)
    v_star = -lam2 * np.log(r / q)
    P_star = lam1 * p + lam2 * q + eps * np.exp(-c / eps) - (lam1 + lam2 + eps) * r
    g = O.DenseGeom(np.array([[c]]))
    one = np.zeros(1)
    out = O.solve(g, np.log([p]), np.log([q]), one, one, O.KL(lam1), O.KL(lam2), eps, tol=1e-15, max_iter=200000)
    assert out["u"][0] == pytest.approx(u_star, rel=1e-10, abs=1e-12)
    assert out["v"][0] == pytest.approx(v_star, rel=1e-10, abs=1e-12)
    ob = O.objective(g, [p], [q], [1.0], [1.0], O.KL(lam1), O.KL(lam2), eps, out["u"], out["v"])
    assert ob["primal"] == pytest.approx(P_star, rel=1e-9)
    assert ob["dual"] == pytest.approx(P_star, rel=1e-9)
    assert ob["transport_cost"] == pytest.approx(c * r, rel=1e-9, abs=1e-300)


# ---------------------------------------------------------------------------
# P2: rank-one kernel (all y_j at one point): C_ij = f(x_i), K_ij = phi_i.
# a_i = (p_i/(phi_i S_b))^z1, b_j = (q_j/S_a)^z2 with S_a = sum dx phi a and
# S_b = sum dy b: a 2x2 linear system in (log S_a, log S_b).
# ---------------------------------------------------------------------------
def test_rank_one_kernel_closed_form():
    rng = np.random.default_rng(3)
    N, M, eps, l1, l2 = 37, 23, 0.05, 0.7, 1.9
    x = rng.uniform(0, 1, (N, 2))
    y = np.tile(rng.uniform(0, 1, (1, 2)), (M, 1))
    p = rng.uniform(0.2, 2, N)
    q = rng.uniform(0.2, 2, M)
    dx = np.full(N, 1.0 / N)
    dy = rng.uniform(0.5, 1.5, M)
    dy /= dy.sum()
    z1, z2 = l1 / (l1 + eps), l2 / (l2 + eps)
    f = np.sum((x - y[0]) ** 2, axis=1)
    logphi = -f / eps
    lA = np.log(np.sum(dx * np.exp((1 - z1) * logphi + z1 * np.log(p))))
    lB = np.log(np.sum(dy * q ** z2))
    lSa = (lA - z1 * lB) / (1 - z1 * z2)
    lSb = lB - z2 * lSa
    u_star = eps * z1 * (np.log(p) - logphi - lSb)
    v_star = eps * z2 * (np.log(q) - lSa)
    g = O.PointsGeom(x, y)
    out = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(l1), O.KL(l2), eps, tol=1e-15, max_iter=100000)
    np.testing.assert_allclose(out["u"], u_star, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["v"], v_star, rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------------------
# P3: cost shift C + c0 (KL/KL): a -> t_a a, b -> t_b b with
# u += c0 z1 (1-z2)/(1-z1 z2), v += c0 z2 (1-z1)/(1-z1 z2),
# plan scaled by exp(-c0 (1-z1)(1-z2) / (eps (1-z1 z2))).
# ---------------------------------------------------------------------------
def test_cost_shift():
    rng = np.random.default_rng(5)
    x, y, p, q, dx, dy = _rand_problem(rng, 19, 27)
    eps, l1, l2, c0 = 0.08, 0.5, 1.5, 0.37
    C = O.sq_dist(x, y)
    args = (np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(l1), O.KL(l2), eps)
    a = O.solve(O.DenseGeom(C), *args, tol=1e-15, max_iter=100000)
    b = O.solve(O.DenseGeom(C + c0), *args, tol=1e-15, max_iter=100000)
    z1, z2 = l1 / (l1 + eps), l2 / (l2 + eps)
    np.testing.assert_allclose(b["u"] - a["u"], c0 * z1 * (1 - z2) / (1 - z1 * z2), rtol=1e-9)
    np.testing.assert_allclose(b["v"] - a["v"], c0 * z2 * (1 - z1) / (1 - z1 * z2), rtol=1e-9)
    oa = O.objective(O.DenseGeom(C), p, q, dx, dy, O.KL(l1), O.KL(l2), eps, a["u"], a["v"])
    ob = O.objective(O.DenseGeom(C + c0), p, q, dx, dy, O.KL(l1), O.KL(l2), eps, b["u"], b["v"])
    ratio = np.exp(-c0 * (1 - z1) * (1 - z2) / (eps * (1 - z1 * z2)))
    assert ob["mass"] / oa["mass"] == pytest.approx(ratio, rel=1e-9)


# ---------------------------------------------------------------------------
# P4: lam -> inf turns the KL row into the = row (Table proximalexplicit
# remark); the = / = iteration is Sinkhorn and matches both marginals.
# ---------------------------------------------------------------------------
def test_large_lambda_is_balanced_sinkhorn():
    rng = np.random.default_rng(11)
    x, y, p, q, dx, dy = _rand_problem(rng, 15, 21)
    q *= np.sum(p * dx) / np.sum(q * dy)   # equal masses
    eps = 0.05
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    eq = O.solve(g, *lg, O.EQ, O.EQ, eps, tol=1e-14, max_iter=200000)
    kl = O.solve(g, *lg, O.KL(1e6), O.KL(1e6), eps, tol=1e-14, max_iter=200000)
    o = O.objective(g, p, q, dx, dy, O.EQ, O.EQ, eps, eq["u"], eq["v"])
    np.testing.assert_allclose(o["pi1"], p, rtol=1e-11)
    np.testing.assert_allclose(o["pi2"], q, rtol=1e-11)
    # both solutions: gauge-fix (u + c, v - c) by mean(u) = mean(v)
    def gauge(s):
        c = (np.mean(s["v"]) - np.mean(s["u"])) / 2
        return s["u"] + c, s["v"] - c
    ue, ve = gauge(eq)
    uk, vk = gauge(kl)
    assert np.max(np.abs(ue - uk)) < 1e-5
    assert np.max(np.abs(ve - vk)) < 1e-5


def test_balanced_plan_matches_lp_as_eps_vanishes():
    """Prop. converg_regul: the regularised optimum tends to an LP optimum."""
    rng = np.random.default_rng(2)
    x, y, p, q, dx, dy = _rand_problem(rng, 6, 5)
    q *= np.sum(p * dx) / np.sum(q * dy)
    C = O.sq_dist(x, y)
    N, M = C.shape
    # LP on the plan density R >= 0 w.r.t. dx dy: R dy = p, R^T dx = q
    A_eq = np.zeros((N + M, N * M))
    for i in range(N):
        A_eq[i, i * M:(i + 1) * M] = dy
    for j in range(M):
        A_eq[N + j, j::M] = dx
    w = (dx[:, None] * dy[None, :]).reshape(-1)
    lp = optimize.linprog(C.reshape(-1) * w, A_eq=A_eq, b_eq=np.r_[p, q], bounds=(0, None), method="highs")
    g = O.DenseGeom(C)
    for eps in (1e-2, 1e-3):
        s = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.EQ, O.EQ, eps, tol=1e-13, max_iter=500000)
        o = O.objective(g, p, q, dx, dy, O.EQ, O.EQ, eps, s["u"], s["v"])
        # entropic plan cost exceeds the LP optimum by at most eps * (entropy range)
        gapc = o["transport_cost"] - lp.fun
        assert -1e-9 <= gapc <= eps * np.log(N * M) * 2 + 1e-9


# ---------------------------------------------------------------------------
# P6 / P7: primal-dual relations (Thm. duality) and duality invariants
# ---------------------------------------------------------------------------
def test_fixed_point_primal_dual_relations():
    rng = np.random.default_rng(9)
    x, y, p, q, dx, dy = _rand_problem(rng, 30, 25)
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    eps = 0.02
    # KL: -u in dF1(pi1) = lam log(pi1/p)  =>  pi1 = p e^{-u/lam}
    s = O.solve(g, *lg, O.KL(0.4), O.KL(0.9), eps, tol=1e-14, max_iter=100000)
    o = O.objective(g, p, q, dx, dy, O.KL(0.4), O.KL(0.9), eps, s["u"], s["v"])
    np.testing.assert_allclose(o["pi1"], p * np.exp(-s["u"] / 0.4), rtol=1e-10)
    np.testing.assert_allclose(o["pi2"], q * np.exp(-s["v"] / 0.9), rtol=1e-10)
    assert abs(o["gap"]) < 1e-10 * abs(o["primal"])
    # TV: -u in lam dphi_TV(pi1/p): |u| <= lam, and pi1 = p where |u| < lam
    s = O.solve(g, *lg, O.TV(0.1), O.TV(0.1), eps, tol=1e-14, max_iter=100000)
    o = O.objective(g, p, q, dx, dy, O.TV(0.1), O.TV(0.1), eps, s["u"], s["v"])
    assert np.all(np.abs(s["u"]) <= 0.1 + 1e-15)
    inner = np.abs(s["u"]) < 0.1 - 1e-9
    np.testing.assert_allclose(o["pi1"][inner], p[inner], rtol=1e-9)
    assert np.all(o["pi1"][s["u"] >= 0.1 - 1e-9] <= p[s["u"] >= 0.1 - 1e-9] * (1 + 1e-9))
    assert abs(o["gap"]) < 1e-9
    # RG: alpha p <= pi1 <= beta p
    s = O.solve(g, *lg, O.RG(0.7, 1.2), O.RG(0.7, 1.2), eps, tol=1e-14, max_iter=100000)
    o = O.objective(g, p, q, dx, dy, O.RG(0.7, 1.2), O.RG(0.7, 1.2), eps, s["u"], s["v"])
    assert np.all(o["pi1"] >= 0.7 * p * (1 - 1e-9)) and np.all(o["pi1"] <= 1.2 * p * (1 + 1e-9))
    assert np.all(o["pi2"] >= 0.7 * q * (1 - 1e-9)) and np.all(o["pi2"] <= 1.2 * q * (1 + 1e-9))


@pytest.mark.parametrize("F", [O.KL(0.3), O.TV(0.08)])
def test_dual_monotone_and_gap_nonnegative(F):
    """Alternating maximisation (eq. alternating_max): the dual never
    decreases over half-steps; the Fenchel-Young gap is >= 0 and -> 0."""
    rng = np.random.default_rng(4)
    x, y, p, q, dx, dy = _rand_problem(rng, 20, 17)
    g = O.PointsGeom(x, y)
    eps = 0.03
    lp_, lq, ldx, ldy = np.log(p), np.log(q), np.log(dx), np.log(dy)
    u = np.zeros(20)
    v = np.zeros(17)
    last = -np.inf
    gaps = []
    for it in range(300):
        _, u, _ = O.half_step_x(g, lp_, ldx, ldy, F, eps, u, v)
        d1 = O.dual_value(g, p, q, dx, dy, F, F, eps, u, v)
        _, v = O.half_step_y(g, lq, ldx, F, eps, u)
        o = O.objective(g, p, q, dx, dy, F, F, eps, u, v)
        assert d1 >= last - 1e-12 * max(1, abs(last))
        assert o["dual"] >= d1 - 1e-12 * max(1, abs(d1))
        last = o["dual"]
        assert o["gap"] >= -1e-12
        gaps.append(o["gap"])
    assert gaps[-1] < 1e-9


def test_thompson_contraction():
    """Thm. convergenceKL: d(a^{l+1}, a^l) <= z1 z2 d(a^l, a^{l-1}) in the
    Thompson metric, i.e. sup|u^{l+1} - u^l| <= z1 z2 sup|u^l - u^{l-1}|."""
    rng = np.random.default_rng(8)
    x, y, p, q, dx, dy = _rand_problem(rng, 25, 30)
    g = O.PointsGeom(x, y)
    eps, l1, l2 = 0.05, 0.3, 0.6
    s = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(l1), O.KL(l2), eps,
                tol=0.0, max_iter=60, record=True)
    z = l1 / (l1 + eps) * l2 / (l2 + eps)
    us = [h[0] for h in s["hist"]]
    d = [np.max(np.abs(us[k + 1] - us[k])) for k in range(len(us) - 1)]
    for k in range(len(d) - 1):
        if d[k] > 1e-12:
            assert d[k + 1] <= z * d[k] * (1 + 1e-9) + 1e-14


# ---------------------------------------------------------------------------
# P9: tiny problems, the regularised dual (D_eps) maximised by a generic
# optimiser, independent of the scaling iteration.
# ---------------------------------------------------------------------------
def _dual_kl(z, K, p, q, dx, dy, l1, l2, eps):
    N = len(p)
    u, v = z[:N], z[N:]
    E = np.exp((u[:, None] + v[None, :]) / eps) * K * dx[:, None] * dy[None, :]
    val = -np.sum(dx * l1 * p * (np.exp(-u / l1) - 1)) - np.sum(dy * l2 * q * (np.exp(-v / l2) - 1)) - eps * np.sum(E - K * dx[:, None] * dy[None, :])
    gu = dx * p * np.exp(-u / l1) - E.sum(1)
    gv = dy * q * np.exp(-v / l2) - E.sum(0)
    H = np.zeros((len(z), len(z)))
    H[:N, :N] = np.diag(-dx * p * np.exp(-u / l1) / l1 - E.sum(1) / eps)
    H[N:, N:] = np.diag(-dy * q * np.exp(-v / l2) / l2 - E.sum(0) / eps)
    H[:N, N:] = -E / eps
    H[N:, :N] = -E.T / eps
    return -val, -np.r_[gu, gv], -H


def test_kl_dual_newton_tiny():
    rng = np.random.default_rng(21)
    for N, M in ((3, 4), (6, 5), (8, 8)):
        x, y, p, q, dx, dy = _rand_problem(rng, N, M)
        eps, l1, l2 = 0.04, 0.6, 1.7
        C = O.sq_dist(x, y)
        K = np.exp(-C / eps)
        r = optimize.minimize(lambda z: _dual_kl(z, K, p, q, dx, dy, l1, l2, eps)[:2], np.zeros(N + M),
                              jac=True, hess=lambda z: _dual_kl(z, K, p, q, dx, dy, l1, l2, eps)[2],
                              method="trust-exact", options=dict(gtol=1e-14))
        s = O.solve(O.DenseGeom(C), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(l1), O.KL(l2), eps,
                    tol=1e-15, max_iter=200000)
        np.testing.assert_allclose(s["u"], r.x[:N], atol=1e-10)
        np.testing.assert_allclose(s["v"], r.x[N:], atol=1e-10)
        o = O.objective(O.DenseGeom(C), p, q, dx, dy, O.KL(l1), O.KL(l2), eps, s["u"], s["v"])
        assert o["dual"] == pytest.approx(-r.fun, rel=1e-11)


def _dual_box(F1, F2, C, p, q, dx, dy, eps):
    """TV: max sum dx p u + sum dy q v - eps sum dx dy (e^{(u+v)/eps} - 1) K over
    the box |u|, |v| <= lam (the finite part of -F*(-u)).  RG: split
    u = u+ - u-, the concave piecewise-linear term is alpha u+ - beta u-."""
    N, M = C.shape
    K = np.exp(-C / eps)
    W = dx[:, None] * dy[None, :]
    if F1.kind == "tv":
        def f(z):
            u, v = z[:N], z[N:]
            E = np.exp((u[:, None] + v[None, :]) / eps) * K * W
            val = np.sum(dx * p * u) + np.sum(dy * q * v) - eps * np.sum(E - K * W)
            return -val, -np.r_[dx * p - E.sum(1), dy * q - E.sum(0)]
        bounds = [(-F1.lam, F1.lam)] * N + [(-F2.lam, F2.lam)] * M
        r = optimize.minimize(f, np.zeros(N + M), jac=True, bounds=bounds, method="L-BFGS-B",
                              options=dict(ftol=1e-16, gtol=1e-13, maxiter=50000, maxcor=50))
        return r.x[:N], r.x[N:], -r.fun
    # RG
    a, b = F1.alpha, F1.beta

    def f(z):
        up, um, vp, vm = z[:N], z[N:2 * N], z[2 * N:2 * N + M], z[2 * N + M:]
        u, v = up - um, vp - vm
        E = np.exp((u[:, None] + v[None, :]) / eps) * K * W
        val = np.sum(dx * p * (a * up - b * um)) + np.sum(dy * q * (a * vp - b * vm)) - eps * np.sum(E - K * W)
        gu = -E.sum(1)
        gv = -E.sum(0)
        g = np.r_[dx * p * a + gu, -dx * p * b - gu, dy * q * a + gv, -dy * q * b - gv]
        return -val, -g
    r = optimize.minimize(f, np.full(2 * (N + M), 0.0), jac=True, bounds=[(0, None)] * (2 * (N + M)),
                          method="L-BFGS-B", options=dict(ftol=1e-16, gtol=1e-13, maxiter=50000, maxcor=50))
    z = r.x
    return z[:N] - z[N:2 * N], z[2 * N:2 * N + M] - z[2 * N + M:], -r.fun


@pytest.mark.parametrize("F", [O.TV(0.05), O.TV(0.3), O.RG(0.7, 1.2)])
def test_tv_rg_dual_box_tiny(F):
    rng = np.random.default_rng(31)
    x, y, p, q, dx, dy = _rand_problem(rng, 5, 6)
    eps = 0.05
    C = O.sq_dist(x, y)
    u_ref, v_ref, dval = _dual_box(F, F, C, p, q, dx, dy, eps)
    s = O.solve(O.DenseGeom(C), np.log(p), np.log(q), np.log(dx), np.log(dy), F, F, eps, tol=1e-15, max_iter=500000)
    o = O.objective(O.DenseGeom(C), p, q, dx, dy, F, F, eps, s["u"], s["v"])
    assert o["dual"] == pytest.approx(dval, rel=1e-8, abs=1e-10)
    np.testing.assert_allclose(s["u"], u_ref, atol=2e-5)
    np.testing.assert_allclose(s["v"], v_ref, atol=2e-5)
    if F.kind == "tv":
        # strong duality: the primal at the plan equals the dual maximum
        assert o["primal"] == pytest.approx(dval, rel=1e-8, abs=1e-10)


def test_tv_lp_limit():
    """Prop. converg_regul with TV marginals: as eps -> 0 the regularised
    plan's J = <C,R> + F1 + F2 tends to the LP optimum (optimal partial
    transport with linear penalties)."""
    rng = np.random.default_rng(17)
    x, y, p, q, dx, dy = _rand_problem(rng, 6, 7)
    lam = 0.15
    C = O.sq_dist(x, y)
    N, M = C.shape
    W = (dx[:, None] * dy[None, :]).reshape(-1)
    # variables: R (N M), e1+ e1- (N), e2+ e2- (M):  R dy - p = e1+ - e1-
    nv = N * M + 2 * N + 2 * M
    c = np.r_[C.reshape(-1) * W, lam * dx, lam * dx, lam * dy, lam * dy]
    A = np.zeros((N + M, nv))
    for i in range(N):
        A[i, i * M:(i + 1) * M] = dy
        A[i, N * M + i] = -1
        A[i, N * M + N + i] = 1
    for j in range(M):
        A[N + j, j:N * M:M] = dx
        A[N + j, N * M + 2 * N + j] = -1
        A[N + j, N * M + 2 * N + M + j] = 1
    lp = optimize.linprog(c, A_eq=A, b_eq=np.r_[p, q], bounds=(0, None), method="highs")
    g = O.DenseGeom(C)
    prev = None
    for eps in (1e-2, 3e-3, 1e-3):
        s = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.TV(lam), O.TV(lam), eps, tol=1e-13, max_iter=2000000)
        o = O.objective(g, p, q, dx, dy, O.TV(lam), O.TV(lam), eps, s["u"], s["v"])
        J = o["transport_cost"] + O.F_value(O.TV(lam), o["pi1"], p, dx) + O.F_value(O.TV(lam), o["pi2"], q, dy)
        assert J >= lp.fun - 1e-9
        assert J - lp.fun <= 3 * eps * np.log(N * M) + 1e-9
        if prev is not None:
            assert J - lp.fun <= prev + 1e-12
        prev = J - lp.fun


# ---------------------------------------------------------------------------
# P12: Algorithm 1, Algorithm 2 (any absorption threshold) and the log-domain
# iteration give the same iterates where Algorithm 1 does not underflow.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("F", [O.EQ, O.KL(0.5), O.TV(0.1), O.RG(0.6, 1.4)])
def test_alg1_alg2_logdomain_same_iterates(F):
    rng = np.random.default_rng(13)
    x, y, p, q, dx, dy = _rand_problem(rng, 12, 9)
    eps = 0.05
    C = O.sq_dist(x, y)
    n = 40
    s = O.solve(O.DenseGeom(C), np.log(p), np.log(q), np.log(dx), np.log(dy), F, F, eps, tol=0.0,
                max_iter=n, record=True)
    a1 = O.scaling_algo(C, p, q, dx, dy, F, F, eps, n)
    for tau in (0.0, 0.5, 3.0, 1e9):
        a2 = O.scaling_algo2(C, p, q, dx, dy, F, F, eps, n, tau)
        for k in range(n):
            np.testing.assert_allclose(a2[k][0], s["hist"][k][0], rtol=1e-9, atol=1e-11)
            np.testing.assert_allclose(a2[k][1], s["hist"][k][1], rtol=1e-9, atol=1e-11)
    for k in range(n):
        np.testing.assert_allclose(a1[k][0], s["hist"][k][0], rtol=1e-9, atol=1e-11)
        np.testing.assert_allclose(a1[k][1], s["hist"][k][1], rtol=1e-9, atol=1e-11)


def test_eps_scaling_alg2_matches_logdomain():
    """The eps-scaling heuristic (absorb, divide eps, rebuild K~) gives the same
    potentials in Algorithm 2 and in the log-domain iteration."""
    rng = np.random.default_rng(14)
    x, y, p, q, dx, dy = _rand_problem(rng, 10, 8)
    C = O.sq_dist(x, y)
    F = O.KL(1.0)
    eps, eps0 = 5e-3, 1.0
    n = 3 * 10 + 15
    s = O.solve(O.DenseGeom(C), np.log(p), np.log(q), np.log(dx), np.log(dy), F, F, eps, tol=0.0, max_iter=n,
                eps0=eps0, n_stages=10, iters_per_stage=3, record=True)
    a2 = O.scaling_algo2(C, p, q, dx, dy, F, F, eps, n, tau=10.0, eps0=eps0, n_stages=10, iters_per_stage=3)
    for k in range(n):
        np.testing.assert_allclose(a2[k][0], s["hist"][k][0], rtol=1e-8, atol=1e-11)
        np.testing.assert_allclose(a2[k][1], s["hist"][k][1], rtol=1e-8, atol=1e-11)


# ---------------------------------------------------------------------------
# P13: symmetry and invariance
# ---------------------------------------------------------------------------
def test_swap_and_rigid_motion():
    rng = np.random.default_rng(23)
    x, y, p, q, dx, dy = _rand_problem(rng, 14, 11, d=3)
    eps = 0.04
    F1, F2 = O.KL(0.4), O.TV(0.2)
    a = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), F1, F2, eps, tol=1e-15, max_iter=200000)
    b = O.solve(O.PointsGeom(y, x), np.log(q), np.log(p), np.log(dy), np.log(dx), F2, F1, eps, tol=1e-15, max_iter=200000)
    np.testing.assert_allclose(a["u"], b["v"], atol=1e-9)
    np.testing.assert_allclose(a["v"], b["u"], atol=1e-9)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    t = rng.standard_normal(3)
    c = O.solve(O.PointsGeom(x @ Q.T + t, y @ Q.T + t), np.log(p), np.log(q), np.log(dx), np.log(dy), F1, F2, eps,
                tol=1e-15, max_iter=200000)
    np.testing.assert_allclose(a["u"], c["u"], atol=1e-9)
    np.testing.assert_allclose(a["v"], c["v"], atol=1e-9)


# ---------------------------------------------------------------------------
# separable grid passes == the dense kernel (Sec. 4.4 separable kernel)
# ---------------------------------------------------------------------------
def test_separable_grid_equals_dense():
    rng = np.random.default_rng(29)
    for shape in ((7,), (6, 5), (4, 3, 5)):
        h = tuple(1.0 / n for n in shape)
        G = O.GridGeom(shape, h)
        D = G.dense()
        w = rng.standard_normal(G.N)
        w[rng.integers(0, G.N, 2)] = -np.inf
        eps = 0.03
        np.testing.assert_allclose(G.lse_x(w, eps), D.lse_x(w, eps), rtol=1e-12, atol=1e-12)
        wx = rng.standard_normal(G.N)
        assert G.cost_moment_log(wx, w, eps) == pytest.approx(D.cost_moment_log(wx, w, eps), rel=1e-12)


def test_lse_all_neg_inf_row():
    a = np.array([[-np.inf, -np.inf], [0.0, -np.inf]])
    out = O.lse(a, axis=1)
    assert out[0] == -np.inf and out[1] == 0.0


def test_zero_density_potentials_are_neg_inf():
    """A9: p_i = 0 gives u_i = -inf under KL (no NaN anywhere)."""
    rng = np.random.default_rng(41)
    x, y, p, q, dx, dy = _rand_problem(rng, 10, 9)
    p[[2, 5]] = 0.0
    g = O.PointsGeom(x, y)
    s = O.solve(g, O.safe_log(p), np.log(q), np.log(dx), np.log(dy), O.KL(0.5), O.KL(0.5), 0.05, tol=1e-13, max_iter=100000)
    assert np.isneginf(s["u"][[2, 5]]).all()
    assert np.isfinite(np.delete(s["u"], [2, 5])).all() and np.isfinite(s["v"]).all()
    o = O.objective(g, p, q, dx, dy, O.KL(0.5), O.KL(0.5), 0.05, s["u"], s["v"])
    assert np.isfinite(o["primal"]) and abs(o["gap"]) < 1e-9


# ---------------------------------------------------------------------------
# P11 / P14: barycentre h of Table estimatebary against brute-force
# minimisation of eq. (prox_barycenter), and the special cases
# ---------------------------------------------------------------------------
def test_bary_h_matches_bruteforce():
    rng = np.random.default_rng(37)
    for _ in range(10):
        n = 4
        s = np.exp(rng.uniform(-2, 2, n))
        alpha = rng.uniform(0.2, 1.0, n)
        eps = rng.uniform(0.05, 0.5)
        lam = rng.uniform(0.1, 2.0)

        def obj(z):  # z = (log s~_1..n, log h)
            st, h = np.exp(z[:n]), np.exp(z[n])
            return sum(alpha[k] * (eps * _kl_bar(st[k], s[k]) + lam * _kl_bar(st[k], h)) for k in range(n))
        r = optimize.minimize(obj, np.r_[np.log(s), np.mean(np.log(s))], method="Nelder-Mead",
                              options=dict(xatol=1e-12, fatol=1e-15, maxiter=40000, maxfev=40000))
        r = optimize.minimize(obj, r.x, method="BFGS", options=dict(gtol=1e-12))
        logh = O.bary_logh(np.log(s)[:, None], alpha, eps, O.KL(lam))[0]
        assert logh == pytest.approx(r.x[n], abs=1e-5)
        # (i): min_h sum alpha_k KLbar(h | s_k) -> weighted geometric mean
        r = optimize.minimize_scalar(lambda lh: sum(alpha[k] * _kl_bar(np.exp(lh), s[k]) for k in range(n)),
                                     bounds=(-5, 5), method="bounded", options=dict(xatol=1e-12))
        assert O.bary_logh(np.log(s)[:, None], alpha, eps, O.EQ)[0] == pytest.approx(r.x, abs=1e-7)
        # lam -> inf: (ii) -> (i)
        big = O.bary_logh(np.log(s)[:, None], alpha, eps, O.KL(1e7))[0]
        assert big == pytest.approx(O.bary_logh(np.log(s)[:, None], alpha, eps, O.EQ)[0], abs=1e-5)


def test_barycenter_special_cases():
    G = O.GridGeom((12, 10), (1 / 12, 1 / 10))
    rng = np.random.default_rng(43)
    ldx = np.full(G.N, np.log(1 / G.N))
    eps = 0.01
    # n = 1: F2(s) = min_h lam KL(s|h) = 0, so b = 1 and v = 0 at every iteration
    p1 = rng.uniform(0.5, 1.5, (1, G.N))
    out = O.barycenter(G, np.log(p1), np.array([1.0]), ldx, ldx, O.KL(0.5), O.KL(0.5), eps, tol=1e-12, max_iter=3000)
    assert np.max(np.abs(out["v"])) < 1e-12
    # all p_k equal: v_k = 0 for all k
    p = np.tile(rng.uniform(0.5, 1.5, G.N), (3, 1))
    out = O.barycenter(G, np.log(p), np.array([0.2, 0.3, 0.5]), ldx, ldx, O.KL(0.5), O.KL(0.5), eps, tol=1e-12, max_iter=3000)
    assert np.max(np.abs(out["v"])) < 1e-12
    # the fixed point is the UOT solution with F2 = 0 (a free second marginal):
    # a = (p / K(dy))^z after one iteration, h = K^T(a dx)
    S = G.lse_x(ldx, eps)
    u1 = eps * 0.5 / (0.5 + eps) * (np.log(p[0]) - S)
    np.testing.assert_allclose(out["u"][0], u1, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(out["logh"], G.lse_y(u1 / eps + ldx, eps), rtol=1e-10, atol=1e-12)


def test_barycenter_fixed_point_optimality():
    """At the fixed point, (u_k, v_k) solve the multi-coupling dual: each
    coupling's X marginal is p_k e^{-u_k/lam} (KL relation) and h is the
    pointwise barycentre of the Y marginals s~_k (Prop. barycenter_general):
    s~_k = h^{z} s_k^{1-z} with z = lam/(lam+eps)."""
    G = O.GridGeom((10, 9), (1 / 10, 1 / 9))
    rng = np.random.default_rng(47)
    ldx = np.full(G.N, np.log(1 / G.N))
    eps, lam = 0.01, 0.5
    p = rng.uniform(0.3, 1.5, (3, G.N))
    alpha = np.array([0.2, 0.5, 0.3])
    out = O.barycenter(G, np.log(p), alpha, ldx, ldx, O.KL(lam), O.KL(lam), eps, tol=1e-14, max_iter=20000)
    for k in range(3):
        S = G.lse_x(out["v"][k] / eps + ldx, eps)
        np.testing.assert_allclose(np.exp(out["u"][k] / eps + S), p[k] * np.exp(-out["u"][k] / lam), rtol=1e-9)
    T = np.stack([G.lse_y(out["u"][k] / eps + ldx, eps) for k in range(3)])
    pi2 = np.exp(out["v"] / eps + T)
    # sum_k alpha_k (1 - s~_k / h) = 0 (KL case of the appendix derivation)
    h = np.exp(out["logh"])
    np.testing.assert_allclose(np.sum(alpha[:, None] * (1 - pi2 / h[None, :]), axis=0), 0.0, atol=1e-9)


def _bary_tv_rg_objective(h, s, alpha, eps, F):
    """Value of the pointwise barycentre problem (Sec. 5.2, the minimisation
    over (s~, h) that defines Table estimatebary) at a given h, with the
    inner minimisation over s~ done in closed form:
      TV : eps KLbar(s~|s) + lam |s~ - h| is minimised by s~ = h clamped to
           [s e^{-lam/eps}, s e^{lam/eps}] (first-order condition);
      RG : the indicator of s~ in [b1 h, b2 h] leaves s~ = s clamped there."""
    if F.kind == "tv":
        lo, hi = s * np.exp(-F.lam / eps), s * np.exp(F.lam / eps)
        st = np.clip(h, lo, hi)
        return float(np.sum(alpha * (eps * _kl_bar_vec(st, s) + F.lam * np.abs(st - h))))
    st = np.clip(s, F.alpha * h, F.beta * h)
    return float(np.sum(alpha * eps * _kl_bar_vec(st, s)))


def _kl_bar_vec(a, b):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(a > 0, a * np.log(a / b) - a + b, b)


@pytest.mark.parametrize("F", [O.TV(0.3), O.TV(0.02), O.RG(0.7, 1.3), O.RG(0.0, 1.5)])
def test_bary_h_tv_rg_minimises_the_pointwise_problem(F):
    """Table estimatebary (iii)/(iv): the oracle's h attains the minimum of the
    defining pointwise problem, found independently by a bounded scalar search
    on log h, and no smaller h does as well (the smallest minimiser is taken
    where the minimiser is an interval)."""
    rng = np.random.default_rng(53)
    for _ in range(12):
        n = 5
        s = np.exp(rng.uniform(-2, 2, n))
        alpha = rng.uniform(0.2, 1.0, n)
        eps = rng.uniform(0.01, 0.3)
        logh = O.bary_logh(np.log(s)[:, None], alpha, eps, F)[0]
        assert np.isfinite(logh)
        val = _bary_tv_rg_objective(np.exp(logh), s, alpha, eps, F)
        obj = lambda lh: _bary_tv_rg_objective(np.exp(lh), s, alpha, eps, F)
        lo, hi = np.log(s).min() - 8, np.log(s).max() + 8
        grid = np.linspace(lo, hi, 4001)
        k = int(np.argmin([obj(x) for x in grid]))
        r = optimize.minimize_scalar(obj, bounds=(grid[max(k - 2, 0)], grid[min(k + 2, 4000)]), method="bounded",
                                     options=dict(xatol=1e-12))
        best = min(r.fun, min(obj(x) for x in grid))
        assert val <= best + 1e-10 * max(1.0, abs(best))
        assert obj(logh - 1e-4) > val + 1e-14


def test_bary_h_tv_rg_special_cases():
    T = np.log(np.full((4, 1), 0.7))
    alpha = np.array([0.1, 0.2, 0.3, 0.4])
    # identical inputs: TV gives h = s; RG gives the smallest minimiser s / b2
    assert O.bary_logh(T, alpha, 0.05, O.TV(0.3))[0] == pytest.approx(np.log(0.7), abs=1e-12)
    assert O.bary_logh(T, alpha, 0.05, O.RG(0.6, 1.25))[0] == pytest.approx(np.log(0.7 / 1.25), abs=1e-12)
    # TV with zeros: h = 0 iff the weight of the zero inputs is at least that of the others
    s = np.array([[0.0], [0.0], [2.0], [1.0]])
    with np.errstate(divide="ignore"):
        L = np.log(s)
    assert np.isneginf(O.bary_logh(L, np.array([0.3, 0.3, 0.2, 0.2]), 0.05, O.TV(0.3))[0])
    assert np.isfinite(O.bary_logh(L, np.array([0.1, 0.1, 0.4, 0.4]), 0.05, O.TV(0.3))[0])
    # RG: any zero input forces h = 0
    assert np.isneginf(O.bary_logh(L, alpha, 0.05, O.RG(0.6, 1.25))[0])
    # lam -> 0 for TV: the clamp saturates at once, h is the weighted median of s
    s = np.array([[1.0], [2.0], [5.0]])
    lh = O.bary_logh(np.log(s), np.array([0.2, 0.5, 0.3]), 1.0, O.TV(1e-9))[0]
    assert lh == pytest.approx(np.log(2.0), abs=1e-6)


@pytest.mark.parametrize("F2", [O.TV(0.05), O.RG(0.8, 1.25)])
def test_barycenter_tv_rg_fixed_point(F2):
    """Barycentres with TV / range penalties on the second marginals (Table
    estimatebary (iii)/(iv)): the iteration converges, and at its fixed point
    each coupling's Y marginal s~_k lies in the band the divergence allows
    around h (TV: h e^{-lam/eps} .. h e^{lam/eps}; RG: b1 h .. b2 h), while h
    solves the pointwise problem for the Y marginals (its objective, checked
    as in the estimate pins, is not improved by a smaller h)."""
    G = O.GridGeom((10, 9), (1 / 10, 1 / 9))
    rng = np.random.default_rng(59)
    ldx = np.full(G.N, np.log(1 / G.N))
    eps = 0.02
    p = rng.uniform(0.3, 1.5, (3, G.N))
    alpha = np.array([0.2, 0.5, 0.3])
    out = O.barycenter(G, np.log(p), alpha, ldx, ldx, O.KL(0.5), F2, eps, tol=1e-12, max_iter=20000)
    assert out["res"][-1] <= 1e-12
    T = np.stack([G.lse_y(out["u"][k] / eps + ldx, eps) for k in range(3)])
    st = np.exp(out["v"] / eps + T)
    h = np.exp(out["logh"])
    if F2.kind == "tv":
        lo, hi = h * np.exp(-F2.lam / eps), h * np.exp(F2.lam / eps)
    else:
        lo, hi = F2.alpha * h, F2.beta * h
    assert np.all(st >= lo * (1 - 1e-9)) and np.all(st <= hi * (1 + 1e-9))
    # h is the estimate of its own inputs: recomputing it from T changes nothing
    np.testing.assert_allclose(O.bary_logh(T, alpha, eps, F2), out["logh"], rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# Algorithm 4: a function F3 of the total mass of the plan
# ---------------------------------------------------------------------------
def test_mass_algo_free_mass_is_algorithm_1():
    """F3 = 0 on the nonnegative reals (RG with bounds 0, inf): z stays 1 and
    Algorithm 4 is Algorithm 1."""
    rng = np.random.default_rng(61)
    x, y, p, q, dx, dy = _rand_problem(rng, 7, 6)
    C = O.sq_dist(x, y)
    eps = 0.05
    a4 = O.mass_scaling_algo(C, p, q, dx, dy, O.KL(0.4), O.TV(0.2), O.RG(0.0, np.inf), 1.0, eps, 30)
    a1 = O.scaling_algo(C, p, q, dx, dy, O.KL(0.4), O.TV(0.2), eps, 30)
    for (u4, v4, lz), (u1, v1) in zip(a4, a1):
        assert lz == 0.0
        np.testing.assert_allclose(u4, u1, rtol=1e-13, atol=1e-15)
        np.testing.assert_allclose(v4, v1, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("F3", [O.EQ, O.KL(0.3), O.TV(0.1), O.RG(0.5, 0.8)])
def test_mass_algo_log_domain_matches_scaling(F3):
    """The log-domain form (potentials and zeta = log z) gives the iterates of
    the scaling form of Algorithm 4."""
    rng = np.random.default_rng(67)
    x, y, p, q, dx, dy = _rand_problem(rng, 8, 9)
    C = O.sq_dist(x, y)
    eps, m0 = 0.05, 0.6
    sc = O.mass_scaling_algo(C, p, q, dx, dy, O.KL(0.5), O.KL(0.5), F3, m0, eps, 25)
    g = O.DenseGeom(C)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    for n in (1, 7, 25):
        s = O.solve_mass(g, *lg, O.KL(0.5), O.KL(0.5), F3, np.log(m0), eps, tol=0.0, max_iter=n)
        u, v, lz = sc[n - 1]
        np.testing.assert_allclose(s["u"], u, rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(s["v"], v, rtol=1e-11, atol=1e-13)
        assert s["zeta"] == pytest.approx(lz, rel=1e-11, abs=1e-13)


def test_partial_transport_lp_limit():
    """Optimal partial transport (Sec. 4.4, Algorithm 4 with F1, F2 the
    domination constraints RG[0, 1] and F3 the equality with m0): as eps -> 0
    the plan's cost tends to the LP optimum of min <C, R> subject to
    R dy <= p, R^T dx <= q, total mass m0, and the plan carries mass m0 and
    respects the dominations."""
    rng = np.random.default_rng(71)
    x, y, p, q, dx, dy = _rand_problem(rng, 6, 7)
    C = O.sq_dist(x, y)
    N, M = C.shape
    m0 = 0.6 * min(np.sum(p * dx), np.sum(q * dy))
    W = (dx[:, None] * dy[None, :]).reshape(-1)
    A_ub = np.zeros((N + M, N * M))
    for i in range(N):
        A_ub[i, i * M:(i + 1) * M] = dy
    for j in range(M):
        A_ub[N + j, j::M] = dx
    lp = optimize.linprog(C.reshape(-1) * W, A_ub=A_ub, b_ub=np.r_[p, q], A_eq=W[None, :], b_eq=[m0],
                          bounds=(0, None), method="highs")
    assert lp.status == 0
    g = O.DenseGeom(C)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    dom = O.RG(0.0, 1.0)
    prev = None
    for eps in (1e-2, 3e-3, 1e-3):
        s = O.solve_mass(g, *lg, dom, dom, O.EQ, np.log(m0), eps, tol=1e-12, max_iter=400000)
        assert s["converged"]
        R = np.exp((s["u"][:, None] + s["v"][None, :] - C) / eps + s["zeta"])
        pi1, pi2 = R @ dy, R.T @ dx
        assert np.sum(R * W.reshape(N, M)) == pytest.approx(m0, rel=1e-9)
        assert np.all(pi1 <= p * (1 + 1e-9)) and np.all(pi2 <= q * (1 + 1e-9))
        cost = np.sum(C * R * W.reshape(N, M))
        assert cost >= lp.fun - 1e-9
        assert cost - lp.fun <= 3 * eps * np.log(N * M) + 1e-9
        if prev is not None:
            assert cost - lp.fun <= prev + 1e-12
        prev = cost - lp.fun


# ---------------------------------------------------------------------------
# mass balance of a starting potential (KL on both marginals)
# ---------------------------------------------------------------------------
def _explicit_first_marginal(x, y, u, v, dy, eps):
    """sum_j exp((u_i + v_j - |x_i - y_j|^2)/eps) dy_j from the plan itself."""
    C = ((x[:, None, :] - y[None, :, :]) ** 2).sum(-1)
    return (np.exp((u[:, None] + v[None, :] - C) / eps) * dy[None, :]).sum(1)


def test_mass_balance_shift_vanishes_at_the_fixed_point():
    """At the fixed point both marginals of the plan carry its mass, so the
    shift is 0 (lam1 != lam2 and non-uniform dx, dy: a swapped lam, a dropped
    reference weight or a wrong exponent sign leaves it non-zero)."""
    rng = np.random.default_rng(21)
    x, y, p, q, dx, dy = _rand_problem(rng, 30, 25)
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    F1, F2, eps = O.KL(0.4), O.KL(0.9), 0.05
    s = O.solve(g, *lg, F1, F2, eps, tol=1e-14, max_iter=100000)
    assert abs(O.mass_balance_shift(g, *lg, F1, F2, eps, s["v"])) < 1e-10
    # away from it the shift is not small
    assert abs(O.mass_balance_shift(g, *lg, F1, F2, eps, s["v"] + 0.05)) > 1e-3


@pytest.mark.parametrize("lams", [(0.4, 0.9), (1.0, 1.0), (2.0, 0.3)])
def test_mass_balance_shift_is_the_root_of_the_mass_mismatch(lams):
    """The shift against a root search: v0 - t for trial t, a full X
    half-step, the first-marginal mass read off the explicit plan, against the
    second-marginal mass q e^(-v/lam2) implied by v0 - t."""
    rng = np.random.default_rng(22)
    x, y, p, q, dx, dy = _rand_problem(rng, 20, 17)
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    F1, F2, eps = O.KL(lams[0]), O.KL(lams[1]), 0.08
    v0 = rng.normal(0.0, 0.2, len(y))

    def mismatch(t):
        v = v0 - t
        _, u1, _ = O.half_step_x(g, lg[0], lg[2], lg[3], F1, eps, np.zeros(len(x)), v)
        P = (_explicit_first_marginal(x, y, u1, v, dy, eps) * dx).sum()
        Q = (q * np.exp(-v / F2.lam) * dy).sum()
        return np.log(P) - np.log(Q)

    t = optimize.brentq(mismatch, -20.0, 20.0, xtol=1e-14)
    s = O.mass_balance_shift(g, *lg, F1, F2, eps, v0)
    assert abs(s - t) < 1e-10
    # exact along constants: a second shift from the shifted start is 0
    assert abs(O.mass_balance_shift(g, *lg, F1, F2, eps, v0 - s)) < 1e-11


def test_mass_balance_keeps_the_fixed_point():
    """By Prop. alternating the start only changes the path: the balanced
    start reaches the same potentials (and, the constant mode being the
    slowest, in fewer iterations here)."""
    rng = np.random.default_rng(23)
    x, y, p, q, dx, dy = _rand_problem(rng, 40, 35)
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    F, eps = O.KL(0.5), 0.02
    cold = O.solve(g, *lg, F, F, eps, tol=1e-12, max_iter=100000)
    s = O.mass_balance_shift(g, *lg, F, F, eps, np.zeros(len(y)))
    bal = O.solve(g, *lg, F, F, eps, tol=1e-12, max_iter=100000, v0=np.full(len(y), -s))
    np.testing.assert_allclose(bal["u"], cold["u"], atol=1e-9)
    np.testing.assert_allclose(bal["v"], cold["v"], atol=1e-9)
    assert bal["iters"] < cold["iters"]


def test_mass_balance_rejects_other_penalties():
    rng = np.random.default_rng(24)
    x, y, p, q, dx, dy = _rand_problem(rng, 5, 4)
    g = O.PointsGeom(x, y)
    with pytest.raises(ValueError):
        O.mass_balance_shift(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.TV(0.1), O.KL(1.0), 0.1,
                             np.zeros(4))


@pytest.mark.parametrize("K", [1, 2, 7])
def test_solve_rebalance_is_a_restart_from_the_balanced_v(K):
    """The in-solve mass balance at iteration K against its definition: the
    plain iteration for K - 1 iterations, the start v - s of
    `mass_balance_shift` (pinned above against a root search on the explicit
    plan), and the plain iteration from there.  The rebalanced solve takes the
    shift after the X half-step (u + theta1 s), so this also pins the affine
    dependence of u on a constant shift of v; lam1 != lam2 and non-uniform
    weights make a swapped lam or a wrong theta visible."""
    rng = np.random.default_rng(25)
    x, y, p, q, dx, dy = _rand_problem(rng, 30, 26)
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.log(dx), np.log(dy))
    F1, F2, eps, n = O.KL(0.4), O.KL(0.9), 0.05, 12
    reb = O.solve(g, *lg, F1, F2, eps, tol=0.0, max_iter=n, rebalance_at=K)
    v, u = np.zeros(len(y)), np.zeros(len(x))
    if K > 1:
        first = O.solve(g, *lg, F1, F2, eps, tol=0.0, max_iter=K - 1)
        v, u = first["v"], first["u"]
    s = O.mass_balance_shift(g, *lg, F1, F2, eps, v)
    assert abs(s) > 1e-3                     # a real shift
    rest = O.solve(g, *lg, F1, F2, eps, tol=0.0, max_iter=n - K + 1, v0=v - s, u0=u)
    np.testing.assert_allclose(reb["u"], rest["u"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(reb["v"], rest["v"], rtol=0, atol=1e-12)
    np.testing.assert_allclose(reb["res"][K:], rest["res"][1:], rtol=1e-9, atol=0)


def test_solve_rebalance_keeps_the_fixed_point_and_converges_faster():
    """Only v enters the iterates (Prop. alternating): the rebalanced solve
    reaches the plain solve's potentials; on this problem (KL 1, eps 5e-3,
    uniform points) the balance once the shape has settled (iteration 30)
    removes most of the slow constant mode."""
    rng = np.random.default_rng(26)
    x, y = rng.uniform(0, 1, (120, 2)), rng.uniform(0, 1, (100, 2))
    p, q = rng.uniform(0.1, 1.0, 120), rng.uniform(0.1, 1.0, 100)
    g = O.PointsGeom(x, y)
    lg = (np.log(p), np.log(q), np.full(120, -np.log(120)), np.full(100, -np.log(100)))
    F, eps = O.KL(1.0), 5e-3
    plain = O.solve(g, *lg, F, F, eps, tol=1e-9, max_iter=100000)
    s0 = O.mass_balance_shift(g, *lg, F, F, eps, np.zeros(100))
    once = O.solve(g, *lg, F, F, eps, tol=1e-9, max_iter=100000, v0=np.full(100, -s0))
    twice = O.solve(g, *lg, F, F, eps, tol=1e-9, max_iter=100000, v0=np.full(100, -s0), rebalance_at=30)
    np.testing.assert_allclose(twice["u"], plain["u"], atol=1e-7)
    np.testing.assert_allclose(twice["v"], plain["v"], atol=1e-7)
    assert twice["iters"] < 0.7 * once["iters"] < 0.7 * plain["iters"]
