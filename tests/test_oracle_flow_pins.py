"""Pins of the oracle's gradient-flow pieces (Sec. 5.3) and of the WF cost
with a cut locus (Definition WF, eq. "logcost"), against what the mathematics
fixes: brute-force minimisation of the pointwise and whole-step problems, the
textbook WF distance between two Dirac masses, the Gaussian closed form of an
entropic heat-flow step, and the decoupling that exact kernel zeros imply."""
import numpy as np
import pytest
from scipy import optimize

from oracle import uot_oracle as O


def kl_pt(s, r):
    s = np.asarray(s, float)
    r = np.asarray(r, float)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(s > 0, s * np.log(s / r), 0.0) - s + r


# ---------------------------------------------------------------------------
# the growth functional of the tumour example and its proxdiv
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("lam", [0.0, 0.1, 0.45])
def test_growth_value_is_the_inner_minimum(lam):
    rng = np.random.default_rng(1)
    for _ in range(40):
        s, p = rng.uniform(0.01, 3.0), rng.uniform(0.1, 2.0)
        res = optimize.minimize_scalar(lambda r: kl_pt(s, r) - lam * r, bounds=(1e-12, p), method="bounded",
                                       options={"xatol": 1e-13})
        assert O.growth_value(s, p, lam) == pytest.approx(min(res.fun, kl_pt(s, p) - lam * p), abs=1e-9)
    # dx-weighted sum in F_value
    s = rng.uniform(0.1, 2, 5)
    p = rng.uniform(0.1, 2, 5)
    dx = rng.uniform(0.5, 1.5, 5)
    assert O.F_value(O.GROWTH(lam), s, p, dx) == pytest.approx(float(np.sum(dx * O.growth_value(s, p, lam))))


@pytest.mark.parametrize("lam,eps", [(0.1, 0.05), (0.3, 0.5), (0.0, 0.2)])
def test_growth_proxdiv_is_the_prox(lam, eps):
    """proxdiv_F(s, u, eps) = argmin_x [eps KL(x | s e^{-u/eps}) + F(x)] / s,
    with F itself an inner minimum over r <= p; both minimisations by brute
    force (a joint convex problem in (x, r))."""
    rng = np.random.default_rng(2)
    F = O.GROWTH(lam)
    for _ in range(30):
        s, p, u = rng.uniform(0.05, 3.0), rng.uniform(0.2, 2.0), rng.uniform(-0.3, 0.3)
        z = s * np.exp(-u / eps)

        def obj(t):
            x, r = np.exp(t[0]), p / (1.0 + np.exp(-t[1]))       # r in (0, p)
            return eps * kl_pt(x, z) + kl_pt(x, r) - lam * r

        best = None
        for t0 in ([np.log(z + 1e-3), 0.0], [0.0, 3.0], [np.log(p), 8.0]):
            r = optimize.minimize(obj, t0, method="Nelder-Mead",
                                  options={"xatol": 1e-12, "fatol": 1e-15, "maxiter": 20000})
            if best is None or r.fun < best.fun:
                best = r
        # the cap itself (r = p) is the limit of the sigmoid: also try it exactly
        rb = optimize.minimize_scalar(lambda lx: eps * kl_pt(np.exp(lx), z) + kl_pt(np.exp(lx), p) - lam * p,
                                      bounds=(-30, 5), method="bounded", options={"xatol": 1e-12})
        x = np.exp(best.x[0]) if best.fun < rb.fun else np.exp(rb.x)
        got = np.exp(O.proxdiv_log(F, np.log(p), np.log(s), u, eps))
        assert got == pytest.approx(x / s, rel=2e-5)


def test_growth_proxdiv_matches_the_printed_two_branch_form():
    """Cap 1: the log form min(...) equals the example's two-branch formula
    (first branch while s <= e^{u/eps} kappa^{(1+eps)/eps})."""
    rng = np.random.default_rng(3)
    for lam, eps in [(0.012, 0.3), (0.2, 0.1), (0.5, 1.0)]:
        s = np.exp(rng.uniform(-12, 3, 400))
        u = rng.uniform(-0.5, 0.5, 400)
        one = np.ones_like(s)
        a = np.exp(O.proxdiv_log(O.GROWTH(lam), np.log(one), np.log(s), u, eps))
        b = O.proxdiv_scaling(O.GROWTH(lam), one, s, u, eps)
        np.testing.assert_allclose(a, b, rtol=1e-10)
        # both branches are exercised
        kap = 1 - lam
        low = s <= np.exp(u / eps) * kap ** ((1 + eps) / eps)
        assert low.any() and (~low).any()


@pytest.mark.parametrize("lam", [0.05, 0.4])
def test_growth_conjugate_is_the_sup(lam):
    rng = np.random.default_rng(4)
    for _ in range(30):
        w, p = rng.uniform(-2.0, 1.5), rng.uniform(0.2, 2.0)
        res = optimize.minimize_scalar(lambda ls: -(w * np.exp(ls) - O.growth_value(np.exp(ls), p, lam)),
                                       bounds=(-40, 8), method="bounded", options={"xatol": 1e-12})
        sup = max(-res.fun, 0.0)                               # s = 0 gives 0
        got = O.F_conj(O.GROWTH(lam), np.array([w]), np.array([p]), np.array([1.0]))
        assert got == pytest.approx(sup, abs=1e-8)


# ---------------------------------------------------------------------------
# several species: joint prox of the growth functional and next densities
# ---------------------------------------------------------------------------
def _joint_min(y, q, lam):
    """min over r >= 0, sum r <= q of sum_k KL(y_k | r_k) - lam sum r_k."""
    n = len(y)
    cons = [{"type": "ineq", "fun": lambda r: q - np.sum(r)}]
    r0 = np.full(n, 0.5 * q / n)
    res = optimize.minimize(lambda r: float(np.sum(kl_pt(y, r)) - lam * np.sum(r)), r0, method="SLSQP",
                            bounds=[(1e-12, q)] * n, constraints=cons, options={"ftol": 1e-15, "maxiter": 1000})
    return res


@pytest.mark.parametrize("lam", [0.1, 0.35])
def test_growth_next_is_the_inner_minimiser(lam):
    rng = np.random.default_rng(5)
    for _ in range(30):
        y = rng.uniform(0.05, 1.2, 2)
        q = rng.uniform(0.5, 1.5)
        r = _joint_min(y, q, lam)
        got = np.exp(O.growth_next_log(np.log(y)[:, None], np.log(np.array([q])), lam))[:, 0]
        np.testing.assert_allclose(got, r.x, rtol=1e-5, atol=1e-8)
    # one species: min(y / kappa, q), as the paper states for the tumour flow
    y = rng.uniform(0.01, 2.0, 50)
    got = np.exp(O.growth_next_log(np.log(y)[None, :], np.zeros(50), 0.2))[0]
    np.testing.assert_allclose(got, np.minimum(y / 0.8, 1.0), rtol=1e-14)


@pytest.mark.parametrize("lam,eps", [(0.1, 0.1), (0.3, 0.5)])
def test_joint_growth_prox_brute_force(lam, eps):
    """Two species at one point: the joint proxdiv (u = 0) of the growth
    functional on s^a + s^b, i.e. argmin_x eps sum_k KL(x_k | s_k) + G(x), by
    brute force over (x, r)."""
    rng = np.random.default_rng(6)
    for _ in range(15):
        s = rng.uniform(0.02, 2.0, 2)
        q = rng.uniform(0.5, 1.5)

        def obj(t):
            x = np.exp(t)
            return eps * float(np.sum(kl_pt(x, s))) + _joint_min(x, q, lam).fun

        res = optimize.minimize(obj, np.log(s), method="Nelder-Mead",
                                options={"xatol": 1e-10, "fatol": 1e-14, "maxiter": 4000})
        x = np.exp(res.x)
        v = O.growth_joint_pot(np.log(s)[:, None], np.log(np.array([q])), lam, eps)[:, 0]
        np.testing.assert_allclose(np.exp(v / eps), x / s, rtol=1e-4)


# ---------------------------------------------------------------------------
# WF cost with a cut locus
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [0.05, 0.17, 0.25, 0.31])
def test_wf_cost_two_diracs(d):
    """WF_1 between m0 delta_x and m1 delta_y is m0 + m1 - 2 sqrt(m0 m1)
    cos_+(theta) (the textbook formula for the cost -log cos_+^2, lambda = 1).
    The unregularised objective <C, R> + KL(pi1|m0) + KL(pi2|m1) at the
    entropic plan r = (m0 m1 e^{-c})^{1/(2+eps)} is within O(eps^2) of it (r
    moves by O(eps) from the unregularised minimiser).  Beyond the cut no mass
    moves and the value is m0 + m1."""
    cut = 0.3
    m0, m1 = 0.7, 1.6
    g = O.PointsGeom(np.array([[0.0]]), np.array([[d]]), cost="wf", cut=cut)
    one = np.array([1.0])
    eps = 1e-3
    r = O.solve(g, np.log([m0]), np.log([m1]), np.log(one), np.log(one), O.KL(1.0), O.KL(1.0), eps,
                tol=1e-12, max_iter=200000)
    assert r["converged"]
    o = O.objective(g, [m0], [m1], one, one, O.KL(1.0), O.KL(1.0), eps, r["u"], r["v"])
    theta = 0.5 * np.pi * min(d / cut, 1.0)
    wf2 = m0 + m1 - 2 * np.sqrt(m0 * m1) * (np.cos(theta) if d < cut else 0.0)
    val = o["transport_cost"] + O.F_value(O.KL(1.0), o["pi1"], np.array([m0]), one) \
        + O.F_value(O.KL(1.0), o["pi2"], np.array([m1]), one)
    assert val == pytest.approx(wf2, abs=1e-5)
    assert o["gap"] == pytest.approx(0.0, abs=1e-9)


def test_wf_grid_1d_matches_dense():
    n, cut = 37, 0.23
    g = O.GridGeom((n,), (1.0 / n,), cost="wf", cut=cut)
    dg = g.dense()
    assert np.isinf(dg.C).any() and np.isfinite(dg.C).any()
    rng = np.random.default_rng(7)
    w = rng.normal(size=n)
    for eps in (1e-3, 0.05):
        np.testing.assert_allclose(g.lse_x(w, eps), dg.lse_x(w, eps), rtol=1e-13, atol=1e-12)
    wx, wy = rng.normal(size=n), rng.normal(size=n)
    assert g.cost_moment_log(wx, wy, 0.05) == pytest.approx(dg.cost_moment_log(wx, wy, 0.05), rel=1e-12)


def test_wf_cut_decouples_clusters():
    """Two clusters farther apart than the cut: K is block diagonal, so the
    joint problem is the two problems side by side (exact zeros of K)."""
    rng = np.random.default_rng(8)
    cut = 0.2
    xa, ya = rng.uniform(0, 0.1, (6, 2)), rng.uniform(0, 0.1, (5, 2))
    xb, yb = rng.uniform(0.5, 0.6, (4, 2)), rng.uniform(0.5, 0.6, (7, 2))
    pa, qa, pb, qb = (rng.uniform(0.5, 1.5, k) for k in (6, 5, 4, 7))
    F = O.KL(0.5)
    eps = 0.01
    run = lambda x, y, p, q: O.solve(O.PointsGeom(x, y, "wf", cut), np.log(p), np.log(q), np.zeros(len(p)),
                                     np.zeros(len(q)), F, F, eps, tol=0.0, max_iter=300)
    ra, rb = run(xa, ya, pa, qa), run(xb, yb, pb, qb)
    r = run(np.vstack([xa, xb]), np.vstack([ya, yb]), np.r_[pa, pb], np.r_[qa, qb])
    np.testing.assert_allclose(r["u"], np.r_[ra["u"], rb["u"]], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(r["v"], np.r_[ra["v"], rb["v"]], rtol=1e-12, atol=1e-14)


def test_isolated_point_carries_no_mass():
    """A point of X with every point of Y beyond the cut: K b vanishes there,
    its row of the plan is zero and the other rows are as without it."""
    cut = 0.2
    x = np.array([[0.0], [0.05], [0.9]])
    y = np.array([[0.02], [0.08]])
    p, q = np.array([1.0, 0.8, 1.3]), np.array([0.9, 1.1])
    F = O.KL(1.0)
    r3 = O.solve(O.PointsGeom(x, y, "wf", cut), np.log(p), np.log(q), np.zeros(3), np.zeros(2), F, F, 0.01,
                 tol=0.0, max_iter=200)
    r2 = O.solve(O.PointsGeom(x[:2], y, "wf", cut), np.log(p[:2]), np.log(q), np.zeros(2), np.zeros(2), F, F,
                 0.01, tol=0.0, max_iter=200)
    assert np.isneginf(r3["S"][2]) and r3["u"][2] == np.inf
    np.testing.assert_allclose(r3["u"][:2], r2["u"], rtol=1e-13)
    np.testing.assert_allclose(r3["v"], r2["v"], rtol=1e-13)
    assert all(np.isfinite(r3["res"]))
    o = O.objective(O.PointsGeom(x, y, "wf", cut), p, q, np.ones(3), np.ones(2), F, F, 0.01, r3["u"], r3["v"])
    assert o["pi1"][2] == 0.0 and np.isfinite(o["primal"]) and np.isfinite(o["dual"])


# ---------------------------------------------------------------------------
# whole steps by brute force on tiny problems
# ---------------------------------------------------------------------------
def _brute_force_plans(C, dx, logp, q, lam, eps):
    """Minimise sum_k [<C, R_k> + eps KL(R_k | dx dy) + KL(R_k dy | p_k)]
    + sum_j dy_j G(sum_k (R_k^T dx)_j) over the entries with finite C."""
    n = logp.shape[0]
    N = C.shape[0]
    mask = np.isfinite(C)
    nz = int(mask.sum())
    W = dx[:, None] * dx[None, :]
    kap = 1.0 - lam
    p = np.exp(logp)
    Cm = np.where(mask, C, 0.0)

    def unpack(t):
        R = np.zeros((n, N, N))
        for k in range(n):
            R[k][mask] = np.exp(t[k * nz:(k + 1) * nz])
        return R

    def f(t):
        R = unpack(t)
        val = 0.0
        grad = np.zeros_like(R)
        X = np.zeros(N)
        for k in range(n):
            Rk = R[k]
            with np.errstate(divide="ignore", invalid="ignore"):
                ent = np.where(Rk > 0, Rk * np.log(Rk), 0.0) - Rk + 1.0
            val += float(np.sum(W * (Cm * Rk + eps * ent)))
            pi1 = Rk @ dx
            val += float(np.sum(dx * kl_pt(pi1, p[k])))
            X += Rk.T @ dx
            with np.errstate(divide="ignore"):
                grad[k] = W * (Cm + eps * np.log(np.where(mask, Rk, 1.0)) + np.log(pi1 / p[k])[:, None])
        val += float(np.sum(dx * O.growth_value(X, q, lam)))
        gp = np.log(np.maximum(kap, X / q))
        for k in range(n):
            grad[k] += W * gp[None, :]
        g = np.concatenate([(grad[k] * R[k])[mask] for k in range(n)])
        return val, g

    t0 = np.concatenate([np.log(np.full(nz, 0.3))] * n)
    res = optimize.minimize(f, t0, jac=True, method="L-BFGS-B",
                            options={"maxiter": 50000, "ftol": 1e-16, "gtol": 1e-13, "maxcor": 50})
    return unpack(res.x)


@pytest.mark.parametrize("species", [1, 2])
def test_growth_step_brute_force(species):
    """One step of the WF growth flow (F1 = KL(. | p_k), joint growth on the
    second marginals, WF cost with some pairs cut): the plans of the scaling
    iteration's fixed point minimise the step's primal."""
    N = 5
    h = 1.0 / N
    g = O.GridGeom((N,), (h,), cost="wf", cut=0.5)
    C = g.dense().C
    assert np.isinf(C).any()
    dx = np.full(N, h)
    rng = np.random.default_rng(10 + species)
    p = rng.uniform(0.3, 1.2, (species, N))
    q = rng.uniform(0.6, 1.0, N)
    lam, eps = 0.2, 0.08
    r = O.solve_species(g, np.log(p), np.log(q), np.log(dx), np.log(dx), lam, eps, tol=1e-14, max_iter=20000)
    assert r["converged"]
    R_it = np.exp((r["u"][:, :, None] + r["v"][:, None, :] - C[None]) / eps)
    R_bf = _brute_force_plans(C, dx, np.log(p), q, lam, eps)
    np.testing.assert_allclose(R_it, R_bf, rtol=2e-5, atol=1e-9)
    if species == 1:
        # one species: the plain iteration with the growth divergence
        r1 = O.solve(g, np.log(p[0]), np.log(q), np.log(dx), np.log(dx), O.KL(1.0), O.GROWTH(lam), eps,
                     tol=1e-14, max_iter=20000)
        np.testing.assert_allclose(r1["v"], r["v"][0], rtol=1e-11, atol=1e-13)
        np.testing.assert_allclose(r1["u"], r["u"][0], rtol=1e-11, atol=1e-13)


# ---------------------------------------------------------------------------
# heat flow: one entropic JKO step of a Gaussian
# ---------------------------------------------------------------------------
def _gaussian_step_var(sig, tau, eps):
    """Among Gaussian plans with first marginal N(0, sig^2): minimise
    E|X - Y|^2 - eps H(plan) - 2 tau H(second marginal), i.e.
    sig^2 + s^2 - 2 c sig s - eps/2 log(sig^2 s^2 (1 - c^2)) - tau log s^2."""
    # stationarity in c: eps c / (1 - c^2) = 2 sig s, a quadratic in c;
    # stationarity in s: s^2 - c sig s - (eps/2 + tau) = 0
    def corr(s):
        a = 2 * sig * s
        return (-eps + np.sqrt(eps * eps + 4 * a * a)) / (2 * a)

    s = optimize.brentq(lambda s: s * s - corr(s) * sig * s - (0.5 * eps + tau), sig, 4 * sig, xtol=1e-16)
    return s * s


def test_heat_step_of_a_gaussian():
    """Heat flow step (F1 = iota_=(p_k), F2 = 2 tau KL(. | 1)) of a Gaussian
    well inside [0, 1]: the next density is the Gaussian whose variance the
    Gaussian optimality conditions give (sampling the grid is exact up to
    exponentially small terms here)."""
    n = 400
    h = 1.0 / n
    xs = (np.arange(n) + 0.5) * h
    sig, tau, eps = 0.05, 4e-4, 2e-4
    p0 = np.exp(-0.5 * ((xs - 0.5) / sig) ** 2)
    p0 /= np.sum(p0) * h
    dens, info = O.flow(O.GridGeom((n,), (h,)), "heat", p0[None], np.ones(n), np.full(n, h), tau, eps, 1, 20000,
                        tol=1e-13)
    assert info[0]["converged"]
    p1 = dens[1][0]
    m = np.sum(p1 * h)
    mu = np.sum(p1 * xs * h) / m
    var = np.sum(p1 * (xs - mu) ** 2 * h) / m
    assert m == pytest.approx(1.0, abs=1e-10)
    assert mu == pytest.approx(0.5, abs=1e-10)
    assert var == pytest.approx(_gaussian_step_var(sig, tau, eps), rel=1e-6)
    assert var > sig * sig


def test_flow_invariants():
    n = 60
    h = 1.0 / n
    xs = (np.arange(n) + 0.5) * h
    p0 = 0.95 * np.exp(-((xs - 0.35) / 0.12) ** 2) + 0.02
    q = np.ones(n)
    dx = np.full(n, h)
    # crowd projection: mass kept, density below the cap
    d, info = O.flow(O.GridGeom((n,), (h,)), "crowd", 2.5 * p0[None], q, dx, 0.0, 1e-3, 1, 20000, tol=1e-11)
    assert np.sum(d[1]) * h == pytest.approx(np.sum(2.5 * p0) * h, rel=1e-9)
    assert d[1].max() <= 1.0 + 1e-12
    # growth: mass grows, density capped; two species share the cap
    g = O.GridGeom((n,), (h,), cost="wf", cut=0.3)
    d, info = O.flow(g, "growth", p0[None], q, dx, 0.05, 2e-3, 3, 400, alpha=1.0)
    masses = [float(np.sum(a) * h) for a in d]
    assert all(b > a for a, b in zip(masses, masses[1:]))
    assert all(a.max() <= 1.0 + 1e-12 for a in d)
    pa = 0.5 * p0
    pb = 0.4 * np.exp(-((xs - 0.7) / 0.1) ** 2) + 0.01
    d2, _ = O.flow(g, "growth", np.stack([pa, pb]), q, dx, 0.05, 2e-3, 3, 400, alpha=1.0)
    tot = [a.sum(axis=0) for a in d2]
    assert all(t.max() <= 1.0 + 1e-12 for t in tot)
    assert all(np.all(a > 0) for a in d2)


# ---------------------------------------------------------------------------
# barycentric projection (colour transfer)
# ---------------------------------------------------------------------------
def _gauss_corr(s1, s2, eps):
    """Correlation of the entropic plan between N(0, s1^2) and N(0, s2^2) for
    the cost |x - y|^2 and entropy weight eps: stationarity of
    -2 c s1 s2 - (eps/2) log(1 - c^2), i.e. eps c / (1 - c^2) = 2 s1 s2."""
    a = 2 * s1 * s2
    return (-eps + np.sqrt(eps * eps + 4 * a * a)) / (2 * a)


@pytest.mark.parametrize("s1,s2", [(0.05, 0.05), (0.04, 0.06)])
def test_barycentric_map_of_gaussians(s1, s2):
    """Balanced entropic OT between two Gaussians well inside [0, 1] (600
    cells): the plan is Gaussian and T(x) = E[Y | X = x] = 0.5 + c (s2/s1)
    (x - 0.5) with c from the Gaussian optimality condition."""
    n = 600
    h = 1.0 / n
    xs = (np.arange(n) + 0.5) * h
    p = np.exp(-0.5 * ((xs - 0.5) / s1) ** 2)
    q = np.exp(-0.5 * ((xs - 0.5) / s2) ** 2)
    p /= p.sum() * h
    q /= q.sum() * h
    eps = 1e-3
    g = O.GridGeom((n,), (h,))
    d = np.full(n, h)
    r = O.solve(g, np.log(p), np.log(q), np.log(d), np.log(d), O.EQ, O.EQ, eps, tol=1e-13, max_iter=20000)
    assert r["converged"]
    rows = np.where(np.abs(xs - 0.5) < 3 * s1)[0]
    T = O.barycentric_map_rows(g, r["v"], np.log(d), eps, rows)[:, 0]
    c = _gauss_corr(s1, s2, eps)
    np.testing.assert_allclose(T, 0.5 + c * (s2 / s1) * (xs[rows] - 0.5), atol=1e-8)


def test_barycentric_map_mean_identity_and_translation():
    """sum_i dx_i pi1_i T_i = sum_j dy_j pi2_j y_j (the definition summed over
    the plan); every T_i lies in the hull of Y; shifting both clouds shifts T."""
    rng = np.random.default_rng(12)
    x, y = rng.uniform(0, 1, (40, 2)), rng.uniform(0, 1, (30, 2)) + 0.2
    p, q = rng.uniform(0.5, 1.5, 40), rng.uniform(0.5, 1.5, 30)
    dx, dy = np.full(40, 1 / 40), np.full(30, 1 / 30)
    F, eps = O.KL(0.3), 0.02
    g = O.PointsGeom(x, y)
    r = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), F, F, eps, tol=1e-12, max_iter=20000)
    T = O.barycentric_map_dense(g.C, y, r["v"], np.log(dy), eps)
    o = O.objective(g, p, q, dx, dy, F, F, eps, r["u"], r["v"])
    np.testing.assert_allclose((dx * o["pi1"]) @ T, (dy * o["pi2"]) @ y, rtol=1e-9)
    assert np.all(T >= y.min(0) - 1e-12) and np.all(T <= y.max(0) + 1e-12)
    t = np.array([-0.7, 0.3])
    g2 = O.PointsGeom(x + t, y + t)
    r2 = O.solve(g2, np.log(p), np.log(q), np.log(dx), np.log(dy), F, F, eps, tol=1e-12, max_iter=20000)
    T2 = O.barycentric_map_dense(g2.C, y + t, r2["v"], np.log(dy), eps)
    np.testing.assert_allclose(T2, T + t, atol=1e-9)
    # rows computed one at a time on a grid equal the dense form
    gg = O.GridGeom((6, 5, 4), (1 / 6, 1 / 5, 1 / 4))
    v = rng.normal(0, 0.01, 120)
    Td = O.barycentric_map_dense(gg.dense().C, O.grid_points(gg.shape, gg.h), v, np.zeros(120), 0.05)
    np.testing.assert_allclose(O.barycentric_map_rows(gg, v, np.zeros(120), 0.05, np.arange(120)), Td, rtol=1e-12)
