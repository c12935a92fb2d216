"""HIP path vs the FP64 oracle, element by element, on the same seeded
inputs, through the C ABI (ctypes binding).  Tolerances: FP64 paths 1e-10
relative on potentials (fixed iteration counts: 1e-11); FP32 paths 1e-5
relative (max |du| / max(|u|_inf, eps))."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import uot_oracle as O
from paper_1607_05816_amd import synth
from tests.helpers import oracle_div, pot_rel_err, rounded

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import uot as U  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def T(a, dtype):
    return torch.tensor(np.asarray(a), dtype=dtype, device=DEV)


# ---------------------------------------------------------------------------
# builders: the same rounded inputs go to both sides
# ---------------------------------------------------------------------------
def points_case(rng, N, M, d, dtype, mass_q=1.3):
    npd = np.float32 if dtype == torch.float32 else np.float64
    x = rounded(rng.uniform(0, 1, (N, d)), npd)
    y = rounded(rng.uniform(0, 1, (M, d)), npd)
    p = rounded(rng.uniform(0.3, 1.5, N), npd)
    q = rounded(rng.uniform(0.3, 1.5, M) * mass_q, npd)
    dx = rounded(np.full(N, 1.0 / N), npd)
    dy = rounded(np.full(M, 1.0 / M), npd)
    return x, y, p, q, dx, dy


def gpu_points(x, y, p, q, dx, dy, F1, F2, dtype):
    return U.points_problem(T(x, dtype), T(y, dtype), T(p, dtype), T(q, dtype), T(dx, dtype), T(dy, dtype), F1, F2)


def oracle_points_run(x, y, p, q, dx, dy, F1, F2, eps, iters, **kw):
    g = O.PointsGeom(x, y)
    return O.solve(g, O.safe_log(p), O.safe_log(q), np.log(dx), np.log(dy), oracle_div(F1), oracle_div(F2), eps,
                   tol=kw.pop("tol", 0.0), max_iter=iters, **kw)


DIVS = [U.KL(0.5), U.EQ(), U.TV(0.1), U.RG(0.7, 1.3)]


# ---------------------------------------------------------------------------
# 1-D FP64 histogram problem (n = m = 256, KL lambda = 1, eps = 1e-2)
# ---------------------------------------------------------------------------
def test_hist1d_fp64_fixed_iterations_and_converged():
    for seed in (0, 3):
        say("case hist1d fp64 seed", seed)
        pr = synth.hist1d(seed)
        n = pr.shape[0]
        xs = (np.arange(n) + 0.5) / n
        dxv = np.full(n, 1.0 / n)
        F = U.KL(1.0)
        prob = U.points_problem(T(xs, torch.float64), T(xs, torch.float64), T(pr.p, torch.float64),
                                T(pr.q, torch.float64), T(dxv, torch.float64), T(dxv, torch.float64), F, F)
        u, v, info = U.solve(prob, 1e-2, tol=0.0, max_iter=40, record=True)
        ref = oracle_points_run(xs, xs, pr.p, pr.q, dxv, dxv, F, F, 1e-2, 40)
        assert info["iters"] == 40
        assert pot_rel_err(u.cpu(), ref["u"], 1e-2) < 1e-11
        assert pot_rel_err(v.cpu(), ref["v"], 1e-2) < 1e-11
        # residual partials are merged in FP32 on the device (they only feed the
        # stopping test): 1e-6 relative on r
        np.testing.assert_allclose(info["res_hist"].numpy()[1:], ref["res"][1:], rtol=1e-6)
        # converged to 1e-9
        u, v, info = U.solve(prob, 1e-2, tol=1e-9, max_iter=5000)
        ref = oracle_points_run(xs, xs, pr.p, pr.q, dxv, dxv, F, F, 1e-2, 5000, tol=1e-9)
        assert info["converged"] and ref["converged"]
        assert abs(info["iters"] - ref["iters"]) <= 1
        assert pot_rel_err(u.cpu(), ref["u"], 1e-2) < 1e-9
        assert pot_rel_err(v.cpu(), ref["v"], 1e-2) < 1e-9


# ---------------------------------------------------------------------------
# dense point clouds, every divergence, d = 1, 2, 3, ragged sizes
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_points_all_divergences_fixed_iterations(dtype, tolr, d):
    rng = np.random.default_rng(100 + d)
    N, M = 301, 517
    x, y, p, q, dx, dy = points_case(rng, N, M, d, dtype)
    eps = 0.05
    for F in DIVS:
        say("case points", dtype, "d", d, "div", F)
        prob = gpu_points(x, y, p, q, dx, dy, F, F, dtype)
        u, v, info = U.solve(prob, eps, tol=0.0, max_iter=25)
        ref = oracle_points_run(x, y, p, q, dx, dy, F, F, eps, 25)
        assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr, F
        assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr, F


def test_points_tiny_and_zero_density():
    # N = M = 1: one-point closed form (KL/KL, dx = dy = 1)
    say("case points 1x1")
    lam1, lam2, p, q, c, eps = 0.7, 1.3, 0.8, 1.9, 0.25, 0.05
    prob = U.points_problem(T([[0.0]], torch.float64), T([[0.5]], torch.float64), T([p], torch.float64),
                            T([q], torch.float64), T([1.0], torch.float64), T([1.0], torch.float64),
                            U.KL(lam1), U.KL(lam2))
    u, v, info = U.solve(prob, eps, tol=1e-14, max_iter=100000)
    r = math.exp((lam1 * math.log(p) + lam2 * math.log(q) - c) / (lam1 + lam2 + eps))
    assert u.item() == pytest.approx(-lam1 * math.log(r / p), rel=1e-10)
    assert v.item() == pytest.approx(-lam2 * math.log(r / q), rel=1e-10)
    # zero densities give exact -inf potentials, no NaN
    say("case points zero density")
    rng = np.random.default_rng(5)
    x, y, pp, qq, dx, dy = points_case(rng, 40, 33, 2, torch.float64)
    pp[[3, 17]] = 0.0
    qq[[0]] = 0.0
    F = U.KL(0.5)
    prob = gpu_points(x, y, pp, qq, dx, dy, F, F, torch.float64)
    u, v, info = U.solve(prob, 0.05, tol=0.0, max_iter=30)
    ref = oracle_points_run(x, y, pp, qq, dx, dy, F, F, 0.05, 30)
    assert pot_rel_err(u.cpu(), ref["u"], 0.05) < 1e-11
    assert pot_rel_err(v.cpu(), ref["v"], 0.05) < 1e-11


# ---------------------------------------------------------------------------
# regular grids (separable passes), 1-D / 2-D / 3-D, ragged extents
# ---------------------------------------------------------------------------
def grid_case(rng, shape, dtype):
    npd = np.float32 if dtype == torch.float32 else np.float64
    size = int(np.prod(shape))
    h = tuple(1.0 / n for n in shape)
    p = rounded(rng.uniform(0.2, 2.0, size), npd)
    q = rounded(rng.uniform(0.2, 2.0, size), npd)
    d = rounded(np.full(size, float(np.prod(h))), npd)
    return h, p, q, d


@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("shape", [(300,), (37, 29), (9, 11, 7), (260, 3)])
def test_grid_all_divergences_fixed_iterations(dtype, tolr, shape):
    rng = np.random.default_rng(len(shape) * 7 + shape[0])
    h, p, q, d = grid_case(rng, shape, dtype)
    eps = 0.01
    G = O.GridGeom(shape, h)
    for F in DIVS:
        say("case grid", shape, dtype, F)
        prob = U.grid_problem(shape, h, T(p, dtype), T(q, dtype), T(d, dtype), T(d, dtype), F, F)
        u, v, info = U.solve(prob, eps, tol=0.0, max_iter=20)
        ref = O.solve(G, np.log(p), np.log(q), np.log(d), np.log(d), oracle_div(F), oracle_div(F), eps, tol=0.0,
                      max_iter=20)
        assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr, F
        assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr, F


def test_grid_eps_scaling_to_tolerance():
    """64 x 64 blob images, KL lambda = 0.1, eps annealed 1e-1 -> 1e-3 (10
    stages of 100 iterations), FP32, iterate to residual 1e-6."""
    pr = synth.blobs2d(1, n=64)
    shape, h = pr.shape, pr.h
    npd = np.float32
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    d = rounded(np.full(pr.size, h[0] * h[1]), npd)
    F = U.KL(0.1)
    say("case grid eps-scaling 64x64")
    prob = U.grid_problem(shape, h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                          T(d, torch.float32), F, F)
    u, v, info = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-6, max_iter=4000)
    ref = O.solve(O.GridGeom(shape, h), np.log(p), np.log(q), np.log(d), np.log(d), O.KL(0.1), O.KL(0.1), 1e-3,
                  tol=1e-6, max_iter=4000, eps0=1e-1)
    assert info["converged"] and ref["converged"]
    assert abs(info["iters"] - ref["iters"]) <= max(3, ref["iters"] // 100)
    # each side stops on its own residual: element-wise parity is with the
    # oracle run for the iterations the GPU took, the converged oracle is a
    # few residuals away
    same = O.solve(O.GridGeom(shape, h), np.log(p), np.log(q), np.log(d), np.log(d), O.KL(0.1), O.KL(0.1), 1e-3,
                   tol=0.0, max_iter=int(info["iters"]), eps0=1e-1)
    assert pot_rel_err(u.cpu(), same["u"], 1e-3) < 1e-5
    assert pot_rel_err(v.cpu(), same["v"], 1e-3) < 1e-5
    assert pot_rel_err(u.cpu(), ref["u"], 1e-3) < 5e-5
    assert pot_rel_err(v.cpu(), ref["v"], 1e-3) < 5e-5


def test_grid_half_step_full_size_256():
    """One X half-step on the 256 x 256 workload, from an identical state."""
    pr = synth.blobs2d(0, n=256)
    npd = np.float32
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    d = rounded(np.full(pr.size, pr.h[0] * pr.h[1]), npd)
    rng = np.random.default_rng(9)
    vstate = rounded(0.05 * rng.standard_normal(pr.size), npd)
    ustate = rounded(0.05 * rng.standard_normal(pr.size), npd)
    eps = 1e-3
    for F in (U.KL(0.1), U.TV(0.05)):
        say("case grid half-step 256x256", F)
        prob = U.grid_problem(pr.shape, pr.h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                              T(d, torch.float32), F, F)
        G = O.GridGeom(pr.shape, pr.h)
        # u_old near the update so that r is a moderate number
        Sr, ur, _ = O.half_step_x(G, np.log(p), np.log(d), np.log(d), oracle_div(F), eps, ustate, vstate)
        ustate = rounded(ur + 1e-5 * rng.standard_normal(pr.size), npd)
        rr = O.marginal_residual(Sr, ustate, ur, np.log(d), eps)
        un, S, r = U.half_step(prob, eps, 0, T(vstate, torch.float32), T(ustate, torch.float32))
        # S is a log of sums of up to 65536 terms: FP32 relative accuracy on |S|
        assert np.max(np.abs(S.cpu().numpy() - Sr)) / np.max(np.abs(Sr)) < 2e-6
        assert pot_rel_err(un.cpu(), ur, eps) < 1e-5
        assert r == pytest.approx(rr, rel=1e-2)


def test_dense_half_step_full_size_20000():
    """One X half-step of the 20000 x 20000 3-D point-cloud workload from an
    identical state; the oracle evaluates all rows in FP64 (chunked)."""
    pr = synth.clouds3d(0)
    npd = np.float32
    x, y = rounded(pr.x, npd), rounded(pr.y, npd)
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    dx, dy = rounded(pr.dx, npd), rounded(pr.dy, npd)
    rng = np.random.default_rng(10)
    vstate = rounded(0.02 * rng.standard_normal(len(q)), npd)
    ustate = rounded(0.02 * rng.standard_normal(len(p)), npd)
    eps = 1e-3
    F = U.KL(1.0)
    say("case dense half-step 20000^2")
    prob = gpu_points(x, y, p, q, dx, dy, F, F, torch.float32)
    w = vstate / eps + np.log(dy)
    Sr = np.empty(len(p))
    for a in range(0, len(p), 1000):
        C = O.sq_dist(x[a:a + 1000], y)
        Sr[a:a + 1000] = O.lse(-C / eps + w[None, :], axis=1)
    ur = eps * O.proxdiv_log(O.KL(1.0), np.log(p), Sr, 0.0, eps)
    ustate = rounded(ur + 1e-5 * rng.standard_normal(len(p)), npd)   # near the update: moderate r
    un, S, r = U.half_step(prob, eps, 0, T(vstate, torch.float32), T(ustate, torch.float32))
    S = S.cpu().numpy()
    un = un.cpu().numpy()
    assert np.max(np.abs(S - Sr)) / np.max(np.abs(Sr)) < 2e-6
    assert pot_rel_err(un, ur, eps) < 1e-5
    rr = O.marginal_residual(Sr, ustate, ur, np.log(dx), eps)
    assert r == pytest.approx(rr, rel=1e-2)


def test_dense_eps_scaling_solve_fp32():
    """3-D clouds (N = 500, M = 400 from the mixture recipe), KL lambda = 1,
    eps-scaling 1 -> 1e-2, residual 1e-6."""
    pr = synth.clouds3d(1, N=500, M=400)
    npd = np.float32
    x, y = rounded(pr.x, npd), rounded(pr.y, npd)
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    dx, dy = rounded(pr.dx, npd), rounded(pr.dy, npd)
    F = U.KL(1.0)
    say("case dense eps-scaling 500x400")
    prob = gpu_points(x, y, p, q, dx, dy, F, F, torch.float32)
    u, v, info = U.solve(prob, 1e-2, eps0=1.0, tol=1e-6, max_iter=6000)
    ref = oracle_points_run(x, y, p, q, dx, dy, F, F, 1e-2, 6000, tol=1e-6, eps0=1.0)
    assert info["converged"] and ref["converged"]
    assert abs(info["iters"] - ref["iters"]) <= max(3, ref["iters"] // 100)
    same = oracle_points_run(x, y, p, q, dx, dy, F, F, 1e-2, int(info["iters"]), tol=0.0, eps0=1.0)
    assert pot_rel_err(u.cpu(), same["u"], 1e-2) < 1e-5
    assert pot_rel_err(v.cpu(), same["v"], 1e-2) < 1e-5
    assert pot_rel_err(u.cpu(), ref["u"], 1e-2) < 5e-5
    assert pot_rel_err(v.cpu(), ref["v"], 1e-2) < 5e-5


# ---------------------------------------------------------------------------
# objective (FP64 reductions) at the oracle's converged potentials
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("geom", ["points", "grid"])
@pytest.mark.parametrize("F", [U.KL(0.4), U.TV(0.1)])
def test_objective_parity(geom, F):
    rng = np.random.default_rng(77)
    eps = 0.02
    dtype = torch.float64
    if geom == "points":
        x, y, p, q, dx, dy = points_case(rng, 120, 95, 2, dtype)
        g = O.PointsGeom(x, y)
        prob = gpu_points(x, y, p, q, dx, dy, F, F, dtype)
    else:
        shape = (24, 19)
        h, p, q, dx = grid_case(rng, shape, dtype)
        dy = dx
        g = O.GridGeom(shape, h)
        prob = U.grid_problem(shape, h, T(p, dtype), T(q, dtype), T(dx, dtype), T(dy, dtype), F, F)
    say("case objective", geom, F)
    s = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), oracle_div(F), oracle_div(F), eps, tol=1e-13,
                max_iter=200000)
    ref = O.objective(g, p, q, dx, dy, oracle_div(F), oracle_div(F), eps, s["u"], s["v"])
    got = U.objective(prob, eps, T(s["u"], dtype), T(s["v"], dtype), marginals=True)
    for k in ("primal", "dual", "transport_cost"):
        assert got[k] == pytest.approx(ref[k], rel=1e-10, abs=1e-13), k
    assert got["mass1"] == pytest.approx(ref["mass"], rel=1e-10)
    assert got["massK"] == pytest.approx(ref["mK"], rel=1e-10)
    assert abs(got["gap"] - ref["gap"]) < 1e-10
    np.testing.assert_allclose(got["pi1"].cpu().numpy(), ref["pi1"], rtol=1e-10)
    np.testing.assert_allclose(got["pi2"].cpu().numpy(), ref["pi2"], rtol=1e-10)


# ---------------------------------------------------------------------------
# barycentres
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("F2", [U.KL(0.5), U.EQ(), U.TV(0.1), U.RG(0.7, 1.3)])
def test_barycenter_fixed_iterations(dtype, tolr, F2):
    npd = np.float32 if dtype == torch.float32 else np.float64
    rng = np.random.default_rng(55)
    shape = (26, 21)
    size = 26 * 21
    h = (1 / 26, 1 / 21)
    n = 3
    p = rounded(rng.uniform(0.3, 1.6, (n, size)), npd)
    if F2.kind == U.UOT_DIV_EQ:
        p *= (1.0 / p.mean(axis=1))[:, None]
        p = rounded(p, npd)
    alpha = np.array([0.2, 0.5, 0.3])
    d = rounded(np.full(size, h[0] * h[1]), npd)
    eps = 0.01
    F1 = U.KL(0.5)
    say("case barycentre", dtype, F2)
    u, v, logh, info = U.barycenter(shape, h, T(p, dtype), alpha, T(d, dtype), T(d, dtype), F1, F2, eps, tol=0.0,
                                    max_iter=30)
    ref = O.barycenter(O.GridGeom(shape, h), np.log(p), alpha, np.log(d), np.log(d), oracle_div(F1), oracle_div(F2),
                       eps, tol=0.0, max_iter=30)
    assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr
    assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr
    assert np.max(np.abs(logh.cpu().numpy() - ref["logh"])) / np.max(np.abs(ref["logh"])) < tolr * 10


# ---------------------------------------------------------------------------
# driver semantics: graphs, resume, status
# ---------------------------------------------------------------------------
def test_graph_replay_matches_direct_launches_and_resume():
    rng = np.random.default_rng(12)
    shape = (48, 40)
    h, p, q, d = grid_case(rng, shape, torch.float32)
    F = U.KL(0.3)
    prob = U.grid_problem(shape, h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32), T(d, torch.float32),
                          F, F)
    say("case graph vs direct")
    u1, v1, i1 = U.solve(prob, 5e-3, eps0=0.5, iters_per_stage=7, tol=0.0, max_iter=137, use_graph=True, check_every=16)
    u2, v2, i2 = U.solve(prob, 5e-3, eps0=0.5, iters_per_stage=7, tol=0.0, max_iter=137, use_graph=False, check_every=5)
    assert i1["iters"] == i2["iters"] == 137
    assert torch.equal(u1, u2) and torch.equal(v1, v2)
    # checkpoint / resume: 60 + 40 iterations from v equal 100 straight (no annealing)
    ua, va, _ = U.solve(prob, 5e-3, tol=0.0, max_iter=100)
    _, vb, _ = U.solve(prob, 5e-3, tol=0.0, max_iter=60)
    uc, vc, _ = U.solve(prob, 5e-3, tol=0.0, max_iter=40, v0=vb)
    assert torch.equal(ua, uc) and torch.equal(va, vc)


def test_not_converged_status_and_validation_errors():
    rng = np.random.default_rng(13)
    h, p, q, d = grid_case(rng, (16, 16), torch.float32)
    F = U.KL(0.3)
    prob = U.grid_problem((16, 16), h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                          T(d, torch.float32), F, F)
    say("case status")
    u, v, info = U.solve(prob, 1e-3, tol=1e-12, max_iter=3)
    assert info["status"] == U.UOT_NOT_CONVERGED and info["iters"] == 3 and not info["converged"]
    with pytest.raises(U.UotError):
        U.solve(prob, -1.0, tol=1e-6, max_iter=3)


# ---------------------------------------------------------------------------
# tile-factored MFMA grid passes (FP32)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(64,), (48, 32), (48, 29), (16, 32, 16)])
def test_grid_mfma_passes_fixed_iterations(shape):
    rng = np.random.default_rng(91 + shape[0])
    h, p, q, d = grid_case(rng, shape, torch.float32)
    eps = 0.01
    G = O.GridGeom(shape, h)
    for F in (U.KL(0.5), U.TV(0.1)):
        say("case grid mfma", shape, F)
        prob = U.grid_problem(shape, h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                              T(d, torch.float32), F, F)
        u, v, info = U.solve(prob, eps, tol=0.0, max_iter=20, grid_kernel=U.GRID_MFMA)
        ref = O.solve(G, np.log(p), np.log(q), np.log(d), np.log(d), oracle_div(F), oracle_div(F), eps, tol=0.0,
                      max_iter=20)
        assert pot_rel_err(u.cpu(), ref["u"], eps) < 1e-5, F
        assert pot_rel_err(v.cpu(), ref["v"], eps) < 1e-5, F


def test_grid_mfma_solve_256_matches_direct_and_oracle_residual():
    """The 256 x 256 workload (KL 0.1, eps 1e-1 -> 1e-3, residual 1e-6) with
    MFMA passes: same potentials as the direct passes to FP32 tolerance, and
    the oracle's residual at the returned state is at the tolerance."""
    pr = synth.blobs2d(0, n=256)
    npd = np.float32
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    d = rounded(np.full(pr.size, pr.h[0] * pr.h[1]), npd)
    F = U.KL(0.1)
    say("case grid mfma 256")
    prob = U.grid_problem(pr.shape, pr.h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                          T(d, torch.float32), F, F)
    u1, v1, i1 = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-6, max_iter=5000, grid_kernel=U.GRID_DIRECT)
    u2, v2, i2 = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-6, max_iter=5000, grid_kernel=U.GRID_MFMA)
    assert i1["converged"] and i2["converged"]
    assert abs(i1["iters"] - i2["iters"]) <= 10
    assert pot_rel_err(u2.cpu(), u1.cpu().numpy().astype(np.float64), 1e-3) < 1e-5
    G = O.GridGeom(pr.shape, pr.h)
    _, _, r = O.half_step_x(G, np.log(p), np.log(d), np.log(d), O.KL(0.1), 1e-3,
                            u2.cpu().numpy().astype(np.float64), v2.cpu().numpy().astype(np.float64))
    assert r < 5e-6, r


# ---------------------------------------------------------------------------
# tile-factored MFMA grid passes with FP16 operands (grid_kernel 3): FP16
# rounding of Khat and of the column factors (2^-11 relative) bounds them at
# 1e-3 relative on potentials, the tolerance of the half-precision paths
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("shape", [(64,), (48, 32), (48, 29), (16, 32, 16)])
def test_grid_mfma16_passes_fixed_iterations(shape):
    rng = np.random.default_rng(191 + shape[0])
    h, p, q, d = grid_case(rng, shape, torch.float32)
    eps = 0.01
    G = O.GridGeom(shape, h)
    for F in (U.KL(0.5), U.TV(0.1)):
        say("case grid mfma16", shape, F)
        prob = U.grid_problem(shape, h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                              T(d, torch.float32), F, F)
        u, v, info = U.solve(prob, eps, tol=0.0, max_iter=20, grid_kernel=U.GRID_MFMA16)
        ref = O.solve(G, np.log(p), np.log(q), np.log(d), np.log(d), oracle_div(F), oracle_div(F), eps, tol=0.0,
                      max_iter=20)
        eu = pot_rel_err(u.cpu(), ref["u"], eps)
        ev = pot_rel_err(v.cpu(), ref["v"], eps)
        assert eu < 1e-3 and ev < 1e-3, (F, eu, ev)
        # where an axis takes the FP16 pass, the error shows it (above the FP32
        # paths' level, far below the tolerance)
        if any(n % 16 == 0 and (1.0 / n) ** 2 * math.log2(math.e) / eps <= 0.125 for n in shape):
            assert max(eu, ev) > 1e-7


def test_grid_mfma16_solve_256_and_barycentre():
    """The 256 x 256 workload (KL 0.1, eps 1e-1 -> 1e-3) and a 128 x 128
    barycentre of 8 images with FP16 operands.  Rounding the operands to FP16
    every iteration leaves a residual floor far above the FP32 paths' (the
    map moves by single FP16 roundings between iterations), so these solves
    run to residual 1e-4, and agree with the FP32 MFMA solves (residual 1e-6)
    to 1e-3."""
    pr = synth.blobs2d(0, n=256)
    npd = np.float32
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    d = rounded(np.full(pr.size, pr.h[0] * pr.h[1]), npd)
    F = U.KL(0.1)
    say("case grid mfma16 256")
    prob = U.grid_problem(pr.shape, pr.h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                          T(d, torch.float32), F, F)
    u1, v1, i1 = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-6, max_iter=5000, grid_kernel=U.GRID_MFMA)
    u2, v2, i2 = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-4, max_iter=5000, grid_kernel=U.GRID_MFMA16, record=True)
    hist = i2["res_hist"].numpy()
    say("fp16 residual after %d iterations: %.2e (min of the last 200: %.2e)" % (i2["iters"], i2["residual"],
                                                                                 hist[-200:].min()))
    assert i1["converged"] and i2["converged"]
    assert pot_rel_err(u2.cpu(), u1.cpu().numpy().astype(np.float64), 1e-3) < 1e-3
    assert pot_rel_err(v2.cpu(), v1.cpu().numpy().astype(np.float64), 1e-3) < 1e-3
    say("case barycentre mfma16 128")
    bp = synth.bary_blobs(0, n_marg=8, n=128)
    pb = T(bp.p, torch.float32)
    hb = (1.0 / 128, 1.0 / 128)
    db = torch.full((128 * 128,), hb[0] * hb[1], dtype=torch.float32, device=DEV)
    Fb = U.KL(0.5)
    _, vb1, lh1, ib1 = U.barycenter((128, 128), hb, pb, bp.alpha, db, db, Fb, Fb, 2e-3, eps0=1e-1, tol=1e-6,
                                    max_iter=6000, grid_kernel=U.GRID_MFMA)
    _, vb2, lh2, ib2 = U.barycenter((128, 128), hb, pb, bp.alpha, db, db, Fb, Fb, 2e-3, eps0=1e-1, tol=1e-4,
                                    max_iter=6000, grid_kernel=U.GRID_MFMA16)
    assert ib1["converged"] and ib2["converged"]
    assert pot_rel_err(lh2.cpu(), lh1.cpu().numpy().astype(np.float64), 1.0) < 1e-3


def test_grid_mixed_precision_reaches_fp32_accuracy():
    """grid_kernel 4: FP16 passes down to residual 1e-4, FP32 passes after.
    The solve reaches residual 1e-6 and lands on the FP32 fixed point (1e-5,
    the FP32 tolerance), on the 256 x 256 workload and a 128 x 128
    barycentre of 8 images; the residual history continues across the
    switch."""
    pr = synth.blobs2d(0, n=256)
    npd = np.float32
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    d = rounded(np.full(pr.size, pr.h[0] * pr.h[1]), npd)
    for F in (U.KL(0.1), U.TV(0.05)):
        say("case grid mixed 256", F)
        prob = U.grid_problem(pr.shape, pr.h, T(p, torch.float32), T(q, torch.float32), T(d, torch.float32),
                              T(d, torch.float32), F, F)
        u1, v1, i1 = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-6, max_iter=5000, grid_kernel=U.GRID_MFMA)
        u2, v2, i2 = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-6, max_iter=5000, grid_kernel=U.GRID_MIXED, record=True)
        assert i1["converged"] and i2["converged"] and i2["residual"] <= 1e-6
        assert abs(i1["iters"] - i2["iters"]) <= 50, (i1["iters"], i2["iters"])
        hist = i2["res_hist"].numpy()
        assert np.all(np.isfinite(hist)) and hist[-1] <= 1e-6
        assert pot_rel_err(u2.cpu(), u1.cpu().numpy().astype(np.float64), 1e-3) < 1e-5
        assert pot_rel_err(v2.cpu(), v1.cpu().numpy().astype(np.float64), 1e-3) < 1e-5
    say("case barycentre mixed 128")
    bp = synth.bary_blobs(0, n_marg=8, n=128)
    pb = T(bp.p, torch.float32)
    hb = (1.0 / 128, 1.0 / 128)
    db = torch.full((128 * 128,), hb[0] * hb[1], dtype=torch.float32, device=DEV)
    Fb = U.KL(0.5)
    _, _, lh1, ib1 = U.barycenter((128, 128), hb, pb, bp.alpha, db, db, Fb, Fb, 2e-3, eps0=1e-1, tol=1e-6,
                                  max_iter=6000, grid_kernel=U.GRID_MFMA)
    _, _, lh2, ib2 = U.barycenter((128, 128), hb, pb, bp.alpha, db, db, Fb, Fb, 2e-3, eps0=1e-1, tol=1e-6,
                                  max_iter=6000, grid_kernel=U.GRID_MIXED)
    assert ib1["converged"] and ib2["converged"]
    assert pot_rel_err(lh2.cpu(), lh1.cpu().numpy().astype(np.float64), 1.0) < 1e-5


# ---------------------------------------------------------------------------
# Algorithm 4: a function F3 of the total mass
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("F3", [U.EQ(), U.KL(0.3), U.RG(0.5, 0.8)])
def test_mass_penalty_fixed_iterations(dtype, tolr, F3):
    rng = np.random.default_rng(81)
    x, y, p, q, dx, dy = points_case(rng, 300, 260, 2, dtype)
    eps, mass = 0.02, 0.6
    F1, F2 = U.KL(0.5), U.TV(0.2)
    say("case mass points", dtype, F3)
    prob = gpu_points(x, y, p, q, dx, dy, F1, F2, dtype)
    u, v, lz, info = U.solve_mass(prob, F3, mass, eps, tol=0.0, max_iter=25)
    g = O.PointsGeom(x, y)
    ref = O.solve_mass(g, O.safe_log(p), O.safe_log(q), np.log(dx), np.log(dy), oracle_div(F1), oracle_div(F2),
                       oracle_div(F3), np.log(mass), eps, tol=0.0, max_iter=25)
    assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr
    assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr
    assert lz == pytest.approx(ref["zeta"], rel=tolr * 10, abs=tolr)
    # the same on a grid (separable passes; FP32 uses the MFMA passes)
    rng = np.random.default_rng(83)
    shape = (48, 32)
    h, pg, qg, dg = grid_case(rng, shape, dtype)
    say("case mass grid", dtype, F3)
    pgp = U.grid_problem(shape, h, T(pg, dtype), T(qg, dtype), T(dg, dtype), T(dg, dtype), F1, F2)
    u, v, lz, info = U.solve_mass(pgp, F3, mass, eps, tol=0.0, max_iter=25)
    G = O.GridGeom(shape, h)
    ref = O.solve_mass(G, np.log(pg), np.log(qg), np.log(dg), np.log(dg), oracle_div(F1), oracle_div(F2),
                       oracle_div(F3), np.log(mass), eps, tol=0.0, max_iter=25)
    assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr
    assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr
    assert lz == pytest.approx(ref["zeta"], rel=tolr * 10, abs=tolr)


def test_mass_penalty_free_mass_and_partial_transport():
    """F3 = 0 on the nonnegative reals leaves z = 1 (the plain solve); partial
    transport (dominations RG[0, 1], total mass fixed) converges on the GPU
    to the oracle's solution, with the mass and the dominations held."""
    rng = np.random.default_rng(85)
    x, y, p, q, dx, dy = points_case(rng, 200, 180, 2, torch.float64)
    eps = 0.02
    F = U.KL(0.4)
    prob = gpu_points(x, y, p, q, dx, dy, F, F, torch.float64)
    say("case mass free")
    u1, v1, lz, i1 = U.solve_mass(prob, U.RG(0.0, math.inf), 1.0, eps, tol=1e-10, max_iter=20000)
    u2, v2, i2 = U.solve(prob, eps, tol=1e-10, max_iter=20000)
    assert lz == 0.0 and i1["iters"] == i2["iters"]
    assert torch.equal(u1, u2) and torch.equal(v1, v2)
    say("case partial transport")
    dom = U.RG(0.0, 1.0)
    pd = gpu_points(x, y, p, q, dx, dy, dom, dom, torch.float64)
    m0 = 0.5 * min(float(np.sum(p * dx)), float(np.sum(q * dy)))
    u, v, lz, info = U.solve_mass(pd, U.EQ(), m0, eps, tol=1e-10, max_iter=50000)
    assert info["converged"]
    g = O.PointsGeom(x, y)
    ref = O.solve_mass(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.RG(0.0, 1.0), O.RG(0.0, 1.0), O.EQ,
                       np.log(m0), eps, tol=1e-10, max_iter=50000)
    assert info["iters"] == ref["iters"]
    assert pot_rel_err(u.cpu(), ref["u"], eps) < 1e-9
    assert lz == pytest.approx(ref["zeta"], rel=1e-9)
    C = O.sq_dist(x, y)
    R = np.exp((u.cpu().numpy()[:, None] + v.cpu().numpy()[None, :] - C) / eps + lz)
    assert np.sum(R * dx[:, None] * dy[None, :]) == pytest.approx(m0, rel=1e-8)
    assert np.all(R @ dy <= p * (1 + 1e-8)) and np.all(R.T @ dx <= q * (1 + 1e-8))


# ---------------------------------------------------------------------------
# sup-norm of the potential change (Thm. convergenceKL), reduced on the device
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_du_inf_matches_oracle(dtype):
    """info["du_inf"] = max_i |u_i^K - u_i^(K-1)| of the last iteration
    against the oracle's recorded iterates: point clouds (KL 0.5, 30
    iterations) and a grid (TV 0.1 and KL 0.5, 25 iterations).  Each GPU
    potential is within the parity tolerance of the oracle's (1e-11 FP64,
    1e-5 FP32 of max(|u|, eps)), so their difference is within twice that;
    the reduction rounds du_inf once to FP32 (2^-24 relative, the FP64 paths
    included).  With zero densities the first iteration moves those
    potentials from 0 to -inf: du_inf is +inf there and finite afterwards."""
    tol = 2e-11 if dtype == torch.float64 else 2e-5
    rng = np.random.default_rng(41)
    x, y, p, q, dx, dy = points_case(rng, 300, 257, 2, dtype)
    F = U.KL(0.5)
    eps = 0.02
    say("case du_inf clouds", dtype)
    prob = gpu_points(x, y, p, q, dx, dy, F, F, dtype)
    _, _, info = U.solve(prob, eps, tol=0.0, max_iter=30)
    ref = oracle_points_run(x, y, p, q, dx, dy, F, F, eps, 30, record=True)
    u29, u30 = ref["hist"][-2][0], ref["hist"][-1][0]
    d_ref = float(np.max(np.abs(u30 - u29)))
    scale = max(float(np.max(np.abs(u30))), eps)
    assert abs(info["du_inf"] - d_ref) <= tol * scale + 2.0 ** -23 * d_ref, (info["du_inf"], d_ref)
    assert d_ref > 100 * tol * scale        # the comparison is not vacuous
    # (40, 33): direct passes; (48, 32): tile-factored passes in FP32 (their
    # first Y pass hosts the control step)
    for shape in ((40, 33), (48, 32)):
        h, pg, qg, dg = grid_case(rng, shape, dtype)
        G = O.GridGeom(shape, h)
        for Fg in (U.TV(0.1), U.KL(0.5)):
            say("case du_inf grid", dtype, shape, Fg)
            prob = U.grid_problem(shape, h, T(pg, dtype), T(qg, dtype), T(dg, dtype), T(dg, dtype), Fg, Fg)
            _, _, info = U.solve(prob, 0.01, tol=0.0, max_iter=25)
            ref = O.solve(G, np.log(pg), np.log(qg), np.log(dg), np.log(dg), oracle_div(Fg), oracle_div(Fg), 0.01,
                          tol=0.0, max_iter=25, record=True)
            d_ref = float(np.max(np.abs(ref["hist"][-1][0] - ref["hist"][-2][0])))
            scale = max(float(np.max(np.abs(ref["u"]))), 0.01)
            assert abs(info["du_inf"] - d_ref) <= tol * scale + 2.0 ** -23 * d_ref, (Fg, info["du_inf"], d_ref)
    # zero densities: -inf potentials appear at the first iteration only
    pz = p.copy()
    pz[[5, 9]] = 0.0
    prob = gpu_points(x, y, pz, q, dx, dy, F, F, dtype)
    _, _, info1 = U.solve(prob, eps, tol=0.0, max_iter=1)
    _, _, info2 = U.solve(prob, eps, tol=0.0, max_iter=4)
    assert info1["du_inf"] == math.inf and math.isfinite(info2["du_inf"])
