"""HIP path vs the FP64 oracle for the WF cost with a cut locus (dense point
clouds with tile skipping, banded 1-D grid passes, FP64 objective), the growth
divergence and the gradient flows of Sec. 5.3 (heat, crowd projection, WF
growth with one and two species), element by element on the same seeded
inputs, through the C ABI.  Tolerances: FP64 1e-10 relative on potentials and
densities; FP32 1e-5 on potentials, and on densities (e^{T + v/eps}) 1e-4
relative to their maximum (one FP32 rounding of v/eps is 6e-8 |v|/eps)."""
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


def npd_of(dtype):
    return np.float64 if dtype == torch.float64 else np.float32


def dens_rel_err(gpu, ref):
    a = np.asarray(gpu, np.float64)
    b = np.asarray(ref, np.float64)
    assert a.shape == b.shape and not np.isnan(a).any()
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def split_inf(gpu, ref):
    """Entries that are +inf in the oracle (a vanishing product under KL) must
    be +inf on the GPU too; the rest is returned for the usual metric."""
    a = np.asarray(gpu, np.float64)
    b = np.asarray(ref, np.float64)
    assert np.array_equal(np.isposinf(a), np.isposinf(b)), "+inf pattern differs"
    keep = ~np.isposinf(b)
    return a[keep], b[keep]


# ---------------------------------------------------------------------------
# WF cost: dense point clouds (tile skipping) and 1-D grids (banded passes)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("d", [1, 2, 3])
def test_wf_points_fixed_iterations(dtype, tolr, d):
    """Clustered clouds in Morton order (N = 1100, M = 900: several row blocks,
    column splits and a ragged tail), cut 0.15: many tiles are skipped."""
    npd = npd_of(dtype)
    cp = synth.clusters_sorted(3 + d, N=1100, M=900, d=d)
    x, y = rounded(cp.x, npd), rounded(cp.y, npd)
    p, q, dx, dy = (rounded(a, npd) for a in (cp.p, cp.q, cp.dx, cp.dy))
    cut, eps = 0.15, 0.01
    F = U.KL(0.5)
    say("case wf points", dtype, d)
    prob = U.points_problem(T(x, dtype), T(y, dtype), T(p, dtype), T(q, dtype), T(dx, dtype), T(dy, dtype), F, F,
                            cost=U.WF(cut))
    u, v, info = U.solve(prob, eps, tol=0.0, max_iter=30)
    g = O.PointsGeom(x, y, "wf", cut)
    ref = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(0.5), O.KL(0.5), eps, tol=0.0, max_iter=30)
    assert pot_rel_err(*split_inf(u.cpu(), ref["u"]), eps) < tolr
    assert pot_rel_err(*split_inf(v.cpu(), ref["v"]), eps) < tolr


@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
def test_wf_points_order_and_isolated_points(dtype, tolr):
    """The same clouds shuffled give the same potentials (permuted), and points
    with no partner within the cut carry +inf potentials and no mass."""
    npd = npd_of(dtype)
    rng = np.random.default_rng(11)
    cp = synth.clusters_sorted(5, N=800, M=700, d=2)
    x = np.vstack([cp.x, [[0.99, 0.01], [0.01, 0.99]]])       # far from every cluster
    p = np.r_[cp.p, 1.0, 1.2]
    x, y = rounded(x, npd), rounded(cp.y, npd)
    p, q = rounded(p, npd), rounded(cp.q, npd)
    dx, dy = rounded(np.full(len(p), 1.0 / len(p)), npd), rounded(cp.dy, npd)
    cut, eps = 0.1, 0.02
    F = U.KL(1.0)
    g = O.PointsGeom(x, y, "wf", cut)
    assert np.isinf(g.C[-2:]).all()
    ref = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), eps, tol=0.0, max_iter=20)
    assert np.isposinf(ref["u"][-2:]).all()
    say("case wf isolated", dtype)
    prob = U.points_problem(T(x, dtype), T(y, dtype), T(p, dtype), T(q, dtype), T(dx, dtype), T(dy, dtype), F, F,
                            cost=U.WF(cut))
    u, v, info = U.solve(prob, eps, tol=0.0, max_iter=20)
    assert np.isfinite(info["residual"])
    assert pot_rel_err(*split_inf(u.cpu(), ref["u"]), eps) < tolr
    assert pot_rel_err(*split_inf(v.cpu(), ref["v"]), eps) < tolr
    # shuffled storage: same potentials up to the permutation
    pi, pj = rng.permutation(len(p)), rng.permutation(len(q))
    prob2 = U.points_problem(T(x[pi], dtype), T(y[pj], dtype), T(p[pi], dtype), T(q[pj], dtype), T(dx[pi], dtype),
                             T(dy[pj], dtype), F, F, cost=U.WF(cut))
    u2, v2, _ = U.solve(prob2, eps, tol=0.0, max_iter=20)
    assert pot_rel_err(*split_inf(u2.cpu().numpy()[np.argsort(pi)], ref["u"]), eps) < tolr
    assert pot_rel_err(*split_inf(v2.cpu().numpy()[np.argsort(pj)], ref["v"]), eps) < tolr


@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
def test_wf_points_block_flags_many_splits(dtype, tolr):
    """The (row block, column split) flags: 600 clustered rows in [0, 0.6]^2
    plus 300 rows in [0.9, 1]^2 beyond the cut (0.3) of every column (the
    last block of 256 rows has no partner at all: +inf potentials), against
    40000 clustered columns in [0, 0.6]^2.  The X products run 1250 splits
    of 32 columns, past the merge's LDS list (its per-split flag loop), the
    Y products 29 splits (the list)."""
    npd = npd_of(dtype)
    rng = np.random.default_rng(17)
    cx = synth.clusters_sorted(8, N=600, M=40000, d=2)
    far = 0.9 + 0.1 * rng.random((300, 2))
    x = rounded(np.vstack([0.6 * cx.x, far]), npd)
    y = rounded(0.6 * cx.y, npd)
    p = rounded(np.r_[cx.p, 0.5 + rng.random(300)], npd)
    q = rounded(cx.q, npd)
    dx, dy = rounded(np.full(900, 1.0 / 900), npd), rounded(np.full(40000, 1.0 / 40000), npd)
    cut, eps = 0.3, 0.02
    F = U.KL(1.0)
    say("case wf block flags", dtype)
    prob = U.points_problem(T(x, dtype), T(y, dtype), T(p, dtype), T(q, dtype), T(dx, dtype), T(dy, dtype), F, F,
                            cost=U.WF(cut))
    u, v, _ = U.solve(prob, eps, tol=0.0, max_iter=6)
    g = O.PointsGeom(x, y, "wf", cut)
    ref = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), eps, tol=0.0, max_iter=6)
    assert np.isposinf(ref["u"][768:]).all()
    assert pot_rel_err(*split_inf(u.cpu(), ref["u"]), eps) < tolr
    assert pot_rel_err(*split_inf(v.cpu(), ref["v"]), eps) < tolr


@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
@pytest.mark.parametrize("n,cut", [(700, 0.05), (700, math.pi / 2), (300, 0.3)])
def test_wf_grid_1d(dtype, tolr, n, cut):
    """1-D grid passes with the WF cost: band of ceil(cut / h) cells (the
    whole line for the unscaled cost pi/2 > 1)."""
    npd = npd_of(dtype)
    pr = synth.hist1d(2, n=n)
    p, q = rounded(pr.p, npd), rounded(pr.q, npd)
    d = rounded(np.full(n, pr.h[0]), npd)
    eps = 1e-3
    F = U.KL(0.5)
    say("case wf grid", dtype, n, cut)
    prob = U.grid_problem(pr.shape, pr.h, T(p, dtype), T(q, dtype), T(d, dtype), T(d, dtype), F, F,
                          cost=U.WF(cut))
    u, v, info = U.solve(prob, eps, tol=0.0, max_iter=40)
    g = O.GridGeom(pr.shape, pr.h, "wf", cut)
    ref = O.solve(g, np.log(p), np.log(q), np.log(d), np.log(d), O.KL(0.5), O.KL(0.5), eps, tol=0.0, max_iter=40)
    assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr
    assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr


@pytest.mark.parametrize("F", [U.KL(0.1), U.TV(0.05)])
def test_wf_grid_1d_eps_scaling_converged(F):
    n = 256
    pr = synth.hist1d(4, n=n)
    p, q = pr.p, pr.q
    d = np.full(n, pr.h[0])
    say("case wf grid converged", F)
    prob = U.grid_problem(pr.shape, pr.h, T(p, torch.float64), T(q, torch.float64), T(d, torch.float64),
                          T(d, torch.float64), F, F, cost=U.WF(0.2))
    u, v, info = U.solve(prob, 1e-3, eps0=1e-1, tol=1e-9, max_iter=8000)
    g = O.GridGeom(pr.shape, pr.h, "wf", 0.2)
    ref = O.solve(g, np.log(p), np.log(q), np.log(d), np.log(d), oracle_div(F), oracle_div(F), 1e-3, tol=1e-9,
                  max_iter=8000, eps0=1e-1)
    assert info["converged"] and ref["converged"]
    assert abs(info["iters"] - ref["iters"]) <= 1
    assert pot_rel_err(u.cpu(), ref["u"], 1e-3) < 1e-8
    assert pot_rel_err(v.cpu(), ref["v"], 1e-3) < 1e-8


@pytest.mark.parametrize("geom", ["points", "grid"])
def test_wf_objective(geom):
    """FP64 objective with the WF cost (transport cost with +inf entries that
    carry no mass) at the oracle's converged potentials."""
    eps = 0.01
    F = U.KL(0.7)
    if geom == "points":
        cp = synth.clusters_sorted(7, N=600, M=500, d=2)
        x, y, p, q, dx, dy = cp.x, cp.y, cp.p, cp.q, cp.dx, cp.dy
        g = O.PointsGeom(x, y, "wf", 0.2)
        prob = U.points_problem(T(x, torch.float64), T(y, torch.float64), T(p, torch.float64), T(q, torch.float64),
                                T(dx, torch.float64), T(dy, torch.float64), F, F, cost=U.WF(0.2))
    else:
        pr = synth.hist1d(5, n=400)
        p, q = pr.p, pr.q
        dx = dy = np.full(400, pr.h[0])
        g = O.GridGeom(pr.shape, pr.h, "wf", 0.2)
        prob = U.grid_problem(pr.shape, pr.h, T(p, torch.float64), T(q, torch.float64), T(dx, torch.float64),
                              T(dy, torch.float64), F, F, cost=U.WF(0.2))
    ref = O.solve(g, np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(0.7), O.KL(0.7), eps, tol=1e-12,
                  max_iter=20000)
    say("case wf objective", geom)
    got = U.objective(prob, eps, T(ref["u"], torch.float64), T(ref["v"], torch.float64))
    want = O.objective(g, p, q, dx, dy, O.KL(0.7), O.KL(0.7), eps, ref["u"], ref["v"])
    for k_got, k_ref in (("primal", "primal"), ("dual", "dual"), ("transport_cost", "transport_cost"),
                         ("mass1", "mass"), ("mass2", "mass2"), ("massK", "mK")):
        assert got[k_got] == pytest.approx(want[k_ref], rel=1e-10), k_got
    assert got["gap"] == pytest.approx(want["gap"], abs=1e-10)


# ---------------------------------------------------------------------------
# growth divergence in a plain solve, and its objective
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("dtype,tolr", [(torch.float64, 1e-11), (torch.float32, 1e-5)])
def test_growth_divergence_solve_and_objective(dtype, tolr):
    npd = npd_of(dtype)
    n = 600
    p0 = rounded(synth.growth_profile_1d(1, n)[0], npd)
    cap = rounded(np.ones(n), npd)
    d = rounded(np.full(n, 1.0 / n), npd)
    lam, eps = 0.1, 2e-3
    say("case growth div", dtype)
    prob = U.grid_problem((n,), (1.0 / n,), T(p0, dtype), T(cap, dtype), T(d, dtype), T(d, dtype), U.KL(1.0),
                          U.GROWTH(lam), cost=U.WF(0.3))
    u, v, info = U.solve(prob, eps, tol=0.0, max_iter=50)
    g = O.GridGeom((n,), (1.0 / n,), "wf", 0.3)
    ref = O.solve(g, np.log(p0), np.log(cap), np.log(d), np.log(d), O.KL(1.0), O.GROWTH(lam), eps, tol=0.0,
                  max_iter=50)
    assert pot_rel_err(u.cpu(), ref["u"], eps) < tolr
    assert pot_rel_err(v.cpu(), ref["v"], eps) < tolr
    if dtype == torch.float64:
        got = U.objective(prob, eps, u, v)
        want = O.objective(g, p0, cap, d, d, O.KL(1.0), O.GROWTH(lam), eps, ref["u"], ref["v"])
        for k in ("primal", "dual"):
            assert got[k] == pytest.approx(want[k], rel=1e-10), k
        assert got["gap"] == pytest.approx(want["gap"], rel=1e-8, abs=1e-12)


# ---------------------------------------------------------------------------
# gradient flows
# ---------------------------------------------------------------------------
def run_flow_both(kind, dtype, p0, q, n_steps, iters, eps, tau, alpha=0.0, shape=None, h=None, x=None,
                  cost=U.SQEUCLID, tol=0.0):
    npd = npd_of(dtype)
    p0 = rounded(np.atleast_2d(p0), npd)
    q = rounded(q, npd)
    N = q.size
    if shape is not None:
        dxv = rounded(np.full(N, float(np.prod(h))), npd)
        g = O.GridGeom(shape, h, "wf" if cost.kind == U.UOT_COST_WF else "sqeuclid", cost.cut or None)
    else:
        x = rounded(x, npd)
        dxv = rounded(np.full(N, 1.0 / N), npd)
        g = O.PointsGeom(x, x, "wf" if cost.kind == U.UOT_COST_WF else "sqeuclid", cost.cut or None)
    dens, v, steps, info = U.flow(kind, T(p0, dtype), T(q, dtype), T(dxv, dtype), tau, eps, n_steps, shape=shape,
                                  h=h, x=None if x is None else T(x, dtype), alpha=alpha, cost=cost, tol=tol,
                                  max_iter=iters, check_every=20)
    ref, rinfo = O.flow(g, kind, p0, q, dxv, tau, eps, n_steps, iters, alpha=alpha, tol=tol)
    return dens.cpu().numpy(), v.cpu().numpy(), steps, ref, rinfo


@pytest.mark.parametrize("dtype,tol_d", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
@pytest.mark.parametrize("cut", [math.pi / 2, 0.2])
def test_flow_growth_one_species(dtype, tol_d, cut):
    """WF growth flow (tumour example): tau = 0.006, alpha = 1 as in the paper,
    on 300 cells, 3 steps of 120 iterations."""
    n = 300
    p0 = synth.growth_profile_1d(0, n)
    say("case flow growth 1", dtype, cut)
    dens, v, steps, ref, rinfo = run_flow_both("growth", dtype, p0, np.ones(n), 3, 120, 1e-2, 0.006, alpha=1.0,
                                               shape=(n,), h=(1.0 / n,), cost=U.WF(cut))
    assert [s["iters"] for s in steps] == [i["iters"] for i in rinfo]
    for k in range(4):
        assert dens_rel_err(dens[k], ref[k]) < tol_d, k
    assert dens[-1].max() <= 1.0 + 1e-5


@pytest.mark.parametrize("dtype,tol_d", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_flow_growth_two_species(dtype, tol_d):
    n = 256
    p0 = synth.growth_profile_1d(3, n, species=2)
    say("case flow growth 2", dtype)
    dens, v, steps, ref, rinfo = run_flow_both("growth", dtype, p0, np.ones(n), 3, 100, 1e-2, 0.004, alpha=1.0,
                                               shape=(n,), h=(1.0 / n,), cost=U.WF(math.pi / 2))
    for k in range(4):
        assert dens_rel_err(dens[k], ref[k]) < tol_d, k
    assert np.allclose(v[0], v[1])
    assert dens[-1].sum(axis=0).max() <= 1.0 + 1e-5


@pytest.mark.parametrize("dtype,tol_d", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
@pytest.mark.parametrize("kind", ["heat", "crowd"])
def test_flow_heat_and_crowd_grids(dtype, tol_d, kind):
    """1-D (400 cells) and 2-D (48 x 48, tile-factored passes in FP32) grids."""
    for shape in ((400,), (48, 48)):
        N = int(np.prod(shape))
        h = tuple(1.0 / s for s in shape)
        gp = synth.blobs2d(1, n=48) if len(shape) == 2 else synth.hist1d(1, n=400)
        p0 = gp.p / gp.p.max() * (2.0 if kind == "crowd" else 1.0)
        q = np.ones(N)
        say("case flow", kind, dtype, shape)
        dens, v, steps, ref, rinfo = run_flow_both(kind, dtype, p0, q, 2, 80, 2e-3, 1e-3, shape=shape, h=h)
        for k in range(3):
            assert dens_rel_err(dens[k], ref[k]) < tol_d, (shape, k)


@pytest.mark.parametrize("dtype,tol_d", [(torch.float64, 1e-10), (torch.float32, 1e-4)])
def test_flow_points_and_convergence(dtype, tol_d):
    """Heat flow on one point cloud (X = Y, dense passes), run to tolerance:
    the iteration counts match the oracle's."""
    cp = synth.clusters_sorted(9, N=500, M=10, d=2)
    x = cp.x
    p0 = np.exp(-((x[:, 0] - 0.4) ** 2 + (x[:, 1] - 0.5) ** 2) / 0.02) + 0.05
    say("case flow points", dtype)
    dens, v, steps, ref, rinfo = run_flow_both("heat", dtype, p0, np.ones(500), 2, 3000, 1e-2, 2e-3, x=x,
                                               tol=1e-7 if dtype == torch.float64 else 1e-5)
    for s, r in zip(steps, rinfo):
        assert s["status"] == 0 and r["converged"]
        assert abs(s["iters"] - r["iters"]) <= 2
    for k in range(3):
        assert dens_rel_err(dens[k], ref[k]) < (tol_d if dtype == torch.float32 else 1e-7), k
    assert abs(dens[-1].sum() - dens[0].sum()) / dens[0].sum() < 1e-5
