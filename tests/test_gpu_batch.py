"""Ragged batched solves vs the FP64 oracle, problem by problem, through the C
ABI.  Every problem of the batch is compared with an independent oracle solve
of that problem alone."""
import sys

import numpy as np
import pytest
import torch

from oracle import uot_oracle as O
from tests.helpers import pot_rel_err, rounded

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import uot as U  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_batch(seed, B, lo, hi, d, npd, extra=()):
    rng = np.random.default_rng(seed)
    Ns = list(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), B))).astype(int)) + [e[0] for e in extra]
    Ms = list(np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), B))).astype(int)) + [e[1] for e in extra]
    probs = []
    for n, m in zip(Ns, Ms):
        x = rounded(rng.uniform(0, 1, (n, d)), npd)
        y = rounded(rng.uniform(0, 1, (m, d)), npd)
        p = rounded(rng.uniform(0.1, 1.0, n), npd)
        q = rounded(rng.uniform(0.1, 1.0, m), npd)
        dx = rounded(np.full(n, 1.0 / n), npd)
        dy = rounded(np.full(m, 1.0 / m), npd)
        probs.append((x, y, p, q, dx, dy))
    return Ns, Ms, probs


def to_gpu(Ns, Ms, probs, F1, F2, dtype):
    cat = lambda k: torch.tensor(np.concatenate([pp[k] for pp in probs]), dtype=dtype, device=DEV)
    return U.BatchProblem(Ns, Ms, cat(0), cat(1), cat(2), cat(3), cat(4), cat(5), F1, F2)


def split(t, off):
    a = t.cpu().numpy()
    return [a[off[b]:off[b + 1]] for b in range(len(off) - 1)]


@pytest.mark.parametrize("dtype,tolr,kern", [(torch.float32, 1e-5, 1), (torch.float32, 1e-5, 4),
                                             (torch.float64, 1e-11, 0)])
def test_batch_fixed_iterations_every_problem(dtype, tolr, kern):
    """dense_kernel 1 / 4 pins the batch tuner to the direct or the
    matrix-core product (problems in Morton order on the device)."""
    npd = np.float32 if dtype == torch.float32 else np.float64
    Ns, Ms, probs = make_batch(3, 29, 20, 700, 2, npd, extra=[(1, 1), (1, 300), (513, 2)])
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, dtype)
    eps = 0.05
    say("case batch fixed", dtype, "B", bp.B, "kernel", kern)
    u, v, info = U.solve_batched(bp, eps, tol=0.0, max_iter=30, dense_kernel=kern)
    assert (info["iters"] == 30).all()
    if kern:
        assert info["product"] == kern
    us, vs = split(u, bp.offN), split(v, bp.offM)
    for b, (x, y, p, q, dx, dy) in enumerate(probs):
        ref = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), eps,
                      tol=0.0, max_iter=30)
        assert pot_rel_err(us[b], ref["u"], eps) < tolr, (b, Ns[b], Ms[b])
        assert pot_rel_err(vs[b], ref["v"], eps) < tolr, (b, Ns[b], Ms[b])


@pytest.mark.parametrize("kern", [0, 4])
def test_batch_converged_each_problem_stops_on_its_own(kern):
    npd = np.float32
    Ns, Ms, probs = make_batch(5, 24, 40, 900, 2, npd)
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    eps = 0.02
    say("case batch converged", kern)
    u, v, info = U.solve_batched(bp, eps, tol=1e-6, max_iter=4000, check_every=32, dense_kernel=kern)
    assert info["converged"] and info["n_converged"] == bp.B
    assert info["tile_rows"] in (256, 512, 1024) and info["blocks_per_cu"] in (4, 8, 16)
    # the matrix-core product gets no more persistent blocks than a compute
    # unit holds at once (4 with 256 rows per item, 2 with 512: then 4)
    if info["product"] == 4:
        assert info["blocks_per_cu"] == 4, info["blocks_per_cu"]
    us, vs = split(u, bp.offN), split(v, bp.offM)
    lat = info["latency_ms"]
    assert np.all(lat > 0)
    its = info["iters"]
    # a problem that needed more iterations cannot have stopped earlier
    order = np.argsort(its)
    assert np.all(np.diff(lat[order]) >= -1e-3)
    for b, (x, y, p, q, dx, dy) in enumerate(probs):
        ref = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), eps,
                      tol=1e-6, max_iter=4000)
        assert abs(int(its[b]) - ref["iters"]) <= max(2, ref["iters"] // 50), (b, its[b], ref["iters"])
        # the two sides stop on their own residual (FP32 here, FP64 in the
        # oracle), a few iterations apart: the element-wise comparison is with
        # the oracle run for exactly the iterations this problem took; the
        # converged oracle solution is only a few residuals away
        same = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0),
                       eps, tol=0.0, max_iter=int(its[b]))
        assert pot_rel_err(us[b], same["u"], eps) < 1e-5, (b, its[b])
        assert pot_rel_err(vs[b], same["v"], eps) < 1e-5, (b, its[b])
        assert pot_rel_err(us[b], ref["u"], eps) < 5e-5
        assert pot_rel_err(vs[b], ref["v"], eps) < 5e-5
    # second call with the same signature reuses the tuned choice; graph and
    # direct launches give identical potentials
    u2, v2, info2 = U.solve_batched(bp, eps, tol=1e-6, max_iter=4000, check_every=32, use_graph=False,
                                    dense_kernel=kern)
    assert info2["tune_ms"] == 0.0
    assert torch.equal(u, u2) and torch.equal(v, v2)
    assert np.array_equal(info2["iters"], its)


def test_batch_matrix_core_large_problem_order():
    """A batch holding a problem above 4096 points (Morton order by counting
    ranks instead of the in-LDS sort) next to small ones: the matrix-core
    product (dense_kernel 4) against the direct one (1), whose parity with
    the oracle the tests above pin."""
    npd = np.float32
    Ns, Ms, probs = make_batch(9, 6, 30, 600, 2, npd, extra=[(5000, 4500)])
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    eps = 0.05
    say("case batch large problem order")
    u1, v1, _ = U.solve_batched(bp, eps, tol=0.0, max_iter=20, dense_kernel=1)
    u4, v4, info = U.solve_batched(bp, eps, tol=0.0, max_iter=20, dense_kernel=4)
    assert info["product"] == 4
    for a, b, off in ((u4, u1, bp.offN), (v4, v1, bp.offM)):
        for x, y in zip(split(a, off), split(b, off)):
            assert pot_rel_err(x, y, eps) < 1e-5



def line_problem(rng, N, M, f32=np.float32):
    """1-D rows in [0.45, 0.55], columns uniform on [0, 1]."""
    x = rounded((0.45 + 0.1 * rng.random(N))[:, None], f32)
    y = rounded(rng.random((M, 1)), f32)
    return (x, y, rounded(rng.random(N) + 0.5, f32), rounded(rng.random(M) + 0.5, f32),
            rounded(np.full(N, 1.0 / N), f32), rounded(np.full(M, 1.0 / M), f32))


def joint_errs(bp, pots1, pots2):
    """Per problem: largest potential difference, and the larger of the two
    reference potentials' magnitudes."""
    (u1, v1), (u2, v2) = pots1, pots2
    U1, V1, U2, V2 = (split(t, off) for t, off in ((u1, bp.offN), (v1, bp.offM), (u2, bp.offN), (v2, bp.offM)))
    return [(max(np.abs(U2[b] - U1[b]).max(), np.abs(V2[b] - V1[b]).max()),
             max(np.abs(U1[b]).max(), np.abs(V1[b]).max())) for b in range(bp.B)]


def test_batch_matrix_core_running_max_jumps():
    """The batched matrix-core product carries a running row maximum from
    chunk to chunk of 256 columns, starting cold in a solve's first product:
    rows in [0.45, 0.55], columns uniform on [0, 1], eps = 1e-5, so left of
    the rows every chunk's exponents exceed the running maximum by hundreds
    of powers of two and right of them fall as far below it (3000 x 20000,
    next to 200 x 1500 and 50 x 700).  Against the direct product after 2
    iterations, relative to the larger of the two potentials' magnitudes
    (after the first iteration far pairs' terms are differences of numbers
    of order 1/eps, so u is small against the rounding of those terms)."""
    rng = np.random.default_rng(21)
    Ns, Ms = [200, 3000, 50], [1500, 20000, 700]
    probs = [line_problem(rng, n, m) for n, m in zip(Ns, Ms)]
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    say("case batch running max jumps")
    u1, v1, _ = U.solve_batched(bp, 1e-5, tol=0.0, max_iter=2, dense_kernel=1)
    u4, v4, info = U.solve_batched(bp, 1e-5, tol=0.0, max_iter=2, dense_kernel=4)
    assert info["product"] == 4
    for b, (err, scale) in enumerate(joint_errs(bp, (u1, v1), (u4, v4))):
        assert err / scale < 1e-5, (b, err / scale)


def test_batch_matrix_core_error_model():
    """The matrix-core product's exponent passes through FP32 intermediates
    of size c r^2 (r: the half-diagonal of the rows' bounding box around the
    block centre, c = 1 / (eps ln 2)), so its potentials carry an absolute
    error of a few 2^-24 r^2 whatever eps and the potentials' size, where the
    direct product's error scales with the potentials.  Uniform 1-D problems
    (one item spans a whole problem: r = 1/2) at eps = 1e-5, where the
    potentials (~1e-4) are far below r^2: the difference from the direct
    product stays within 8 * 2^-24 * r^2 after 2 iterations."""
    npd = np.float32
    Ns, Ms, probs = make_batch(4, 6, 40, 300, 1, npd)
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    say("case batch matrix-core error model")
    u1, v1, _ = U.solve_batched(bp, 1e-5, tol=0.0, max_iter=2, dense_kernel=1)
    u4, v4, _ = U.solve_batched(bp, 1e-5, tol=0.0, max_iter=2, dense_kernel=4)
    for b, (err, scale) in enumerate(joint_errs(bp, (u1, v1), (u4, v4))):
        x = probs[b][0]
        r2 = float(((x.max(0) - x.min(0)) / 2).astype(np.float64) @ ((x.max(0) - x.min(0)) / 2))
        assert err <= 8 * 2.0 ** -24 * r2, (b, err, r2)


def test_batch_matrix_core_converged_bench_eps():
    """The batch benchmark's setting (2-D uniform points, KL 1, eps 5e-3,
    tol 1e-6) with the matrix-core product: each problem converged, compared
    with the oracle run for the iterations it took.  The shape of the
    potentials (each minus its mean) meets the FP32 bar 1e-5.  Their common
    level carries the FP32 rounding of every iteration in the slowest mode:
    a few 2^-24 of S's log2 size L enter u as theta eps ln2 per half-step and
    the constant direction contracts only by theta^2 per iteration
    (Thm. convergenceKL's rate for KL on both sides, theta = lam/(lam+eps)),
    so it collects up to 4 2^-24 L theta eps ln2 / (1 - theta^2)."""
    npd = np.float32
    Ns, Ms, probs = make_batch(6, 8, 64, 400, 2, npd)
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    eps = 5e-3
    say("case batch converged bench eps")
    u, v, info = U.solve_batched(bp, eps, tol=1e-6, max_iter=4000, check_every=32, dense_kernel=4)
    assert info["converged"] and info["product"] == 4
    us, vs = split(u, bp.offN), split(v, bp.offM)
    its = info["iters"]
    th = 1.0 / (1.0 + eps)
    for b, (x, y, p, q, dx, dy) in enumerate(probs):
        same = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0),
                       eps, tol=0.0, max_iter=int(its[b]))
        L = float(np.max(np.abs(same["S"]))) / np.log(2.0)
        level = 4 * 2.0 ** -24 * L * th * eps * np.log(2.0) / (1 - th * th)
        for got, ref in ((us[b], same["u"]), (vs[b], same["v"])):
            got = np.asarray(got, np.float64)
            shape = pot_rel_err(got - got.mean(), ref - ref.mean(), eps)
            assert shape < 1e-5, (b, its[b], shape)
            assert abs(got.mean() - ref.mean()) <= level, (b, its[b], got.mean() - ref.mean(), level)
            assert pot_rel_err(got, ref, eps) < 1e-5 + level / max(np.abs(ref).max(), eps), (b, its[b])


def test_tuning_table_round_trip():
    """The tuners' choices move to a new context as text: the batch solve
    there skips tuning, takes the same choice and gives the same potentials;
    a matrix-core dense solve adds its block target; tables that name a
    choice the tuners do not make are refused whole."""
    npd = np.float32
    Ns, Ms, probs = make_batch(11, 16, 40, 600, 2, npd)
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    say("case tuning table round trip")
    c1, c2 = U.Context(), U.Context()
    u1, v1, i1 = U.solve_batched(bp, 0.05, ctx=c1, tol=0.0, max_iter=20)
    assert i1["tune_ms"] > 0.0
    rng = np.random.default_rng(2)
    n, m = 2048, 2560   # two shapes: one block target per side
    T = lambda a: torch.tensor(a, dtype=torch.float32, device=DEV)
    pb = U.points_problem(T(rng.uniform(0, 1, (n, 2))), T(rng.uniform(0, 1, (m, 2))), T(np.full(n, 1.0)),
                          T(np.full(m, 1.0)), T(np.full(n, 1.0 / n)), T(np.full(m, 1.0 / m)), F, F)
    U.solve(pb, 0.05, ctx=c1, tol=0.0, max_iter=4, dense_kernel=4)
    text = U.export_tuning(c1)
    lines = [l.split() for l in text.splitlines()]
    assert sum(l[0] == "batch" for l in lines) == 1 and sum(l[0] == "dense" for l in lines) == 2, text
    batch_line = [l for l in lines if l[0] == "batch"][0]
    assert int(batch_line[2]) == i1["product"] and int(batch_line[4]) == i1["blocks_per_cu"]
    assert int(batch_line[3]) * 256 == i1["tile_rows"]
    for bad in ("batch sig 3 1 4\n", "batch sig 4 4 8\n", "batch sig 1 1 5\n", "dense k 999\n", "dense k\n",
                "other a 1\n", "batch sig 1 1 4 extra\n"):
        with pytest.raises(U.UotError):
            U.import_tuning(text + bad, c2)
    assert U.export_tuning(c2) == ""
    U.import_tuning("\n" + text + "\n", c2)
    assert U.export_tuning(c2) == text
    u2, v2, i2 = U.solve_batched(bp, 0.05, ctx=c2, tol=0.0, max_iter=20)
    assert i2["tune_ms"] == 0.0
    assert (i2["product"], i2["tile_rows"], i2["blocks_per_cu"]) == (i1["product"], i1["tile_rows"],
                                                                      i1["blocks_per_cu"])
    assert torch.equal(u1, u2) and torch.equal(v1, v2)
    c1.close()
    c2.close()


@pytest.mark.parametrize("dtype,tolr,kern", [(torch.float32, 1e-5, 1), (torch.float32, 1e-5, 4),
                                             (torch.float64, 1e-11, 1)])
def test_batch_rebalance_matches_oracle(dtype, tolr, kern):
    """The in-solve mass balance (rebalance_at = 9) against the oracle's, problem
    by problem, for a fixed 24 iterations from a random start (so the shift is
    large): the X and Y mass partials, the per-problem shift in the control
    step and the moved potentials and column weights all enter."""
    npd = np.float32 if dtype == torch.float32 else np.float64
    Ns, Ms, probs = make_batch(41, 25, 20, 700, 2, npd, extra=[(1, 3), (300, 1), (513, 257)])
    F1, F2 = U.KL(0.7), U.KL(1.3)
    bp = to_gpu(Ns, Ms, probs, F1, F2, dtype)
    eps = 0.04
    rng = np.random.default_rng(42)
    v0 = [rounded(rng.normal(0.0, 0.3, m), npd) for m in Ms]
    say("case batch rebalance", dtype, kern)
    u, v, info = U.solve_batched(bp, eps, v0=torch.tensor(np.concatenate(v0), dtype=dtype, device=DEV), tol=0.0,
                                 max_iter=24, dense_kernel=kern, rebalance_at=9)
    # a problem with a single point on one side is solved exactly by the
    # balance (its constant is the only freedom there): its residual reaches
    # 0 <= tol and it stops; the others run the 24 iterations
    its = info["iters"]
    assert (its == 24).sum() >= len(probs) - 2 and (its > 9).all()
    us, vs = split(u, bp.offN), split(v, bp.offM)
    moved = 0
    for b, (x, y, p, q, dx, dy) in enumerate(probs):
        args = (O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(0.7), O.KL(1.3), eps)
        ref = O.solve(*args, tol=-1.0, max_iter=int(its[b]), v0=v0[b], rebalance_at=9)
        plain = O.solve(*args, tol=-1.0, max_iter=int(its[b]), v0=v0[b])
        assert pot_rel_err(us[b], ref["u"], eps) < tolr, (b, Ns[b], Ms[b])
        assert pot_rel_err(vs[b], ref["v"], eps) < tolr, (b, Ns[b], Ms[b])
        moved += pot_rel_err(plain["v"], ref["v"], eps) > 100 * tolr
    assert moved >= len(probs) // 2


@pytest.mark.parametrize("kern", [1, 4])
def test_batch_rebalance_converged_fewer_iterations(kern):
    """Converged solves with the balance at the start and again at iteration
    30: every problem stops within a few iterations of the oracle's own
    rebalanced solve, at the oracle's potentials, and in fewer iterations than
    without the second balance."""
    npd = np.float32
    Ns, Ms, probs = make_batch(43, 16, 40, 600, 2, npd)
    F = U.KL(1.0)
    bp = to_gpu(Ns, Ms, probs, F, F, torch.float32)
    eps = 0.02   # (the matrix-core product's FP32 error model holds 1e-5 here)
    say("case batch rebalance converged", kern)
    v0 = torch.zeros(bp.totM, dtype=torch.float32, device=DEV)
    U.batch_balance(bp, eps, v0)
    kw = dict(tol=1e-6, max_iter=20000, check_every=32, dense_kernel=kern)
    u, v, info = U.solve_batched(bp, eps, v0=v0.clone(), rebalance_at=30, **kw)
    _, _, once = U.solve_batched(bp, eps, v0=v0.clone(), **kw)
    assert info["converged"] and info["n_converged"] == bp.B
    assert info["iters"].sum() < 0.85 * once["iters"].sum()
    us, vs = split(u, bp.offN), split(v, bp.offM)
    v0s = split(v0, bp.offM)
    for b, (x, y, p, q, dx, dy) in enumerate(probs):
        args = (O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), eps)
        ref = O.solve(*args, tol=1e-6, max_iter=20000, v0=v0s[b], rebalance_at=30)
        its = int(info["iters"][b])
        assert abs(its - ref["iters"]) <= max(2, ref["iters"] // 50), (b, its, ref["iters"])
        same = O.solve(*args, tol=0.0, max_iter=its, v0=v0s[b], rebalance_at=30)
        assert pot_rel_err(us[b], same["u"], eps) < 1e-5, (b, its)
        assert pot_rel_err(vs[b], same["v"], eps) < 1e-5, (b, its)


def test_rebalance_argument_checks():
    npd = np.float32
    Ns, Ms, probs = make_batch(44, 3, 20, 60, 2, npd)
    bp = to_gpu(Ns, Ms, probs, U.KL(1.0), U.TV(0.5), torch.float32)
    with pytest.raises(U.UotError):
        U.solve_batched(bp, 0.05, tol=0.0, max_iter=5, rebalance_at=3)     # TV: no closed form
    bp = to_gpu(Ns, Ms, probs, U.KL(1.0), U.KL(1.0), torch.float32)
    with pytest.raises(U.UotError):
        U.solve_batched(bp, 0.05, tol=0.0, max_iter=5, rebalance_at=1)     # the start takes uot_batch_balance
    x, y, p, q, dx, dy = probs[0]
    T = lambda a: torch.tensor(a, dtype=torch.float32, device=DEV)
    pb = U.points_problem(T(x), T(y), T(p), T(q), T(dx), T(dy), U.KL(1.0), U.KL(1.0))
    with pytest.raises(U.UotError):
        U.solve(pb, 0.05, tol=0.0, max_iter=5, rebalance_at=3)            # batches only
