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
