"""The asynchronous calls of the boundary (uot_solve_async / uot_sync_result):
the enqueued iteration, with its no-op chunks after the stop, must leave
exactly the potentials, iteration count, residual and status of uot_solve
(bitwise: the same kernels run on the same data, and a stopped iteration
changes nothing), on a grid and on point clouds through the matrix-core
product (Morton-ordered copies, potentials scattered back), FP32 and FP64;
and a context with a pending solve refuses other calls until the result is
collected."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import synth  # noqa: E402
from paper_1607_05816_amd import uot as U  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grid(dtype):
    pr = synth.blobs2d(3, n=64)
    T = lambda a: torch.tensor(np.asarray(a), dtype=dtype, device=DEV)
    d = T(np.full(pr.size, pr.h[0] * pr.h[1]))
    return U.grid_problem(pr.shape, pr.h, T(pr.p), T(pr.q), d, d, U.KL(0.1), U.KL(0.1))


def clouds(dtype):
    pr = synth.uniform_clouds(np.random.default_rng(5), 2500, 2300)
    T = lambda a: torch.tensor(np.asarray(a), dtype=dtype, device=DEV)
    return U.points_problem(T(pr.x), T(pr.y), T(pr.p), T(pr.q), T(pr.dx), T(pr.dy), U.KL(1.0), U.KL(1.0),
                            layout="nd")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("make,eps,kw", [(grid, 1e-3, dict(eps0=1e-1)), (clouds, 2e-2, {})])
def test_async_solve_matches_solve(make, eps, kw, dtype):
    prob = make(dtype)
    ctx = U.Context()
    say("case async", make.__name__, dtype)
    u, v, info = U.solve(prob, eps, ctx=ctx, tol=1e-6, max_iter=3000, check_every=50, **kw)
    assert info["converged"]
    pend = U.solve_async(prob, eps, ctx=ctx, tol=1e-6, max_iter=3000, check_every=50, **kw)
    got = pend.result()
    assert got["converged"] and got["iters"] == info["iters"] and got["status"] == info["status"]
    assert got["residual"] == info["residual"] and got["du_inf"] == info["du_inf"]
    assert torch.equal(pend.u, u) and torch.equal(pend.v, v)
    assert got["elapsed_ms"] > 0
    # a fixed iteration count (tol = 0): every enqueued iteration runs
    pend = U.solve_async(prob, eps, ctx=ctx, tol=0.0, max_iter=120, check_every=50, **kw)
    u2, v2, i2 = U.solve(prob, eps, ctx=U.Context(), tol=0.0, max_iter=120, check_every=50, **kw)
    got = pend.result()
    assert got["iters"] == 120 and not got["converged"] and i2["iters"] == 120
    assert torch.equal(pend.u, u2) and torch.equal(pend.v, v2)


def test_pending_solve_blocks_the_context():
    prob = grid(torch.float32)
    ctx = U.Context()
    say("case async pending")
    pend = U.solve_async(prob, 1e-2, ctx=ctx, tol=1e-6, max_iter=400, check_every=40)
    with pytest.raises(U.UotError) as e:
        U.solve(prob, 1e-2, ctx=ctx, tol=1e-6, max_iter=400)
    assert e.value.code == U.UOT_E_INVALID
    info = pend.result()
    assert info["iters"] > 0
    assert pend.result() is info                       # collected once
    res = U.UotResult()
    assert U.lib().uot_sync_result(ctx.handle, res) == U.UOT_E_INVALID   # nothing pending
    U.solve(prob, 1e-2, ctx=ctx, tol=1e-6, max_iter=400)                 # the context works again
