"""The no-allocation half-step (uot_half_step_noalloc) against uot_half_step
on the same inputs: two calls in a row, the second on a smaller problem, for
a grid and for point clouds, both half-steps.  The two entry points launch the
same kernels on the same inputs (only the workspace address differs), so the
potentials, the log-sum-exps and the residual agree to FP32 rounding (they
are in fact bit-equal).  A problem whose workspace exceeds the library's
scratch is rejected before anything runs."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import uot as U  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def grid_prob(rng, shape):
    size = int(np.prod(shape))
    h = tuple(1.0 / n for n in shape)
    T = lambda a: torch.tensor(a, dtype=torch.float32, device=DEV)
    p, q = T(rng.uniform(0.2, 2.0, size)), T(rng.uniform(0.2, 2.0, size))
    d = T(np.full(size, float(np.prod(h))))
    return U.grid_problem(shape, h, p, q, d, d, U.KL(0.5), U.KL(0.5))


def cloud_prob(rng, N, M):
    T = lambda a: torch.tensor(a, dtype=torch.float32, device=DEV)
    x, y = T(rng.uniform(0, 1, (N, 2))), T(rng.uniform(0, 1, (M, 2)))
    return U.points_problem(x, y, T(rng.uniform(0.1, 1, N)), T(rng.uniform(0.1, 1, M)),
                            T(np.full(N, 1.0 / N)), T(np.full(M, 1.0 / M)), U.KL(1.0), U.KL(1.0))


def compare(prob, eps, rng):
    for side in (0, 1):
        n_in, n_out = (prob.M, prob.N) if side == 0 else (prob.N, prob.M)
        pin = torch.tensor(rng.uniform(-0.05, 0.05, n_in), dtype=torch.float32, device=DEV)
        pold = torch.tensor(rng.uniform(-0.05, 0.05, n_out), dtype=torch.float32, device=DEV)
        a, sa, ra = U.half_step(prob, eps, side, pin, pold)
        b, sb, rb = U.half_step_noalloc(prob, eps, side, pin, pold)
        a, b, sa, sb = (t.cpu().numpy() for t in (a, b, sa, sb))
        np.testing.assert_allclose(b, a, rtol=1e-6, atol=1e-9 * np.max(np.abs(a)))
        np.testing.assert_allclose(sb, sa, rtol=1e-6, atol=1e-6)
        assert rb == pytest.approx(ra, rel=1e-6, abs=1e-12)
        say("   side %d: bit-equal %s" % (side, bool(np.array_equal(a, b) and np.array_equal(sa, sb) and ra == rb)))


def test_noalloc_half_step_matches_workspace_entry_point():
    rng = np.random.default_rng(17)
    for shape in ((96, 80), (40, 30)):
        say("case noalloc grid", shape)
        compare(grid_prob(rng, shape), 0.01, rng)
    for N, M in ((3000, 2500), (700, 500)):
        say("case noalloc clouds", N, M)
        compare(cloud_prob(rng, N, M), 5e-3, rng)


def test_noalloc_rejects_problems_beyond_the_scratch():
    rng = np.random.default_rng(18)
    prob = grid_prob(rng, (1024, 1024))      # 37 MB of half-step workspace > 32 MiB
    say("case noalloc too large")
    v = torch.zeros(prob.M, dtype=torch.float32, device=DEV)
    u = torch.zeros(prob.N, dtype=torch.float32, device=DEV)
    with pytest.raises(U.UotError, match="scratch"):
        U.half_step_noalloc(prob, 0.01, 0, v, u)
