"""The factored dense products against the FP64 oracle and against the direct
product, FP32: dense_kernel 2 (Morton-ordered copies, tile pairs factored
exactly, wide pairs summed directly; inputs are given in random order, the
library orders them itself and returns potentials in the caller's order) and
dense_kernels 3 and 4 (exponents of 16 x 16 pairs as one MFMA product around
a centre per block of rows: FP32 operands, or operands split into three bf16
parts).  Tolerance 1e-5 relative on potentials (FP32)."""
import sys

import numpy as np
import pytest
import torch

from oracle import uot_oracle as O
from paper_1607_05816_amd import synth
from tests.helpers import pot_rel_err, rounded

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import uot as U  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def T(a):
    return torch.tensor(np.asarray(a), dtype=torch.float32, device=DEV)


def mixture(seed, N, M, d):
    pr = synth.clouds3d(seed, N=N, M=M)
    x, y = pr.x[:, :d], pr.y[:, :d]
    return (rounded(x, np.float32), rounded(y, np.float32), rounded(pr.p, np.float32), rounded(pr.q, np.float32),
            rounded(pr.dx, np.float32), rounded(pr.dy, np.float32))


KERNELS = [pytest.param(U.DENSE_TF, id="tf"), pytest.param(U.DENSE_MF, id="mfma"),
           pytest.param(U.DENSE_MF3, id="mfma_bf16x3")]


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("d", [1, 2, 3])
@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_dense_tf_fixed_iterations(d, eps, kern):
    """N = 3000, M = 2500 (ragged tails), KL 1; at eps = 1e-4 many tile pairs
    are too wide to factor and are summed directly (kernel 2)."""
    x, y, p, q, dx, dy = mixture(d, 3000, 2500, d)
    F = U.KL(1.0)
    say("case dense factored", kern, d, eps)
    prob = U.points_problem(T(x), T(y), T(p), T(q), T(dx), T(dy), F, F)
    u, v, info = U.solve(prob, eps, tol=0.0, max_iter=20, dense_kernel=kern)
    ref = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), eps,
                  tol=0.0, max_iter=20)
    assert pot_rel_err(u.cpu(), ref["u"], eps) < 1e-5
    assert pot_rel_err(v.cpu(), ref["v"], eps) < 1e-5


@pytest.mark.parametrize("kern", KERNELS)
def test_dense_tf_eps_scaling_and_residuals(kern):
    """eps-scaling 1e-1 -> 1e-3 with a warm start and the residual history:
    the factored run follows the oracle's iterates."""
    x, y, p, q, dx, dy = mixture(7, 1500, 1800, 3)
    F = U.TV(0.2)
    rng = np.random.default_rng(3)
    v0 = rounded(0.01 * rng.standard_normal(1800), np.float32)
    say("case dense factored eps-scaling", kern)
    prob = U.points_problem(T(x), T(y), T(p), T(q), T(dx), T(dy), F, F)
    u, v, info = U.solve(prob, 1e-3, eps0=1e-1, iters_per_stage=10, tol=0.0, max_iter=120, v0=T(v0),
                         dense_kernel=kern, record=True)
    ref = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.TV(0.2), O.TV(0.2), 1e-3,
                  tol=0.0, max_iter=120, eps0=1e-1, iters_per_stage=10, v0=v0)
    assert pot_rel_err(u.cpu(), ref["u"], 1e-3) < 1e-5
    assert pot_rel_err(v.cpu(), ref["v"], 1e-3) < 1e-5
    np.testing.assert_allclose(info["res_hist"].numpy()[1:], ref["res"][1:], rtol=1e-3, atol=1e-7)


@pytest.mark.parametrize("kern", KERNELS)
def test_dense_tf_matches_direct_full_size(kern):
    """N = M = 20000 3-D mixture clouds, eps = 1e-3, 40 iterations: the
    factored and the direct product give the same potentials."""
    pr = synth.clouds3d(0, N=20000, M=20000)
    F = U.KL(1.0)
    say("case dense factored full size", kern)
    prob = U.points_problem(T(pr.x), T(pr.y), T(pr.p), T(pr.q), T(pr.dx), T(pr.dy), F, F)
    u1, v1, _ = U.solve(prob, 1e-3, tol=0.0, max_iter=40, dense_kernel=U.DENSE_DIRECT)
    u2, v2, _ = U.solve(prob, 1e-3, tol=0.0, max_iter=40, dense_kernel=kern)
    assert pot_rel_err(u2.cpu(), u1.cpu().numpy(), 1e-3) < 1e-5
    assert pot_rel_err(v2.cpu(), v1.cpu().numpy(), 1e-3) < 1e-5


@pytest.mark.parametrize("kern", KERNELS)
@pytest.mark.parametrize("N,M", [(1, 1), (1, 37), (53, 1), (700, 513)])
def test_dense_factored_small_and_vanishing(N, M, kern):
    """Degenerate sizes (one row, one column, tails shorter than a tile) and
    zero densities on both sides (the vanishing-product rule: -inf potentials
    where the density is zero), KL 0.5, eps = 1e-2."""
    rng = np.random.default_rng(N * 1000 + M)
    x = rounded(rng.random((N, 2)), np.float32)
    y = rounded(rng.random((M, 2)), np.float32)
    p = rng.random(N) + 0.1
    q = rng.random(M) + 0.1
    if N > 1:
        p[::5] = 0.0
    if M > 1:
        q[1::4] = 0.0
    p, q = rounded(p, np.float32), rounded(q, np.float32)
    dx = rounded(np.full(N, 1.0 / N), np.float32)
    dy = rounded(np.full(M, 1.0 / M), np.float32)
    F = U.KL(0.5)
    say("case dense factored small", kern, N, M)
    prob = U.points_problem(T(x), T(y), T(p), T(q), T(dx), T(dy), F, F)
    u, v, info = U.solve(prob, 1e-2, tol=0.0, max_iter=15, dense_kernel=kern)
    ref = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(0.5), O.KL(0.5), 1e-2,
                  tol=0.0, max_iter=15)
    assert pot_rel_err(u.cpu(), ref["u"], 1e-2) < 1e-5
    assert pot_rel_err(v.cpu(), ref["v"], 1e-2) < 1e-5


def line_jumps(pattern, N, M, seed):
    """1-D clouds whose exponents, in the Morton (here: coordinate) order the
    matrix-core products sort the columns into, jump from chunk to chunk.
    'distance': rows in [0.45, 0.55], columns uniform on [0, 1], eps = 1e-5;
    one column step moves a far column's exponent by about a nat, so left of
    the rows each chunk's exponents exceed the running maximum by hundreds of
    powers of two (the lazy sum overflows and the chunk is redone with a
    maximum pass), right of them they fall as far below it.  'density':
    eps = 0.1, columns in alternating bands of width 0.02 (about 2000 sorted
    columns) with densities 1e-36 and O(1), so entering a dense band lifts
    the exponents by about 2^120: a finite lazy total above 2^100, which
    also triggers the redo.  Returns the problem arrays and eps."""
    rng = np.random.default_rng(seed)
    y = rng.random(M)
    if pattern == "distance":
        x, eps, q = 0.45 + 0.1 * rng.random(N), 1e-5, rng.random(M) + 0.5
    else:
        x, eps = rng.random(N), 1e-1
        q = np.where(np.floor(y * 50) % 2 == 0, 1e-36, rng.random(M) + 0.5)
    x, y = rounded(x[:, None], np.float32), rounded(y[:, None], np.float32)
    p = rounded(rng.random(N) + 0.5, np.float32)
    q = rounded(q, np.float32)
    dx = rounded(np.full(N, 1.0 / N), np.float32)
    dy = rounded(np.full(M, 1.0 / M), np.float32)
    return (x, y, p, q, dx, dy), eps


def joint_rel_err(u2, v2, u1, v1):
    """Largest difference relative to the larger of the two reference
    potentials' magnitudes: after the first iteration the terms of far pairs
    are differences of two numbers of order 1/eps, so each FP32 product errs
    by about 2^-24 of the larger potential, however small the other is."""
    u1, v1, u2, v2 = (t.cpu().numpy().astype(np.float64) for t in (u1, v1, u2, v2))
    scale = max(np.abs(u1).max(), np.abs(v1).max())
    return max(np.abs(u2 - u1).max(), np.abs(v2 - v1).max()) / scale


@pytest.mark.parametrize("kern", [pytest.param(U.DENSE_MF, id="mfma"), pytest.param(U.DENSE_MF3, id="mfma_bf16x3")])
@pytest.mark.parametrize("pattern", ["distance", "density"])
def test_dense_mf_running_max_jumps(pattern, kern):
    """Kernels 3 and 4 carry a running row maximum from chunk to chunk of 512
    columns, starting cold in a solve's first product.  N = 3000,
    M = 100000: a column split holds about 1200 columns, so splits that open
    with a chunk of low exponents and then meet high ones are many (the
    patterns are those of line_jumps).  Compared with the direct product,
    which the oracle parity tests pin, after 2 iterations."""
    (x, y, p, q, dx, dy), eps = line_jumps(pattern, 3000, 100000, 11)
    F = U.KL(1.0)
    say("case dense mf running max", pattern, kern)
    prob = U.points_problem(T(x), T(y), T(p), T(q), T(dx), T(dy), F, F)
    u1, v1, _ = U.solve(prob, eps, tol=0.0, max_iter=2, dense_kernel=U.DENSE_DIRECT)
    u2, v2, _ = U.solve(prob, eps, tol=0.0, max_iter=2, dense_kernel=kern)
    assert joint_rel_err(u2, v2, u1, v1) < 1e-5


@pytest.mark.parametrize("fill", ["random_bytes", "large_finite"])
def test_dense_mf_warm_maxima_any_workspace(fill):
    """Kernel 4 starts each product from the row maxima the previous product
    of the same side left in the workspace.  Whatever that memory holds
    (random bytes: NaN, inf, denormals; or finite values far above the true
    maxima), the result is that of the oracle: a start too low is caught by
    the overflow redo, one too high by the final-total check.  3-D mixture,
    N = 2000, M = 2300, KL 1, eps 1e-1 -> 1e-3, 30 iterations."""
    x, y, p, q, dx, dy = mixture(5, 2000, 2300, 3)
    F = U.KL(1.0)
    say("case dense mf warm maxima", fill)
    prob = U.points_problem(T(x), T(y), T(p), T(q), T(dx), T(dy), F, F)
    ws = prob.workspace()
    if fill == "random_bytes":
        ws.random_(0, 256)
    else:
        ws.view(torch.float32)[:] = 3.0e4
    u, v, _ = U.solve(prob, 1e-3, eps0=1e-1, iters_per_stage=5, tol=0.0, max_iter=30, dense_kernel=U.DENSE_MF3)
    ref = O.solve(O.PointsGeom(x, y), np.log(p), np.log(q), np.log(dx), np.log(dy), O.KL(1.0), O.KL(1.0), 1e-3,
                  tol=0.0, max_iter=30, eps0=1e-1, iters_per_stage=5)
    assert pot_rel_err(u.cpu(), ref["u"], 1e-3) < 1e-5
    assert pot_rel_err(v.cpu(), ref["v"], 1e-3) < 1e-5
