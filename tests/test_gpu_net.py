"""GPU checks of the warm-start network kernels against the FP64 reference
(oracle/net_oracle.py) and of the grid field batches against the scaling
oracle.  GEMM: BF16 operands are exact in FP32, so the MFMA product must
match an FP64 product of the same BF16 values to FP32 accumulation error."""
import sys

import numpy as np
import pytest
import torch

from oracle import net_oracle as NO
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


@pytest.mark.parametrize("ta,tb", [(False, False), (False, True), (True, False), (True, True)])
@pytest.mark.parametrize("M,N,K", [(70, 45, 100), (64, 64, 32), (5, 130, 7), (256, 256, 512)])
def test_gemm_bf16_layouts(ta, tb, M, N, K):
    say("case gemm", ta, tb, M, N, K)
    rng = np.random.default_rng(M * 7 + N + K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    Ab = torch.tensor(A, device=DEV)
    Bb = torch.tensor(B, device=DEV)
    C = U.gemm_bf16(U.bf16_bits(Ab).contiguous(), U.bf16_bits(Bb).contiguous(), M, N, K, ta=ta, tb=tb).cpu().numpy()
    Aq, Bq = NO.bf16_round(A), NO.bf16_round(B)
    ref = (Aq.T if ta else Aq) @ (Bq.T if tb else Bq)
    err = np.max(np.abs(C - ref)) / max(np.max(np.abs(ref)), 1e-30)
    assert err < 2e-6, err


def test_net_gradient_matches_reference():
    rng = np.random.default_rng(4)
    n_in, width, n_out, batch = 64, 32, 48, 20
    net = U.WarmStartNet(n_in, width, n_out, DEV, seed=3, in_scale=0.5, in_shift=0.1)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    t = rng.standard_normal((batch, n_out)).astype(np.float32) * 0.3
    say("case net grad")
    g, loss = net.grad(torch.tensor(x, device=DEV), torch.tensor(t, device=DEV))
    theta = net.master.cpu().numpy().astype(np.float64)
    lref, gref = NO.loss_and_grad(theta, x, t, n_in, width, n_out, 0.5, 0.1, bf16=True)
    assert loss == pytest.approx(lref, rel=1e-4)
    g = g.cpu().numpy()
    # per parameter block: relative error in norm (BF16 rounding of gradients
    # that differ in the last FP32 bits can flip)
    sizes = [n_in * width, width, width * width, width, width * width, width, width * n_out, n_out]
    o = 0
    for s in sizes:
        a, b = g[o:o + s], gref[o:o + s]
        assert np.linalg.norm(a - b) <= 2e-2 * np.linalg.norm(b) + 1e-7, (o, s)
        o += s
    # inference agrees with the reference forward
    y = net.infer(torch.tensor(x, device=DEV)).cpu().numpy()
    yref, _ = NO.forward(theta, x, n_in, width, n_out, 0.5, 0.1, bf16=True)
    assert np.max(np.abs(y - yref)) < 1e-3 * np.max(np.abs(yref))


def test_net_training_reduces_loss():
    rng = np.random.default_rng(5)
    n_in, width, n_out, batch = 32, 64, 16, 64
    net = U.WarmStartNet(n_in, width, n_out, DEV, seed=1)
    W = rng.standard_normal((n_out, n_in)) / np.sqrt(n_in)
    x = rng.standard_normal((batch, n_in)).astype(np.float32)
    t = np.tanh(x @ W.T).astype(np.float32)
    xt, tt = torch.tensor(x, device=DEV), torch.tensor(t, device=DEV)
    say("case net train")
    l0 = net.train_step(xt, tt, 1e-3, want_loss=True)
    for _ in range(300):
        net.train_step(xt, tt, 1e-3)
    l1 = net.train_step(xt, tt, 1e-3, want_loss=True)
    assert l1 < 0.2 * l0, (l0, l1)


def test_features_and_upsample():
    rng = np.random.default_rng(6)
    nb, R, r = 3, 16, 8
    p = rng.uniform(0.1, 2.0, (nb, R * R)).astype(np.float32)
    q = rng.uniform(0.1, 2.0, (nb, R * R)).astype(np.float32)
    say("case features")
    x = U.warmstart_features(torch.tensor(p, device=DEV), torch.tensor(q, device=DEV), R, r).cpu().numpy()
    pool = lambda a: a.reshape(nb, r, 2, r, 2).mean(axis=(2, 4)).reshape(nb, r * r)
    ref = np.concatenate([np.log(pool(p)), np.log(pool(q))], axis=1)
    np.testing.assert_allclose(x, ref, rtol=1e-5, atol=1e-6)
    y = rng.standard_normal((nb, r * r)).astype(np.float32)
    up = U.grid_upsample(torch.tensor(y, device=DEV), r, R).cpu().numpy()
    # bilinear interpolation of cell centres, clamped: compare with a direct evaluation
    c = (np.arange(R) + 0.5) * r / R - 0.5
    c = np.clip(c, 0, r - 1)
    i0 = np.floor(c).astype(int)
    i1 = np.minimum(i0 + 1, r - 1)
    a = c - i0
    Y = y.reshape(nb, r, r)
    rows = Y[:, i0, :] * (1 - a)[None, :, None] + Y[:, i1, :] * a[None, :, None]
    refu = rows[:, :, i0] * (1 - a)[None, None, :] + rows[:, :, i1] * a[None, None, :]
    np.testing.assert_allclose(up.reshape(nb, R, R), refu, rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("shape", [(20, 17), (40,)])
def test_fields_fixed_iterations(shape):
    rng = np.random.default_rng(7)
    nb = 5
    size = int(np.prod(shape))
    h = tuple(1.0 / n for n in shape)
    p = rounded(rng.uniform(0.2, 2.0, (nb, size)), np.float32)
    q = rounded(rng.uniform(0.2, 2.0, (nb, size)), np.float32)
    d = rounded(np.full(size, float(np.prod(h))), np.float32)
    T = lambda a: torch.tensor(a, dtype=torch.float32, device=DEV)
    F = U.KL(0.5)
    eps = 0.01
    say("case fields", shape)
    u, v, info = U.solve_fields(shape, h, T(p), T(q), T(d), T(d), F, F, eps, tol=0.0, max_iter=25)
    G = O.GridGeom(shape, h)
    for k in range(nb):
        ref = O.solve(G, np.log(p[k]), np.log(q[k]), np.log(d), np.log(d), O.KL(0.5), O.KL(0.5), eps, tol=0.0,
                      max_iter=25)
        assert pot_rel_err(u[k].cpu(), ref["u"], eps) < 1e-5
        assert pot_rel_err(v[k].cpu(), ref["v"], eps) < 1e-5
    # to tolerance: every field's own residual (oracle half-step at the final
    # state) is at most the tolerance
    u, v, info = U.solve_fields(shape, h, T(p), T(q), T(d), T(d), F, F, eps, tol=1e-6, max_iter=5000)
    assert info["converged"]
    for k in range(nb):
        _, _, r = O.half_step_x(G, np.log(p[k]), np.log(d), np.log(d), O.KL(0.5), eps,
                                u[k].cpu().numpy().astype(np.float64), v[k].cpu().numpy().astype(np.float64))
        assert r < 5e-6, (k, r)
