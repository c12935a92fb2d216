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
from tests import net_cases
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


PROD = (8192, 256, 4096, 256)   # n_in, width, n_out, batch of the warm-start network


@pytest.mark.parametrize("ta,tb,M,N,K", [
    (False, True, 256, 256, 8192),    # forward layer 1 (split K)
    (False, True, 256, 4096, 256),    # forward layer 4
    (True, False, 256, 8192, 256),    # weight gradient of layer 1
    (True, False, 4096, 256, 256),    # weight gradient of layer 4
    (False, False, 256, 256, 4096),   # input gradient of layer 4 (split K)
])
def test_gemm_bf16_production_products(ta, tb, M, N, K):
    """The network's five product shapes on generic data, element by element
    against the FP64 product of the same BF16 values.  BF16 x BF16 products
    are exact in FP32, so the only error is FP32 summation of K terms, which
    in any order is at most K 2^-24 sum_k |a_mk b_kn| (plus second order)."""
    say("case gemm production", ta, tb, M, N, K)
    rng = np.random.default_rng(M + 3 * N + 7 * K)
    A = rng.standard_normal((K, M) if ta else (M, K)).astype(np.float32)
    B = rng.standard_normal((N, K) if tb else (K, N)).astype(np.float32)
    C = U.gemm_bf16(U.bf16_bits(torch.tensor(A, device=DEV)).contiguous(),
                    U.bf16_bits(torch.tensor(B, device=DEV)).contiguous(), M, N, K, ta=ta, tb=tb).cpu().numpy()
    Aq, Bq = NO.bf16_round(A), NO.bf16_round(B)
    Aq, Bq = (Aq.T if ta else Aq), (Bq.T if tb else Bq)
    ref = Aq @ Bq
    bound = 1.01 * K * 2.0 ** -24 * (np.abs(Aq) @ np.abs(Bq))
    assert np.all(np.abs(C - ref) <= bound)


def test_net_production_shape_bit_exact_and_adam():
    """The warm-start network at its production shape (8192 -> 256 -> 256 ->
    256 -> 4096, batch 256; layer 1 and the layer-4 input gradient run split
    K with FP32 atomics) on integer-valued sparse weights, integer inputs and
    targets one to three units off the output (tests/net_cases.py).  Every
    sum is then exact in FP32 in any order and every BF16 rounding acts on
    exact values, so the forward output, the loss and the whole gradient must
    equal the FP64 reference bit for bit.  One Adam step (the same batch)
    must then match the reference Adam step element by element: FP32
    evaluation of the update formula, with the kernel's FP32 constants, within
    a few units in the last place."""
    n_in, width, n_out, batch = PROD
    theta, x, t = net_cases.dyadic_net(11, n_in, width, n_out, batch)
    fwd, bwd = net_cases.exact_margins(theta, x, t, n_in, width, n_out)
    assert fwd < 2 ** 24 and bwd < 2 ** 24
    net = U.WarmStartNet(n_in, width, n_out, DEV, params=theta.astype(np.float32), in_scale=1.0, in_shift=0.0)
    xt = torch.tensor(x, dtype=torch.float32, device=DEV)
    tt = torch.tensor(t, dtype=torch.float32, device=DEV)
    say("case net production forward")
    y = net.infer(xt).cpu().numpy().astype(np.float64)
    yref, _ = NO.forward(theta, x, n_in, width, n_out, bf16=True)
    assert np.array_equal(y, yref), np.max(np.abs(y - yref))
    say("case net production gradient")
    g, loss = net.grad(xt, tt)
    lref, gref = NO.loss_and_grad(theta, x, t, n_in, width, n_out, bf16=True)
    g = g.cpu().numpy().astype(np.float64)
    assert loss == lref
    bad = np.flatnonzero(g != gref)
    assert bad.size == 0, (bad.size, bad[:10])
    say("case net production adam")
    lr = 1e-3
    net.train_step(xt, tt, lr)
    f = lambda c: float(np.float32(c))
    wref, mref, vref = NO.adam_step(theta, gref, np.zeros_like(theta), np.zeros_like(theta), 1, f(lr),
                                    beta1=f(0.9), beta2=f(0.999), eps=f(1e-8))
    w = net.master.cpu().numpy().astype(np.float64)
    step = np.abs(wref - theta)
    assert np.all(np.abs(w - wref) <= 2.0 ** -24 * np.abs(wref) + 2.0 ** -21 * step)
    assert np.array_equal(w == theta, gref == 0)
    np.testing.assert_allclose(net.m.cpu().numpy(), mref, rtol=2.0 ** -21, atol=0)
    np.testing.assert_allclose(net.v.cpu().numpy(), vref, rtol=2.0 ** -20, atol=0)
    wb = NO.bf16_round(w.astype(np.float32)).astype(np.float32).view(np.uint32) >> 16
    assert np.array_equal(net.wbf16.cpu().numpy().view(np.uint16), wb.astype(np.uint16)), "BF16 copy of the weights"


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
