"""Pins of the network reference: the FP64 backward against central finite
differences of the FP64 forward, and the BF16 rounding against torch's own
float32 -> bfloat16 conversion."""
import numpy as np
import torch

from oracle import net_oracle as N


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(5000).astype(np.float32) * 10 ** rng.uniform(-6, 6, 5000).astype(np.float32),
                        np.array([0.0, -0.0, 1.0, 1.00390625, 1.01171875, 3.4e38, 1e-40], np.float32)])
    ours = N.bf16_round(x)
    ref = torch.tensor(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ours, ref)


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    n_in, width, n_out, batch = 6, 5, 4, 3
    cnt = n_in * width + width + 2 * (width * width + width) + width * n_out + n_out
    theta = rng.standard_normal(cnt) * 0.5
    x = rng.standard_normal((batch, n_in))
    t = rng.standard_normal((batch, n_out))
    loss, g = N.loss_and_grad(theta, x, t, n_in, width, n_out, 0.7, 0.1, bf16=False)
    h = 1e-6
    for k in rng.choice(cnt, 40, replace=False):
        e = np.zeros(cnt)
        e[k] = h
        lp, _ = N.loss_and_grad(theta + e, x, t, n_in, width, n_out, 0.7, 0.1, bf16=False)
        lm, _ = N.loss_and_grad(theta - e, x, t, n_in, width, n_out, 0.7, 0.1, bf16=False)
        assert abs((lp - lm) / (2 * h) - g[k]) < 1e-6 * max(1.0, abs(g[k]))


def test_forward_is_the_plain_mlp():
    """Without rounding the forward is relu(relu(relu(x W1^T + b1) W2^T + b2) W3^T + b3) W4^T + b4."""
    rng = np.random.default_rng(2)
    n_in, width, n_out = 8, 6, 5
    cnt = n_in * width + width + 2 * (width * width + width) + width * n_out + n_out
    theta = rng.standard_normal(cnt)
    x = rng.standard_normal((4, n_in))
    y, _ = N.forward(theta, x, n_in, width, n_out, bf16=False)
    Ws, bs = N.unpack(theta, n_in, width, n_out)
    r = lambda a: np.maximum(a, 0)
    ref = r(r(r(x @ Ws[0].T + bs[0]) @ Ws[1].T + bs[1]) @ Ws[2].T + bs[2]) @ Ws[3].T + bs[3]
    np.testing.assert_allclose(y, ref, rtol=1e-13)


# ---------------------------------------------------------------------------
# Adam (Kingma & Ba 2015, Algorithm 1)
# ---------------------------------------------------------------------------
def test_adam_first_step_hand_computed():
    """At t = 1 the bias corrections make mhat = g and vhat = g^2, so the step
    is -lr g / (|g| + eps).  Values worked out by hand for lr = 0.01,
    eps = 1e-8: 0.5 -> -0.01 * 0.5 / 0.50000001, -2e-3 -> +0.01 * 2e-3 /
    0.00200001, 0 -> 0, 1e-9 -> -0.01 / 11."""
    w0 = np.array([1.0, -1.0, 0.25, 3.0])
    g = np.array([0.5, -2e-3, 0.0, 1e-9])
    w1, m1, v1 = N.adam_step(w0, g, np.zeros(4), np.zeros(4), 1, 0.01)
    step = np.array([-0.0099999998000000004, 0.0099999500002499987, 0.0, -0.00090909090909090909])
    np.testing.assert_allclose(w1 - w0, step, rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 1e-3 * g * g, rtol=1e-12)


def test_adam_constant_gradient_steps_are_identical():
    """Under a constant gradient the bias-corrected moments equal g and g^2 at
    every step, so every step is the first one again."""
    rng = np.random.default_rng(3)
    g = rng.standard_normal(50)
    w = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    first = None
    for t in range(1, 41):
        w_new, m, v = N.adam_step(w, g, m, v, t, 1e-3)
        if first is None:
            first = w_new - w
        np.testing.assert_allclose(w_new - w, first, rtol=1e-9)
        w = w_new


def test_adam_is_invariant_to_gradient_scale():
    """With eps = 0 the update depends on g only through g / sqrt(E g^2):
    gradients scaled by c > 0 give the same trajectory."""
    rng = np.random.default_rng(4)
    gs = rng.standard_normal((12, 30))
    traj = []
    for c in (1.0, 37.5, 1e-4):
        w, m, v = np.ones(30), np.zeros(30), np.zeros(30)
        for t, g in enumerate(gs, start=1):
            w, m, v = N.adam_step(w, c * g, m, v, t, 0.05, eps=0.0)
        traj.append(w)
    np.testing.assert_allclose(traj[1], traj[0], rtol=1e-12)
    np.testing.assert_allclose(traj[2], traj[0], rtol=1e-12)


def test_adam_minimises_a_quadratic():
    """Steps go against the gradient: on f(w) = sum a_i (w_i - c_i)^2 Adam
    ends within a few learning rates of the minimiser c."""
    rng = np.random.default_rng(5)
    a = rng.uniform(0.1, 10.0, 20)
    c = rng.standard_normal(20)
    w, m, v = np.zeros(20), np.zeros(20), np.zeros(20)
    lr = 1e-2
    for t in range(1, 3001):
        w, m, v = N.adam_step(w, 2 * a * (w - c), m, v, t, lr)
    assert np.max(np.abs(w - c)) < 3 * lr


def test_dyadic_network_design_is_exact_in_fp32():
    """The integer-valued network of tests/net_cases.py (used for the
    bit-exact GPU test at the production shape) meets its exactness
    precondition, and an FP32 evaluation in another summation order (BLAS
    sgemm) gives the FP64 reference's forward output bit for bit."""
    from tests import net_cases
    n_in, width, n_out, batch = 8192, 256, 4096, 256
    theta, x, t = net_cases.dyadic_net(11, n_in, width, n_out, batch)
    fwd, bwd = net_cases.exact_margins(theta, x, t, n_in, width, n_out)
    assert fwd < 2 ** 24 and bwd < 2 ** 24
    y64, _ = N.forward(theta, x, n_in, width, n_out, bf16=True)
    Ws, bs = N.unpack(theta, n_in, width, n_out)
    h = x.astype(np.float32)
    for l in range(4):
        z = h @ Ws[l].T.astype(np.float32) + bs[l].astype(np.float32)
        h = N.bf16_round(np.maximum(z, 0)).astype(np.float32) if l < 3 else z
    assert np.array_equal(h.astype(np.float64), y64)
