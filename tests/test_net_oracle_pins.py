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
