"""Seeded inputs for the network tests.

`dyadic_net` draws a network whose weights, biases and inputs are small
integers on sparse rows, and targets t = y - s with y the reference output and
s a small integer.  Every product and partial sum of the forward pass is then
an integer below 2^24, and every one of the backward pass a multiple of 2^-19
(the loss coefficient 2 / (256 * 4096) = 2^-19 at the production shape) whose
absolute partial sums stay below 2^24 * 2^-19.  FP32 represents all of them
exactly, whatever the summation order (split K with atomics included), and
the BF16 roundings act on exact values, so the GPU network must reproduce the
FP64 reference bit for bit.  `exact_margins` checks that precondition on the
reference's own values.
"""
import numpy as np

from oracle import net_oracle as NO


def _sparse_rows(rng, fo, fi, nnz):
    W = np.zeros((fo, fi))
    for r in range(fo):
        cols = rng.choice(fi, nnz, replace=False)
        W[r, cols] = rng.choice([-2.0, -1.0, 1.0, 2.0], nnz)
    return W


def dyadic_net(seed, n_in, width, n_out, batch, nnz=(8, 8, 8, 8)):
    """(theta, x, t): integer-valued sparse weights, integer biases, inputs in
    {-1, 0, 1}; targets t = y - s, s in {-3..3}, from the FP64 reference."""
    rng = np.random.default_rng(seed)
    ins = [n_in, width, width, width]
    outs = [width, width, width, n_out]
    parts = []
    for l in range(4):
        parts.append(_sparse_rows(rng, outs[l], ins[l], nnz[l]).reshape(-1))
        parts.append(rng.integers(-2, 3, outs[l]).astype(np.float64))
    theta = np.concatenate(parts)
    x = rng.integers(-1, 2, (batch, n_in)).astype(np.float64)
    y, _ = NO.forward(theta, x, n_in, width, n_out, bf16=True)
    t = y - rng.integers(-3, 4, y.shape)
    return theta, x, t


def exact_margins(theta, x, t, n_in, width, n_out):
    """Largest sum of absolute terms over every dot product of the forward
    pass (in units of 1) and of the backward pass (in units of the loss
    coefficient); FP32 is exact when both are below 2^24 and every value is
    an integer in its unit."""
    Ws, bs = NO.unpack(theta, n_in, width, n_out)
    y, cache = NO.forward(theta, x, n_in, width, n_out, bf16=True)
    fwd = 0.0
    for l in range(4):
        h = cache["h"][l]
        fwd = max(fwd, float(np.max(np.abs(h) @ np.abs(Ws[l]).T + np.abs(bs[l]))))
        assert np.array_equal(h, np.round(h)), "activations must be integers"
    coef = 2.0 / y.size
    d = y - t
    assert np.array_equal(d, np.round(d))
    g = NO.bf16_round(coef * d) / coef           # backward values in units of coef
    bwd = 0.0
    for l in range(3, -1, -1):
        h = cache["h"][l]
        bwd = max(bwd, float(np.max(np.abs(g).T @ np.abs(h))), float(np.max(np.abs(g).sum(axis=0))))
        if l == 0:
            break
        dh = g @ Ws[l]
        bwd = max(bwd, float(np.max(np.abs(g) @ np.abs(Ws[l]))))
        assert np.array_equal(dh, np.round(dh))
        g = np.where(cache["z"][l - 1] > 0, NO.bf16_round(dh * coef) / coef, 0.0)
        assert np.array_equal(g, np.round(g))
    return fwd, bwd
