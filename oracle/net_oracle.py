"""FP64 CPU reference of the warm-start network (TEST INFRASTRUCTURE ONLY).

4-layer MLP n_in -> width -> width -> width -> n_out, ReLU on hidden layers,
loss = mean over batch x n_out of (y - t)^2.  With bf16=True the inputs of
every matrix product (weights and activations) are rounded to BF16 (round to
nearest even) exactly where the GPU network rounds them, and the backward
pass treats the rounding as the identity (straight-through), which is what
the GPU gradient computes.  Parameter layout: W1 [width x n_in], b1, W2, b2,
W3, b3, W4 [n_out x width], b4.  The optimiser is Adam (`adam_step`), in
FP64.
"""
import numpy as np


def bf16_round(a):
    """Round float32 values to the nearest BF16 (ties to even), as float64."""
    x = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    bits = x.view(np.uint32).astype(np.uint64)
    rounded = ((bits + 0x7FFF + ((bits >> 16) & 1)) >> 16) << 16
    finite = np.isfinite(x)
    out = np.where(finite, rounded, bits).astype(np.uint32).view(np.float32)
    return out.astype(np.float64)


def unpack(theta, n_in, width, n_out):
    ins = [n_in, width, width, width]
    outs = [width, width, width, n_out]
    Ws, bs, o = [], [], 0
    for fi, fo in zip(ins, outs):
        Ws.append(np.asarray(theta[o:o + fi * fo], np.float64).reshape(fo, fi))
        o += fi * fo
        bs.append(np.asarray(theta[o:o + fo], np.float64))
        o += fo
    return Ws, bs


def forward(theta, x, n_in, width, n_out, in_scale=1.0, in_shift=0.0, bf16=True):
    """Returns (y, cache).  x: (batch, n_in)."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    Ws, bs = unpack(theta, n_in, width, n_out)
    h = q(np.float32(in_scale) * np.asarray(x, np.float32) + np.float32(in_shift)) if bf16 else \
        in_scale * np.asarray(x, np.float64) + in_shift
    cache = {"h": [h], "z": []}
    for l in range(4):
        z = h @ q(Ws[l]).T + bs[l]
        if l < 3:
            cache["z"].append(z)
            h = q(np.maximum(z, 0.0))
            cache["h"].append(h)
        else:
            y = z
    return y, cache


def loss_and_grad(theta, x, t, n_in, width, n_out, in_scale=1.0, in_shift=0.0, bf16=True):
    """loss = mean (y - t)^2 and d loss / d theta (flat, parameter layout)."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, np.float64))
    Ws, bs = unpack(theta, n_in, width, n_out)
    y, cache = forward(theta, x, n_in, width, n_out, in_scale, in_shift, bf16)
    d = y - np.asarray(t, np.float64)
    loss = float(np.mean(d * d))
    g = q(2.0 * d / d.size)
    gW, gb = [None] * 4, [None] * 4
    for l in range(3, -1, -1):
        gW[l] = g.T @ cache["h"][l]
        gb[l] = g.sum(axis=0)
        if l == 0:
            break
        dh = g @ q(Ws[l])
        g = q(np.where(cache["z"][l - 1] > 0, dh, 0.0))
    flat = []
    for l in range(4):
        flat.append(gW[l].reshape(-1))
        flat.append(gb[l])
    return loss, np.concatenate(flat)


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One step of Adam (Kingma & Ba, "Adam: a method for stochastic
    optimization", ICLR 2015, Algorithm 1), in FP64: the moment estimates
    m <- beta1 m + (1 - beta1) g and v <- beta2 v + (1 - beta2) g^2, their
    bias corrections m / (1 - beta1^t), v / (1 - beta2^t) at step t >= 1, and
    w <- w - lr mhat / (sqrt(vhat) + eps).  Returns (w, m, v) as new arrays."""
    w, g, m, v = (np.asarray(a, np.float64) for a in (w, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return w - lr * mhat / (np.sqrt(vhat) + eps), m, v
