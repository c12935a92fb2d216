"""Learned warm start for ragged batches of point-cloud problems.

By Prop. "alternating" only v^(0) enters the iterates.  At the fixed point
of a KL(lambda) second marginal, v_j = z eps log q_j - z eps T(y_j) with
z = lambda / (lambda + eps) (Table proximalexplicit, KL row, in the log
domain): a pointwise part that the input gives exactly, and a smooth part,
-z eps times the log of the Gibbs product of the first measure's scaled
potential, which depends on the two measures near y_j at the kernel's width.
The network (4-layer MLP 16 -> 64 -> 64 -> 64 -> 1, BF16 weights, FP32
accumulation; kernels in csrc/uot_net.hip) predicts that smooth part point
by point from 16 features (uot_cloud_features: the masses of both measures
and of both reference measures near y_j at several kernel widths, Gibbs
products of the library, and the problem's total masses and size ratio).
v^(0) = z eps log q + prediction (uot_cloud_v0).  Last, each problem's
constant is set by the mass balance (uot_batch_balance): one X half-step
from v^(0), then the shift of v^(0) that makes the plan's first-marginal mass
agree with the second-marginal mass v^(0) implies, as the two do at the fixed
point.  The constant is the mode the iteration contracts most slowly (by
z^2 per iteration), so the network predicts the shape and the balance sets
the level.  The plain iteration then runs to the same tolerance, so the
warm start changes the number of iterations, never the answer.

Everything here is orchestration: every arithmetic step of the warm start
runs in libuot.
"""
from __future__ import annotations

import os

import numpy as np
import torch

from . import synth
from . import uot as U

EPS = 5e-3
LAM = 1.0
TOL = 1e-6
WIDTH = 64
WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "data", "warmstart_cloud.npz")


def zeps(eps=EPS, lam=LAM):
    return eps * lam / (lam + eps)


def batch_problem(probs, device, lam=LAM) -> U.BatchProblem:
    """A BatchProblem (FP32, KL(lam) on both marginals) of synth.CloudProblem's."""
    cat = lambda f: torch.tensor(np.concatenate([f(p) for p in probs]).astype(np.float32), device=device)
    F = U.KL(lam)
    return U.BatchProblem([p.x.shape[0] for p in probs], [p.y.shape[0] for p in probs], cat(lambda p: p.x),
                          cat(lambda p: p.y), cat(lambda p: p.p), cat(lambda p: p.q), cat(lambda p: p.dx),
                          cat(lambda p: p.dy), F, F, layout="nd")


class CloudWarmStart:
    """The trained network with its input and output normalisation."""

    def __init__(self, net: U.WarmStartNet, shift, scale, out_shift, out_scale, eps=EPS, lam=LAM):
        self.net = net
        self.shift = np.asarray(shift, np.float32)
        self.scale = np.asarray(scale, np.float32)
        self.out_shift, self.out_scale = float(out_shift), float(out_scale)
        self.eps, self.lam = float(eps), float(lam)

    def features(self, bp: U.BatchProblem, ctx=None):
        return U.cloud_features(bp, self.eps, self.shift, self.scale, ctx=ctx)

    def v0(self, bp: U.BatchProblem, ctx=None, chunk=1 << 20, balance=True):
        """v^(0) (totM) for every problem of the batch; balance: finish with
        the mass balance of each problem's constant."""
        x = self.features(bp, ctx=ctx)
        y = torch.empty(bp.totM, dtype=torch.float32, device=x.device)
        for a in range(0, bp.totM, chunk):
            y[a:a + chunk] = self.net.infer(x[a:a + chunk].contiguous(), ctx=ctx).reshape(-1)
        v0 = U.cloud_v0(bp.q, zeps(self.eps, self.lam), y, self.out_scale, self.out_shift, ctx=ctx)
        return U.batch_balance(bp, self.eps, v0, ctx=ctx) if balance else v0

    def target(self, bp: U.BatchProblem, v, ctx=None):
        """Training target of the network for converged potentials v: the
        normalised smooth part (v - z eps log q - out_shift) / out_scale."""
        return U.cloud_v0(bp.q, -zeps(self.eps, self.lam) / self.out_scale, v.contiguous(), 1.0 / self.out_scale,
                          -self.out_shift / self.out_scale, ctx=ctx)

    def save(self, path):
        from .train_warmstart import save_weights
        save_weights(self.net, path, extra=dict(shift=self.shift, scale=self.scale, out_shift=self.out_shift,
                                                 out_scale=self.out_scale, eps=self.eps, lam=self.lam))

    @staticmethod
    def load(path, device):
        from .train_warmstart import load_weights
        net = load_weights(path, device)
        z = np.load(path, allow_pickle=False)
        return CloudWarmStart(net, z["shift"], z["scale"], float(z["out_shift"]), float(z["out_scale"]),
                              float(z["eps"]), float(z["lam"]))


def balanced_cold_v0(bp: U.BatchProblem, eps=EPS, ctx=None):
    """The start without a network: v^(0) = 0 with each problem's constant
    set by the mass balance."""
    v0 = torch.zeros(bp.totM, dtype=torch.float32, device=bp.q.device)
    return U.batch_balance(bp, eps, v0, ctx=ctx)


def ragged(seed, B=4096, lo=64, hi=4096):
    return synth.ragged_batch(seed, B=B, lo=lo, hi=hi)


def solve(bp, v0=None, ctx=None, **kw):
    kw.setdefault("tol", TOL)
    kw.setdefault("max_iter", 20000)
    kw.setdefault("check_every", 50)
    return U.solve_batched(bp, EPS, v0=v0, ctx=ctx, **kw)
