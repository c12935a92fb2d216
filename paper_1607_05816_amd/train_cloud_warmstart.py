"""Train the warm-start network of ragged point-cloud batches on the
library's own batched solves, then compare cold and warm batched solves.

    python -m paper_1607_05816_amd.train_cloud_warmstart --batches 4 \
        --out paper_1607_05816_amd/data/warmstart_cloud.npz --report report.json

Training data: ragged batches of 4096 problems (seeds 101 .. 100 + batches;
N, M log-uniform on [64, 4096], uniform points in [0,1]^2, densities
U[0.1, 1], KL lambda = 1 on both marginals, eps = 5e-3), solved cold to
residual 1e-6 by uot_solve_batched; one sample per point of the second
clouds: its 16 features and the smooth part of its converged v, minus that
part's mean over the problem (--centred, the default): the warm start ends
with the mass balance, which sets each problem's level exactly (a constant
added to v^(0) moves the balance shift by the same constant), so the
network only has the shape to learn.  Validation: the batch of seed 100.
Evaluation: held-out batches (seeds --eval-seeds), cold, the mass balance
alone and the full warm start, all batched, to residual 1e-6.

The input normalisation (per-feature mean and standard deviation), the
per-problem means of the targets and the target normalisation are
statistics of the training set, taken with torch reductions; every product,
feature, forward and backward pass and Adam step runs in libuot.
"""
import argparse
import json
import sys
import time

import numpy as np
import torch

from . import cloud_warmstart as CW
from . import uot as U


def solved_batch(seed, dev, B, log):
    bp = CW.batch_problem(CW.ragged(seed, B=B), dev)
    t = time.perf_counter()
    _, v, info = CW.solve(bp)
    torch.cuda.synchronize()
    log("seed %d: %d problems solved cold in %.2f s, mean %.0f iterations, %d converged"
        % (seed, bp.B, time.perf_counter() - t, info["iters"].mean(), info["n_converged"]))
    return bp, v, info


def centred(bp, t):
    """t (totM) minus its mean over each problem's points."""
    M = torch.tensor(np.diff(bp.offM), dtype=torch.int64, device=t.device)
    ids = torch.repeat_interleave(torch.arange(bp.B, device=t.device), M)
    mean = torch.zeros(bp.B, dtype=t.dtype, device=t.device).index_add_(0, ids, t) / M.to(t.dtype)
    return t - mean[ids]


def evaluate(cw, seeds, dev, B, log):
    rows = []
    for s in seeds:
        bp = CW.batch_problem(CW.ragged(s, B=B), dev)
        CW.solve(bp)                                    # tunes the batch signature once
        res = {"seed": int(s)}
        for name in ("cold", "pointwise", "balance", "warm"):
            torch.cuda.synchronize()
            t = time.perf_counter()
            if name == "warm":
                v0 = cw.v0(bp)
            elif name == "pointwise":       # v0 = z eps log q: the exact pointwise part alone, no network
                v0 = U.cloud_v0(bp.q, CW.zeps(), torch.zeros_like(bp.q), 1.0, 0.0)
            elif name == "balance":         # the mass balance of v0 = 0, no network
                v0 = CW.balanced_cold_v0(bp)
            else:
                v0 = None
            _, v, info = CW.solve(bp, v0=v0)
            torch.cuda.synchronize()
            res[name] = dict(seconds=time.perf_counter() - t, iters_mean=float(info["iters"].mean()),
                             iters_total=int(info["iters"].sum()), converged=int(info["n_converged"]))
            res[name + "_v"] = v
        dv = float((res["warm_v"] - res["cold_v"]).abs().max() / res["cold_v"].abs().max())
        del res["warm_v"], res["cold_v"], res["pointwise_v"], res["balance_v"]
        res["v_rel_diff_warm_cold"] = dv
        res["speedup"] = res["cold"]["seconds"] / res["warm"]["seconds"]
        res["iters_ratio"] = res["cold"]["iters_total"] / res["warm"]["iters_total"]
        log("eval seed %d: %s" % (s, json.dumps(res)))
        rows.append(res)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batches", type=int, default=4)
    ap.add_argument("--B", type=int, default=4096)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--eval-seeds", type=int, nargs="*", default=[0])
    ap.add_argument("--centred", type=int, default=1, help="targets minus their per-problem mean")
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    log = lambda *a: (print(*a, flush=True), sys.stdout.flush())
    # training and validation data: features and converged potentials
    net = U.WarmStartNet(U.CLOUD_FEATURES, CW.WIDTH, 1, dev, seed=0)
    ident = CW.CloudWarmStart(net, np.zeros(U.CLOUD_FEATURES), np.ones(U.CLOUD_FEATURES), 0.0, 1.0)
    t0 = time.perf_counter()
    data = []
    for s in [100] + list(range(101, 101 + args.batches)):
        bp, v, info = solved_batch(s, dev, args.B, log)
        y = ident.target(bp, v)
        data.append((bp, v, ident.features(bp), centred(bp, y) if args.centred else y))
    solve_s = time.perf_counter() - t0
    X = torch.cat([d[2] for d in data[1:]])
    Y = torch.cat([d[3] for d in data[1:]])
    mu, sd = X.mean(0), X.std(0).clamp_min(1e-12)
    ymu, ysd = float(Y.mean()), float(Y.std())
    cw = CW.CloudWarmStart(net, mu.cpu().numpy(), (1.0 / sd).cpu().numpy(), ymu, ysd)
    # normalised targets: (t - ymu) / ysd of the (centred) smooth part
    tgt = lambda bp, v: (centred(bp, ident.target(bp, v)) if args.centred else ident.target(bp, v)) - ymu
    Xn = cw.features(data[0][0])        # validation features, normalised by the kernel
    Yv = (tgt(data[0][0], data[0][1]) / ysd).reshape(-1, 1)
    Xt = torch.cat([cw.features(d[0]) for d in data[1:]])
    Yt = torch.cat([tgt(d[0], d[1]) / ysd for d in data[1:]]).reshape(-1, 1)
    del data, X, Y
    log("features of %d training points (%d validation) in %.1f s; target std %.3e"
        % (Xt.shape[0], Xn.shape[0], time.perf_counter() - t0, ysd))
    from .warmstart import train
    tl = train(net, Xt, Yt, Xn, Yv, epochs=args.epochs, batch=args.batch, lr=args.lr)
    log("trained %d steps in %.1f s; validation loss (normalised target) per epoch %s"
        % (tl.steps, tl.seconds, ["%.4f" % v for v in tl.val_loss]))
    rows = evaluate(cw, args.eval_seeds, dev, args.B, log)
    report = dict(batches=args.batches, B=args.B, centred=bool(args.centred), solve_seconds=solve_s,
                  train_points=int(Xt.shape[0]),
                  train_seconds=tl.seconds, train_steps=tl.steps, val_loss=tl.val_loss, train_loss=tl.train_loss,
                  target_std=ysd, eval=rows)
    if args.out:
        cw.save(args.out)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f)


if __name__ == "__main__":
    main()
