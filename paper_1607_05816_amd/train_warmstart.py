"""Train the warm-start network on solves of the library's own grid solver,
then compare cold and warm barycentre solves.

    python -m paper_1607_05816_amd.train_warmstart --pairs 50000 --epochs 30 \
        --out paper_1607_05816_amd/data/warmstart_mlp64.npz --report report.json

Training pairs: blob image pairs at 64 x 64 (seeds 1000 .. 1000 + pairs - 1),
targets v of UOT(p, q) with KL lambda = 0.5, eps = 2e-3 (eps-scaling from
1e-1, residual 1e-6).  Evaluation: barycentres of 8 blob images at 128 x 128
(seeds 0 .. n_eval - 1), alpha_k = 1/8, same eps and lambda, residual 1e-6:
  * cold + eps-scaling (the paper's recipe for small eps),
  * cold without annealing (v^(0) = 0),
  * warm: v^(0) from the network, no annealing.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

from . import synth
from . import uot as U
from . import warmstart as W

WIDTH = 256


def save_weights(net: U.WarmStartNet, path, extra=None):
    """Weights as their BF16 values (what the GEMMs use) plus FP32 biases;
    `extra` (name -> array) is stored beside them."""
    theta = net.master.cpu().numpy()
    wb = net.wbf16.cpu().numpy().view(np.uint16)
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez_compressed(path, wbf16=wb, theta_fp32_bias_mask=_bias_mask(net), biases=theta[_bias_mask(net)],
                        n_in=net.c.n_in, width=net.c.width, n_out=net.c.n_out, in_scale=net.c.in_scale,
                        in_shift=net.c.in_shift, **(extra or {}))


def _bias_mask(net):
    n_in, w, n_out = net.c.n_in, net.c.width, net.c.n_out
    mask = np.zeros(net.n_params, bool)
    o = 0
    for fi, fo in ((n_in, w), (w, w), (w, w), (w, n_out)):
        o += fi * fo
        mask[o:o + fo] = True
        o += fo
    return mask


def load_weights(path, device):
    z = np.load(path, allow_pickle=False)
    theta = (z["wbf16"].astype(np.uint32) << 16).view(np.float32).copy()
    mask = z["theta_fp32_bias_mask"]
    theta[mask] = z["biases"]
    return U.WarmStartNet(int(z["n_in"]), int(z["width"]), int(z["n_out"]), device, in_scale=float(z["in_scale"]),
                          in_shift=float(z["in_shift"]), params=theta)


def evaluate(net, seeds, device, R=128, n_marg=8, log=print):
    rows = []
    for s in seeds:
        pr = synth.bary_blobs(int(s), n_marg=n_marg, n=R)
        p = torch.tensor(pr.p, dtype=torch.float32, device=device)
        alpha = pr.alpha
        res = {"seed": int(s)}
        for name, kw in (("cold_eps_scaling", dict(eps0=W.EPS0)), ("cold", dict()), ("warm", None)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kw is None:
                v0 = W.barycenter_v0(net, p, alpha, R)
                _, _, _, info = W.barycenter_solve(p, alpha, R, v0=v0.contiguous())
            else:
                _, _, _, info = W.barycenter_solve(p, alpha, R, **kw)
            torch.cuda.synchronize()
            res[name] = dict(iters=int(info["iters"]), ms=(time.perf_counter() - t0) * 1e3,
                             converged=bool(info["converged"]))
        rows.append(res)
        log("eval seed %d: %s" % (s, {k: v for k, v in res.items() if k != "seed"}))
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--pairs", type=int, default=50000)
    ap.add_argument("--val", type=int, default=2000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n-eval", type=int, default=20)
    ap.add_argument("--out", default=None)
    ap.add_argument("--report", default=None)
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    log = lambda *a: (print(*a, flush=True), sys.stdout.flush())
    t0 = time.perf_counter()
    P, Q = W.pair_densities(range(1000, 1000 + args.pairs))
    log("generated %d pairs in %.1f s" % (args.pairs, time.perf_counter() - t0))
    t1 = time.perf_counter()
    V, infos = W.solve_pairs(P, Q, dev)
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t1
    log("solved %d pairs in %.1f s (%d iterations per batch; largest per-field residual of the last iteration "
        "per batch: %s)" % (args.pairs, solve_s, W.SOLVE_ITERS, ["%.1e" % i["residual"] for i in infos]))
    X = W.features(P, Q, W.RES, dev)
    ntr = args.pairs - args.val
    net = U.WarmStartNet(2 * W.RES * W.RES, WIDTH, W.RES * W.RES, dev, seed=0, in_scale=W.IN_SCALE,
                         in_shift=W.IN_SHIFT)
    tl = W.train(net, X[:ntr].contiguous(), V[:ntr].contiguous(), X[ntr:].contiguous(), V[ntr:].contiguous(),
                 epochs=args.epochs, batch=args.batch, lr=args.lr)
    log("trained %d steps in %.1f s; val loss per epoch %s" % (tl.steps, tl.seconds,
                                                              ["%.3e" % v for v in tl.val_loss]))
    vscale = float(V[ntr:].double().pow(2).mean())
    rows = evaluate(net, range(args.n_eval), dev, log=log)
    summary = {}
    for k in ("cold_eps_scaling", "cold", "warm"):
        summary[k] = dict(iters_mean=float(np.mean([r[k]["iters"] for r in rows])),
                          ms_mean=float(np.mean([r[k]["ms"] for r in rows])),
                          all_converged=all(r[k]["converged"] for r in rows))
    report = dict(pairs=args.pairs, solve_seconds=solve_s, solve_iters=[int(i["iters"]) for i in infos],
                  solve_final_max_residual=[float(i["residual"]) for i in infos],
                  train_seconds=tl.seconds, train_steps=tl.steps, val_loss=tl.val_loss, train_loss=tl.train_loss,
                  val_target_mean_square=vscale, eval=rows, summary=summary)
    log(json.dumps(summary))
    if args.out:
        save_weights(net, args.out)
    if args.report:
        with open(args.report, "w") as f:
            json.dump(report, f)


if __name__ == "__main__":
    main()
