#!/usr/bin/env python
"""Benchmark: Sinkhorn iterations per second and time to residual 1e-6 of the
generalized scaling iteration on one MI355X.

Workload (one "step" = one pass of the whole hot path over one input pair):
  2-D grid unbalanced OT between two 256 x 256 densities on [0,1]^2, each a
  sum of 5 random Gaussian blobs plus a 1e-6 floor, masses U[0.5, 2]
  (seeded synthetic stand-ins for the paper's 2-D experiment images);
  separable Gaussian kernel applied as log-domain 1-D passes; eps annealed
  1e-1 -> 1e-3 in 10 stages of 100 iterations, then iterated to residual
  1e-6; solved once with KL (lambda = 0.1) and once with TV (lambda = 0.05)
  penalties, each followed by the FP64 objective / gap reduction.  FP32.

Prints ONE JSON line.  value = total iterations / timed seconds (both solves
of every timed step); ms_per_step = time to residual 1e-6 for the KL + TV pair.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_GRID = 256
EPS, EPS0, TOL = 1e-3, 1e-1, 1e-6
PENALTIES = (("KL", 0.1), ("TV", 0.05))
MAX_ITER = 8000
PEAK_CLOCK_HZ = 2.4e9
N_CU = 256


def exp_peak():
    """v_exp_f32 issue peak from unit counts: 256 CUs x 4 SIMDs x 16 lanes x
    2.4 GHz, transcendentals at half the FP32 VALU rate on gfx950."""
    return N_CU * 64 * PEAK_CLOCK_HZ / 2.0


def cpu_baseline(prob_np, budget_s=15.0):
    """The FP64 oracle as it stands, on the same workload (KL solve from a cold
    start at the first eps stage), for a bounded number of iterations."""
    import numpy as np
    from oracle import uot_oracle as O
    G = O.GridGeom(prob_np.shape, prob_np.h)
    d = np.full(prob_np.size, prob_np.h[0] * prob_np.h[1])
    lp, lq, ld = np.log(prob_np.p), np.log(prob_np.q), np.log(d)
    F = O.KL(PENALTIES[0][1])
    O.solve(G, lp, lq, ld, ld, F, F, EPS0, tol=0.0, max_iter=1)      # warm caches
    it = 0
    t0 = time.perf_counter()
    v = None
    while time.perf_counter() - t0 < budget_s or it < 3:
        s = O.solve(G, lp, lq, ld, ld, F, F, EPS0, tol=0.0, max_iter=1, v0=v)
        v = s["v"]
        it += 1
    dt = time.perf_counter() - t0
    return dict(value=it / dt, unit="iters/s", cores=1, kind="oracle",
                sample="%d iterations of the KL solve on the 256x256 workload at eps=1e-1 "
                       "(numpy FP64, one thread), %.1f s" % (it, dt))


def warm_batched(U, ctx, dev, np, torch):
    """Warm+batched forms against the plain cold single-problem iteration:
    (a) ragged batch of 4096 point-cloud problems (N, M log-uniform on
        [64, 4096], uniform points in [0,1]^2, KL 1, eps 5e-3, tol 1e-6) in
        one persistent launch per half-step vs plain solves of a 16-problem
        sample (extrapolated);
    (b) unbalanced barycentre of 8 blob images at 128 x 128 (KL 0.5, eps 2e-3,
        tol 1e-6): plain = cold start with eps-scaling, warm = v^(0) from the
        trained network (no annealing)."""
    from paper_1607_05816_amd import synth, warmstart as W
    from paper_1607_05816_amd.train_warmstart import load_weights
    out = {}
    probs = synth.ragged_batch(0, B=4096)
    Ns = [p.x.shape[0] for p in probs]
    Ms = [p.y.shape[0] for p in probs]
    cat = lambda f: torch.tensor(np.concatenate([f(p) for p in probs]).astype(np.float32), device=dev)
    F = U.KL(1.0)
    bp = U.BatchProblem(Ns, Ms, cat(lambda p: p.x), cat(lambda p: p.y), cat(lambda p: p.p), cat(lambda p: p.q),
                        cat(lambda p: p.dx), cat(lambda p: p.dy), F, F)
    U.solve_batched(bp, 5e-3, tol=1e-6, max_iter=20000, check_every=50, ctx=ctx)       # tunes, warms
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = U.solve_batched(bp, 5e-3, tol=1e-6, max_iter=20000, check_every=50, ctx=ctx)
    torch.cuda.synchronize()
    bs = time.perf_counter() - t0
    it = info["iters"]
    pairs = np.array(Ns, float) * np.array(Ms, float)
    rng = np.random.default_rng(1)
    idx = rng.choice(len(probs), 16, replace=False)
    plain = 0.0
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    for k in idx:
        p = probs[k]
        pb = U.points_problem(T(p.x), T(p.y), T(p.p), T(p.q), T(p.dx), T(p.dy), F, F)
        pb.workspace()
        # untimed first solve: a shape's one-time product tuning stays out of
        # the plain time, as the batch's tuning stays out of the batched one
        U.solve(pb, 5e-3, tol=1e-6, max_iter=20000, check_every=50, ctx=ctx)
        torch.cuda.synchronize()
        a = time.perf_counter()
        U.solve(pb, 5e-3, tol=1e-6, max_iter=20000, check_every=50, ctx=ctx)
        torch.cuda.synchronize()
        plain += time.perf_counter() - a
    plain_per = plain / len(idx)
    out["ragged_batch_4096"] = {
        "converged": int(info["n_converged"]), "problems": len(probs), "seconds": bs,
        "problems_per_s": len(probs) / bs, "problem_iters_per_s": float(it.sum()) / bs,
        "pair_evals_per_s": float((pairs * it).sum()) * 2 / bs,
        "pair_evals_frac_of_exp_peak": float((pairs * it).sum()) * 2 / bs / exp_peak(),
        "latency_ms_p50": float(np.percentile(info["latency_ms"], 50)),
        "latency_ms_p99": float(np.percentile(info["latency_ms"], 99)),
        "tile_rows": info["tile_rows"], "blocks_per_cu": info["blocks_per_cu"],
        "product": {1: "direct", 4: "mfma_bf16x3"}.get(int(info["product"]), str(info["product"])),
        "plain_ms_per_problem_sample16": plain_per * 1e3,
        "speedup_vs_plain": plain_per * len(probs) / bs}
    net = load_weights(os.path.join(ROOT, "paper_1607_05816_amd", "data", "warmstart_mlp64.npz"), dev)
    pr = synth.bary_blobs(0, n_marg=8, n=128)
    p = torch.tensor(pr.p, dtype=torch.float32, device=dev)
    res = {}
    for name in ("plain_cold_eps_scaling", "warm"):
        for rep in range(2):
            torch.cuda.synchronize()
            a = time.perf_counter()
            if name == "warm":
                v0 = W.barycenter_v0(net, p, pr.alpha, 128, ctx=ctx)
                _, _, _, bi = W.barycenter_solve(p, pr.alpha, 128, v0=v0.contiguous(), ctx=ctx)
            else:
                _, _, _, bi = W.barycenter_solve(p, pr.alpha, 128, eps0=W.EPS0, ctx=ctx)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - a) * 1e3
        res[name] = {"iters": int(bi["iters"]), "ms": ms, "converged": bool(bi["converged"])}
    res["speedup"] = res["plain_cold_eps_scaling"]["ms"] / res["warm"]["ms"]
    out["barycenter_8x128"] = res
    return out


def extensions(U, pr, ctx, dev, np, torch):
    """Solves beyond the KL/TV pair, timed to tol 1e-6 (FP32, device-resident):
    (a) barycentres of 8 blob images at 128 x 128 with TV 0.1 and RG [0.7, 1.3]
        penalties on the barycentre side (Table estimatebary iii/iv), KL 0.5 on
        the input side, eps 1e-1 -> 2e-3;
    (b) Algorithm 4 on the 256 x 256 workload: optimal partial transport
        (dominations RG[0, 1] on both marginals, total mass fixed to 0.7 of the
        smaller marginal's mass), eps 1e-1 -> 1e-2."""
    from paper_1607_05816_amd import synth
    out = {}
    bb = synth.bary_blobs(0, n_marg=8, n=128)
    p = torch.tensor(bb.p, dtype=torch.float32, device=dev)
    d = torch.full((128 * 128,), bb.h[0] * bb.h[1], dtype=torch.float32, device=dev)
    for name, F2 in (("TV0.1", U.TV(0.1)), ("RG0.7-1.3", U.RG(0.7, 1.3))):
        for rep in range(2):
            torch.cuda.synchronize()
            a = time.perf_counter()
            _, _, _, bi = U.barycenter(bb.shape, bb.h, p, bb.alpha, d, d, U.KL(0.5), F2, 2e-3, eps0=1e-1, tol=1e-6,
                                       max_iter=20000, check_every=50, ctx=ctx)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - a) * 1e3
        out["barycenter_8x128_" + name] = {"iters": int(bi["iters"]), "ms": ms, "converged": bool(bi["converged"]),
                                           "iters_per_s": bi["iters"] / (ms * 1e-3)}
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    cw = pr.h[0] * pr.h[1]
    dd = np.full(pr.size, cw)
    m0 = 0.7 * min(pr.p.sum(), pr.q.sum()) * cw
    F = U.RG(0.0, 1.0)
    pb = U.grid_problem(pr.shape, pr.h, t(pr.p), t(pr.q), t(dd), t(dd), F, F)
    pb.workspace()
    for rep in range(2):
        torch.cuda.synchronize()
        a = time.perf_counter()
        u, v, lz, info = U.solve_mass(pb, U.EQ(), m0, 1e-2, eps0=1e-1, tol=1e-6, max_iter=20000, check_every=50,
                                      ctx=ctx)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - a) * 1e3
    out["partial_transport_256x256"] = {"iters": int(info["iters"]), "ms": ms, "converged": bool(info["converged"]),
                                        "iters_per_s": info["iters"] / (ms * 1e-3), "log_z": lz,
                                        "mass_target": float(m0)}
    return out


PASS_NAMES = ["k_grid_tf<false, 4>", "k_grid_tf<true, 4>"]

# HBM bytes per launch (calibrated FETCH_SIZE read + WRITE_SIZE written) of the
# two passes at both launch shapes, from the two counter runs of
# `bench.py --pmc-workload`; they hold for the kernel source they were taken
# on (sha256 of the pass's file and the headers it includes) and are reported
# as null otherwise.
TRAFFIC_SOURCES = ["uot_grid_tf.hip", "uot_epilogue.h", "uot_device.h", "uot_launch.h"]
TRAFFIC_SOURCE_SHA256 = "38bc0ed204173d6a9cc25effd79c3265698ce3347e6b5fafe54186552afeb729"
TRAFFIC_BYTES = {
    ('k_grid_tf<false, 4>', 1): (2273408, 259840),
    ('k_grid_tf<false, 4>', 256): (67287172, 67108864),
    ('k_grid_tf<true, 4>', 1): (3096797, 523671),
    ('k_grid_tf<true, 4>', 256): (406346152, 134348800),
}


def tf_source_sha256():
    import hashlib
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_1607_05816_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic(kernel, fields):
    """(bytes read, bytes written) per launch, or None once the kernel changed."""
    if tf_source_sha256() != TRAFFIC_SOURCE_SHA256:
        return None
    return TRAFFIC_BYTES.get((kernel, fields))


def exp2_executed_per_launch(lines, n, tpc=4):
    """exp2 instructions one tile-factored pass executes, counted from the
    kernel, per (line, 16-cell output tile): 16 column factors per tap tile,
    16 (1 + tpc) per chunk of tpc tap tiles for the online combination, 64
    for the Khat operands and 96 for merging the four waves."""
    nt = n // 16
    return float(lines) * nt * (nt * 16 + (nt // tpc) * 16 * (1 + tpc) + 64 + 96)


def grid_roofline(U, probs, last, ctx, torch, np, nb_fields=256):
    """Roofline of the dominant kernel: the two Gibbs-product passes of one X
    half-step at the final eps (KL problem, converged v), each launched back
    to back between two HIP events on the library stream.  Algorithmic work
    of a pass = one exp per tap, n1 n2 n taps per field (the separable
    product written as direct log-sum-exps), priced against the v_exp_f32
    issue peak.  Measured on the single 256 x 256 problem of the headline
    (latency-bound: 256 blocks, one per CU) and on a batch of nb_fields
    fields of the same size in one launch (throughput-bound)."""
    ms = U.time_half_step(probs[0][1], EPS, last[0][3], reps=200, ctx=ctx)
    k = int(np.argmax(ms))
    taps = float(N_GRID) ** 3
    peak = exp_peak()
    out = {"bound": "alu", "achieved": taps / (ms[k] * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "Texp/s",
           "frac": taps / (ms[k] * 1e-3) / peak, "traffic": None, "kernel": PASS_NAMES[k], "kernel_avg_ms": ms[k],
           "work_per_launch": taps, "work_unit": "exp (one per tap: n1 n2 n)",
           "exp2_executed_per_launch": exp2_executed_per_launch(N_GRID, N_GRID),
           "avg_ms_by_kernel": dict(zip(PASS_NAMES, ms)), "launch": "single 256x256 problem"}
    out["executed_exp2_frac"] = out["exp2_executed_per_launch"] / (ms[k] * 1e-3) / peak
    tr = traffic(PASS_NAMES[k], 1)
    if tr is not None:
        out["traffic"] = float(sum(tr))
        out["traffic_read_written"] = list(tr)
        # the X-side strided pass reads its input, log p, u_old, log dx and
        # writes u, w (4 B each per cell); the contiguous pass reads w, writes t
        out["traffic_algorithmic"] = float(N_GRID * N_GRID * 4 * (6 if k == 1 else 2))
    pb = probs[0][1]
    p = pb.p.reshape(1, -1).expand(nb_fields, -1).contiguous()
    v = last[0][3].reshape(1, -1).expand(nb_fields, -1).contiguous()
    h = (1.0 / N_GRID, 1.0 / N_GRID)
    msb = U.time_fields_half_step((N_GRID, N_GRID), h, p, pb.dx, pb.dy, U.KL(PENALTIES[0][1]), EPS, v, reps=20,
                                  ctx=ctx)
    kb = int(np.argmax(msb))
    tb = taps * nb_fields
    out["batched"] = {"fields": nb_fields, "kernel": PASS_NAMES[kb], "kernel_avg_ms": msb[kb],
                      "achieved": tb / (msb[kb] * 1e-3) / 1e12, "frac": tb / (msb[kb] * 1e-3) / peak,
                      "work_per_launch": tb, "avg_ms_by_kernel": dict(zip(PASS_NAMES, msb)),
                      "exp2_executed_per_launch": exp2_executed_per_launch(nb_fields * N_GRID, N_GRID)}
    out["batched"]["executed_exp2_frac"] = out["batched"]["exp2_executed_per_launch"] / (msb[kb] * 1e-3) / peak
    # the same launches with FP16 MFMA operands (grid_kernel 3, ~1e-3 relative)
    msh = U.time_fields_half_step((N_GRID, N_GRID), h, p, pb.dx, pb.dy, U.KL(PENALTIES[0][1]), EPS, v, reps=20,
                                  ctx=ctx, grid_kernel=U.GRID_MFMA16)
    kh = int(np.argmax(msh))
    out["batched_fp16"] = {"fields": nb_fields, "kernel": PASS_NAMES[kh] + " fp16", "kernel_avg_ms": msh[kh],
                           "achieved": tb / (msh[kh] * 1e-3) / 1e12, "frac": tb / (msh[kh] * 1e-3) / peak,
                           "avg_ms_by_kernel": dict(zip(PASS_NAMES, msh))}
    trb = traffic(PASS_NAMES[kb], nb_fields)
    out["batched"]["traffic"] = None if trb is None else float(sum(trb))
    del p, v
    torch.cuda.empty_cache()
    return out


DENSE_KERNELS = ((1, "direct", "k_dense_lse<float, 3, 2, 0>"), (2, "tile_factored", "k_dense_tf<3, 2>"),
                 (3, "mfma_fp32", "k_dense_mf<3, 4, false>"), (4, "mfma_bf16x3", "k_dense_mf<3, 4, true>"))


def dense_roofline(U, torch, np, dev, ctx, n=20000, eps=1e-3):
    """Dense point-cloud product (3-D clouds, N = M = 20000, 8-component
    mixtures, FP32 data): the column-split log-sum-exp kernel of one X
    half-step, launched back to back between HIP events, for each product
    kernel (the default is the BF16 x 3 matrix-core one).  Algorithmic work:
    one exp per pair (N M per launch), priced against the v_exp_f32 issue
    peak; with one add per pair beside it the vector units cap a kernel at
    2/3 of that peak."""
    from paper_1607_05816_amd import synth
    pr = synth.clouds3d(0, N=n, M=n)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    F = U.KL(1.0)
    pb = U.points_problem(T(pr.x), T(pr.y), T(pr.p), T(pr.q), T(pr.dx), T(pr.dy), F, F)
    pb.workspace()
    v = torch.zeros(n, dtype=torch.float32, device=dev)
    pairs = float(n) * n
    peak = exp_peak()
    by = {}
    for k, name, kern in DENSE_KERNELS:
        ms = U.time_half_step(pb, eps, v, reps=20, ctx=ctx, grid_kernel=k)
        by[name] = {"kernel": kern, "kernel_avg_ms": ms[0], "merge_epilogue_ms": ms[1],
                    "frac": pairs / (ms[0] * 1e-3) / peak}
    d = by["mfma_bf16x3"]
    return {"bound": "alu", "kernel": d["kernel"], "kernel_avg_ms": d["kernel_avg_ms"],
            "achieved": pairs / (d["kernel_avg_ms"] * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "Texp/s",
            "frac": d["frac"], "work_per_launch": pairs, "work_unit": "exp (one per pair)",
            "epilogue_ms": d["merge_epilogue_ms"], "by_kernel": by,
            "workload": "clouds3d N=M=%d eps=%g FP32, v = 0" % (n, eps)}


def dense_solve(U, torch, np, dev, ctx, n=20000):
    """The dense configuration end to end: N = M = 20000 3-D mixture clouds,
    KL 1, eps 1e-1 -> 1e-3 (10 stages of 100 iterations, then on), FP32 data.
    The default (matrix-core) product runs to residual 1e-6 (time to
    residual); both it and the direct product run a fixed 3000 iterations
    (iterations/s), and their potentials are compared."""
    from paper_1607_05816_amd import synth
    pr = synth.clouds3d(0, N=n, M=n)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    F = U.KL(1.0)
    pb = U.points_problem(T(pr.x), T(pr.y), T(pr.p), T(pr.q), T(pr.dx), T(pr.dy), F, F)
    pb.workspace()
    out = {"workload": "clouds3d N=M=%d KL1 eps 1e-1->1e-3 10x100 FP32" % n}
    pots = {}
    for k, name in ((0, "default_mfma_bf16x3"), (1, "direct")):
        U.solve(pb, 1e-3, eps0=1e-1, tol=0.0, max_iter=300, check_every=50, ctx=ctx, dense_kernel=k)   # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, v, info = U.solve(pb, 1e-3, eps0=1e-1, tol=0.0, max_iter=3000, check_every=50, ctx=ctx,
                             dense_kernel=k)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        pots[name] = (u.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64))
        out[name] = {"seconds": dt, "iters": int(info["iters"]), "iters_per_s": info["iters"] / dt,
                     "residual": float(info["residual"])}
    (u1, v1), (u2, v2) = pots["default_mfma_bf16x3"], pots["direct"]
    sc = max(np.abs(u2).max(), np.abs(v2).max())
    out["max_potential_diff_rel"] = float(max(np.abs(u1 - u2).max(), np.abs(v1 - v2).max()) / sc)
    out["speedup_vs_direct"] = out["direct"]["seconds"] / out["default_mfma_bf16x3"]["seconds"]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, _, info = U.solve(pb, 1e-3, eps0=1e-1, tol=1e-6, max_iter=40000, check_every=50, ctx=ctx)
    torch.cuda.synchronize()
    out["time_to_residual_1e-6"] = {"seconds": time.perf_counter() - t0, "iters": int(info["iters"]),
                                    "converged": bool(info["converged"]), "residual": float(info["residual"])}
    return out


def wf_dense_roofline(U, torch, np, dev, ctx, n=20000, cut=0.1, eps=1e-3):
    """Dense product with the WF cost and cut locus 0.1 (2-D clustered clouds,
    N = M = 20000, FP32): the same launch timed on Morton-ordered clouds (tiles
    beyond the cut skipped), on the same clouds shuffled (nothing skippable),
    and with the squared Euclidean cost.  Algorithmic work: the pairs within
    the cut (the non-zero kernel entries), each one exp and one log, priced at
    half the transcendental issue peak."""
    from paper_1607_05816_amd import synth
    cp = synth.clusters_sorted(0, N=n, M=n, d=2)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    rng = np.random.default_rng(0)
    # pairs within the cut: exact count by rows in chunks
    inside = 0
    for a in range(0, n, 2000):
        d2 = ((cp.x[a:a + 2000, None, :] - cp.y[None, :, :]) ** 2).sum(-1)
        inside += int((d2 < cut * cut).sum())
    F = U.KL(1.0)
    v = torch.zeros(n, dtype=torch.float32, device=dev)
    out = {}
    perm = rng.permutation(n)
    for name, x, y, cost in (("sorted", cp.x, cp.y, U.WF(cut)), ("shuffled", cp.x[perm], cp.y[perm], U.WF(cut)),
                             ("sqeuclid", cp.x, cp.y, U.SQEUCLID)):
        pb = U.points_problem(T(x), T(y), T(cp.p), T(cp.q), T(cp.dx), T(cp.dy), F, F, cost=cost)
        pb.workspace()
        out[name + "_ms"] = U.time_half_step(pb, eps, v, reps=20, ctx=ctx)[0]
    peak = exp_peak() / 2
    ms = out["sorted_ms"]
    out.update({"bound": "alu", "kernel": "k_dense_lse<float, 2, 1, 1>", "kernel_avg_ms": ms,
                "achieved": inside / (ms * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "Tpairs/s",
                "frac": inside / (ms * 1e-3) / peak, "work_per_launch": float(inside),
                "work_unit": "pair within the cut (one exp + one log)", "pairs_within_cut_frac": inside / float(n) ** 2,
                "dense_pairs_per_s_equivalent": float(n) ** 2 / (ms * 1e-3),
                "workload": "clusters_sorted 2-D N=M=%d, WF cut %g, eps %g, FP32" % (n, cut, eps)})
    return out


def flows_bench(U, torch, np, dev, ctx, steps=10):
    """The gradient-flow experiments' shapes (Sec. 5.3): [0, 1] in 3000 cells,
    WF cost (cut pi/2 beyond the segment), 500 iterations per step, FP64
    (eps 1e-8 / 1e-7 puts potentials / eps near 1e8): the tumour growth flow
    (tau 0.006, alpha 1, eps 1e-8) and two species (tau 0.004, alpha 1,
    eps 1e-7), `steps` steps each, densities kept on the device."""
    from paper_1607_05816_amd import synth
    n = 3000
    out = {}
    for name, species, tau, eps in (("growth_1species", 1, 0.006, 1e-8), ("growth_2species", 2, 0.004, 1e-7)):
        p0 = torch.tensor(synth.growth_profile_1d(0, n, species=species), dtype=torch.float64, device=dev)
        q = torch.ones(n, dtype=torch.float64, device=dev)
        dx = torch.full((n,), 1.0 / n, dtype=torch.float64, device=dev)
        U.flow("growth", p0, q, dx, tau, eps, 1, shape=(n,), h=(1.0 / n,), alpha=1.0, cost=U.WF(math.pi / 2),
               tol=0.0, max_iter=500, check_every=50, ctx=ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dens, v, st, info = U.flow("growth", p0, q, dx, tau, eps, steps, shape=(n,), h=(1.0 / n,), alpha=1.0,
                                   cost=U.WF(math.pi / 2), tol=0.0, max_iter=500, check_every=50, ctx=ctx)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        mass = (dens.sum(dim=(1, 2)) / n).cpu().numpy()
        out[name] = {"steps": steps, "iters_per_step": 500, "ms_per_step": dt / steps * 1e3,
                     "iters_per_s": steps * 500 / dt, "mass_first_last": [float(mass[0]), float(mass[-1])],
                     "max_density_last": float(dens[-1].sum(0).max()), "dtype": "f64"}
    return out


def colour_transfer_bench(U, torch, np, dev, ctx):
    """The colour-transfer experiment's configuration (Sec. 5.1): 64 x 32 x 32
    colour bins of [0, 1]^3 with unit reference mass, synthetic image
    histograms, F1 = equality and F2 = 0.03 KL / RG[0, 5] / 0.2 TV, eps = 2e-3,
    2000 iterations (as in the paper, no tolerance), FP32, then the barycentric
    projection map; times include the device synchronisation."""
    from paper_1607_05816_amd import synth
    shape, h = (64, 32, 32), (1 / 64, 1 / 32, 1 / 32)
    cp = synth.colour_histograms(0, shape=shape)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    one = t(np.ones(cp.p.size))
    out = {}
    for name, F2 in (("KL0.03", U.KL(0.03)), ("RG0-5", U.RG(0.0, 5.0)), ("TV0.2", U.TV(0.2))):
        pb = U.grid_problem(shape, h, t(cp.p), t(cp.q), one, one, U.EQ(), F2)
        pb.workspace()
        for rep in range(2):
            torch.cuda.synchronize()
            a = time.perf_counter()
            u, v, info = U.solve(pb, 2e-3, tol=0.0, max_iter=2000, check_every=100, ctx=ctx)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - a) * 1e3
            a = time.perf_counter()
            T = U.barycentric_map(pb, 2e-3, v, ctx=ctx)
            torch.cuda.synchronize()
            ms_map = (time.perf_counter() - a) * 1e3
        out[name] = {"iters": int(info["iters"]), "ms": ms, "ms_per_iter": ms / info["iters"], "map_ms": ms_map,
                     "map_finite": bool(torch.isfinite(T).all().item())}
    out["workload"] = "64x32x32 colour bins, dx = dy = 1, F1 = equality, eps 2e-3, 2000 iterations, FP32"
    return out


def pmc_workload(U, torch, np, dev, ctx):
    """The launches the HBM-traffic counters are read on (rocprofv3 --pmc
    FETCH_SIZE, then WRITE_SIZE): a plain device copy of 256 MiB (the
    calibration kernel of known size), then the two passes of one X
    half-step on the headline field (single launch shape) and on a batch of
    256 such fields."""
    from paper_1607_05816_amd import synth
    src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    pr = synth.blobs2d(0, n=N_GRID)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    d = np.full(pr.size, pr.h[0] * pr.h[1])
    F = U.KL(PENALTIES[0][1])
    pb = U.grid_problem(pr.shape, pr.h, t(pr.p), t(pr.q), t(d), t(d), F, F)
    u, v, info = U.solve(pb, EPS, eps0=EPS0, tol=TOL, max_iter=MAX_ITER, check_every=50, ctx=ctx)
    U.time_half_step(pb, EPS, v, reps=20, ctx=ctx)
    nb = 256
    p = pb.p.reshape(1, -1).expand(nb, -1).contiguous()
    vb = v.reshape(1, -1).expand(nb, -1).contiguous()
    U.time_fields_half_step((N_GRID, N_GRID), pr.h, p, pb.dx, pb.dy, F, EPS, vb, reps=5, ctx=ctx)
    torch.cuda.synchronize()
    print("pmc workload done", flush=True)


def pmc_workload_dense(U, torch, np, dev, ctx, n=20000):
    """The launches the dense products' instruction counters are read on:
    three back-to-back launches of each product kernel on one X half-step of
    the 20000^2 3-D mixture clouds (eps 1e-3, v = 0), as in roofline_dense."""
    from paper_1607_05816_amd import synth
    pr = synth.clouds3d(0, N=n, M=n)
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    F = U.KL(1.0)
    pb = U.points_problem(T(pr.x), T(pr.y), T(pr.p), T(pr.q), T(pr.dx), T(pr.dy), F, F)
    v = torch.zeros(n, dtype=torch.float32, device=dev)
    for k, _, _ in DENSE_KERNELS:
        U.time_half_step(pb, 1e-3, v, reps=3, ctx=ctx, grid_kernel=k)
    torch.cuda.synchronize()
    print("pmc dense workload done", flush=True)


BF16_MFMA_PEAK = 2.5e15     # MI355X dense BF16 MFMA, FLOP/s


def gemm_roofline(U, torch, np, dev, ctx, batch=256):
    """Training GEMMs of the warm-start net (8192 -> 256 -> 256 -> 256 -> 4096,
    BF16 operands, FP32 accumulation) at batch 256: the four largest products
    of one Adam step, each launched back to back between HIP events, priced
    against the dense BF16 MFMA peak; plus the whole training step (forward,
    loss, backward, Adam) timed over 20 steps."""
    g = torch.Generator(device="cpu")
    g.manual_seed(0)
    rnd = lambda *s: U.bf16_bits(torch.randn(*s, generator=g).to(dev)).contiguous()
    shapes = [("forward layer 1", False, True, batch, 256, 8192), ("backward dh layer 4", False, False, batch, 256, 4096),
              ("backward dW layer 1", True, False, 256, 8192, batch), ("forward layer 4", False, True, batch, 4096, 256)]
    out = {"bound": "mfma", "peak": BF16_MFMA_PEAK / 1e12, "unit": "TFLOP/s", "gemms": []}
    for name, ta, tb, M, N, K in shapes:
        A = rnd(K, M) if ta else rnd(M, K)
        B = rnd(N, K) if tb else rnd(K, N)
        ms = U.time_gemm_bf16(A, B, M, N, K, ta=ta, tb=tb, reps=20, ctx=ctx)
        fl = 2.0 * M * N * K
        out["gemms"].append({"name": name, "M": M, "N": N, "K": K, "ms": ms, "achieved": fl / (ms * 1e-3) / 1e12,
                             "frac": fl / (ms * 1e-3) / BF16_MFMA_PEAK})
    net = U.WarmStartNet(8192, 256, 4096, dev, seed=0)
    x = torch.randn(batch, 8192, generator=g).to(dev)
    t = torch.randn(batch, 4096, generator=g).to(dev) * 0.1
    for _ in range(3):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(20):
        net.train_step(x, t, 1e-4)
    torch.cuda.synchronize()
    step_ms = (time.perf_counter() - t0) / 20 * 1e3
    step_flops = 3 * 2.0 * batch * (8192 * 256 + 2 * 256 * 256 + 256 * 4096)
    out["train_step"] = {"batch": batch, "ms": step_ms, "achieved": step_flops / (step_ms * 1e-3) / 1e12,
                         "frac": step_flops / (step_ms * 1e-3) / BF16_MFMA_PEAK}
    return out


def mixed_precision(U, probs, last, ctx, torch, reps=3):
    """The headline solves with grid_kernel 4 (FP16 MFMA operands until the
    residual reaches 1e-4, FP32 operands down to 1e-6): time to residual 1e-6,
    iterations, and the largest deviation of v from the FP32 solve of the
    timed steps (relative to max(|v|, eps)).  Reported beside the FP32
    headline, not in place of it."""
    out = {}
    tot_it, tot_ms = 0, 0.0
    for (name, pb), (_, _, _, v32) in zip(probs, last):
        U.solve(pb, EPS, eps0=EPS0, tol=TOL, max_iter=MAX_ITER, check_every=50, ctx=ctx, grid_kernel=U.GRID_MIXED)
        best = None
        for _ in range(reps):
            u, v, info = U.solve(pb, EPS, eps0=EPS0, tol=TOL, max_iter=MAX_ITER, check_every=50, ctx=ctx,
                                 grid_kernel=U.GRID_MIXED)
            if best is None or info["elapsed_ms"] < best[0]["elapsed_ms"]:
                best = (info, v)
        info, v = best
        dv = float((v - v32).abs().max()) / max(float(v32.abs().max()), EPS)
        out[name] = {"time_to_residual_ms": info["elapsed_ms"], "iters": info["iters"], "converged": info["converged"],
                     "v_rel_dev_vs_fp32": dv}
        tot_it += info["iters"]
        tot_ms += info["elapsed_ms"]
    out["iters_per_s"] = tot_it / (tot_ms * 1e-3)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-warm-batched", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-gemm", action="store_true")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--pmc-workload", nargs="?", const="grid", choices=("grid", "dense"),
                    help="only run the launches counters are read on: the grid passes (HBM traffic) or "
                         "the dense products at 20000^2 (instruction counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1607_05816_amd import synth
    from paper_1607_05816_amd import uot as U

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda:0")
    if args.pmc_workload == "grid":
        pmc_workload(U, torch, np, dev, U.default_context())
        return
    if args.pmc_workload == "dense":
        pmc_workload_dense(U, torch, np, dev, U.default_context())
        return
    pr = synth.blobs2d(args.seed, n=N_GRID)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    d = np.full(pr.size, pr.h[0] * pr.h[1])
    probs = []
    for name, lam in PENALTIES:
        F = U.KL(lam) if name == "KL" else U.TV(lam)
        probs.append((name, U.grid_problem(pr.shape, pr.h, t(pr.p), t(pr.q), t(d), t(d), F, F)))
    ctx = U.default_context()
    for _, pb in probs:
        pb.workspace()

    def step():
        out = []
        for name, pb in probs:
            u, v, info = U.solve(pb, EPS, eps0=EPS0, tol=TOL, max_iter=MAX_ITER, check_every=50, ctx=ctx)
            obj = U.objective(pb, EPS, u, v, ctx=ctx)
            out.append((name, info, obj, v))
        return out

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    last = None
    for _ in range(args.steps):
        last = step()
        iters += sum(o[1]["iters"] for o in last)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    converged = all(o[1]["converged"] for o in last)

    roofline = grid_roofline(U, probs, last, ctx, torch, np)
    mixed = mixed_precision(U, probs, last, ctx, torch)
    line = {
        "metric": "Sinkhorn iters/s and time-to-residual 1e-6 (2-D grid 256x256, KL+TV, eps 1e-1->1e-3)",
        "value": iters / dt,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian-blob densities)",
        "config": {"workload": "grid2d-256x256-blobs5-KL0.1+TV0.05-eps1e-1to1e-3-10x100-tol1e-6",
                   "grid": [N_GRID, N_GRID], "eps": EPS, "eps0": EPS0, "tol": TOL, "seed": args.seed,
                   "parallelism": "single-gpu"},
        "time_to_residual_ms": {o[0]: o[1]["elapsed_ms"] for o in last},
        "iters_per_solve": {o[0]: o[1]["iters"] for o in last},
        "converged": converged,
        "gap": {o[0]: o[2]["gap"] for o in last},
        "roofline": roofline,
        "mixed_fp16_fp32": mixed,
    }
    if not args.no_dense:
        line["roofline_dense"] = dense_roofline(U, torch, np, dev, ctx)
        line["dense_solve"] = dense_solve(U, torch, np, dev, ctx)
    if not args.no_gemm:
        line["roofline_gemm"] = gemm_roofline(U, torch, np, dev, ctx)
    if not args.no_extensions:
        line["extensions"] = extensions(U, pr, ctx, dev, np, torch)
        line["extensions"]["roofline_wf_dense"] = wf_dense_roofline(U, torch, np, dev, ctx)
        line["extensions"]["gradient_flows"] = flows_bench(U, torch, np, dev, ctx)
        line["extensions"]["colour_transfer"] = colour_transfer_bench(U, torch, np, dev, ctx)
    if not args.no_warm_batched:
        line["warm_batched_vs_plain"] = warm_batched(U, ctx, dev, np, torch)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pr, args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
