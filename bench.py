#!/usr/bin/env python
"""Benchmark: Sinkhorn iterations per second and time to residual 1e-6 of the
generalized scaling iteration on one MI355X, warm+batched against plain.

Headline workload (one "step" = one pass of the whole hot path over one
batch): 4096 independent unbalanced OT problems between point clouds of
uneven size (N, M log-uniform on [64, 4096], uniform points in [0,1]^2,
densities U[0.1, 1] w.r.t. dx = 1/N, squared Euclidean cost, KL lambda = 1
on both marginals, eps = 5e-3, FP32; seeded synthetic inputs).  A step is
the learned warm start of every problem (features from batched Gibbs
products, the network, v^(0)) followed by one batched solve of all 4096
problems to residual 1e-6 (persistent launches over an atomic work cursor,
captured in hipGraph chunks).  Plain = the cold single-problem solver, one
problem after another (a stratified sample, extrapolated).

Prints ONE JSON line.  value = problems brought to residual 1e-6 per second
by the warm+batched form (whole job); ms_per_step = its time to residual 1e-6
for the whole batch.  Beside it: Sinkhorn iterations per second, the plain
and cold-batched times and speedups, the roofline of the dominant kernel
(the batched matrix-core product), the oracle's CPU baseline on the same
workload, and the other workloads (the 2-D grid, dense clouds, the
barycentre warm start, training GEMMs, extensions).
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


RAGGED_B, RAGGED_EPS = 4096, 5e-3
# the warm+batched form balances each problem's constant again at this
# iteration, once the shape of v has settled (any iteration from 15 to 100
# gives the same count on the bench batch)
RAGGED_REBALANCE = 30


def _oracle_iter_seconds(prob, eps, iters):
    """Seconds per iteration of the FP64 oracle on one problem (cold start)."""
    import numpy as np
    from oracle import uot_oracle as O
    g = O.PointsGeom(prob.x, prob.y)
    F = O.KL(1.0)
    args = (g, np.log(prob.p), np.log(prob.q), np.log(prob.dx), np.log(prob.dy), F, F, eps)
    t = time.perf_counter()
    O.solve(*args, tol=0.0, max_iter=iters)
    return (time.perf_counter() - t) / iters


_CPU_PROBS = None      # the sampled problems, inherited by the forked workers


def _oracle_worker(job):
    idxs, eps, iters = job
    return [(k, _oracle_iter_seconds(_CPU_PROBS[k], eps, iters)) for k in idxs]


def cpu_sample(seed=0, n_sample=64, iters=20):
    """The FP64 oracle as it stands on a stratified sample of the ragged
    workload: every (B / n_sample)-th problem in order of N M, `iters`
    iterations each, timed on one thread and then on every core the process
    may run on (os.sched_getaffinity; one worker process per core, the
    problems split between them).  Runs before the GPU is touched (the worker
    processes are forked).  Returns per-problem seconds per iteration and the
    wall times."""
    import multiprocessing as mp
    import numpy as np
    from paper_1607_05816_amd import synth
    sizes = synth.ragged_sizes(seed, B=RAGGED_B)
    order = np.argsort(np.asarray(sizes[0], float) * np.asarray(sizes[1], float), kind="stable")
    step = len(order) // n_sample
    idx = [int(order[step // 2 + k * step]) for k in range(n_sample)]
    global _CPU_PROBS
    probs = synth.ragged_batch(seed, B=RAGGED_B)
    _CPU_PROBS = {k: probs[k] for k in idx}
    _oracle_iter_seconds(probs[idx[0]], RAGGED_EPS, 2)                      # warm caches
    t = time.perf_counter()
    one = {k: _oracle_iter_seconds(probs[k], RAGGED_EPS, iters) for k in idx}
    wall1 = time.perf_counter() - t
    cores = len(os.sched_getaffinity(0))
    workers = max(1, min(cores, n_sample))
    # one job per problem, largest first, handed out as workers free up
    jobs = [([k], RAGGED_EPS, iters) for k in sorted(idx, key=lambda k: -one[k])]
    ctx = mp.get_context("fork")
    with ctx.Pool(workers) as pool:
        pool.map(_oracle_worker, [([idx[0]], RAGGED_EPS, 1)] * workers)   # start-up
        t = time.perf_counter()
        par = dict(kv for part in pool.imap_unordered(_oracle_worker, jobs, chunksize=1) for kv in part)
        wallN = time.perf_counter() - t
    return dict(idx=idx, order=order, step=step, one=one, par=par, wall1=wall1, wallN=wallN, cores=cores,
                workers=workers, iters=iters)


def cpu_baseline_ragged(cs, iters_cold, Ns, Ms):
    """Extrapolate the oracle's sample to the whole workload: every problem
    takes the per-iteration time of the sampled problem of its size stratum
    (the same stratum of N M order), times its own iteration count to
    residual 1e-6 (the GPU's count for the same cold iteration).  One thread:
    the sum of those times; all cores: that sum scaled by the sample's
    measured parallel speed-up."""
    import numpy as np
    order, step = cs["order"], cs["step"]
    strat = {}
    for rank, b in enumerate(order):
        strat[int(b)] = cs["idx"][min(rank // step, len(cs["idx"]) - 1)]
    t1 = sum(cs["one"][strat[b]] * float(iters_cold[b]) for b in range(len(order)))
    sample_work = sum(cs["one"][k] * cs["iters"] for k in cs["idx"])
    speedup = sample_work / cs["wallN"]
    tN = t1 / speedup
    return {"value": len(order) / tN, "unit": "problems/s to residual 1e-6", "cores": cs["workers"], "kind": "oracle",
            "sample": "FP64 numpy oracle, %d problems of the 4096 (one per N*M stratum, every %d-th in size order), "
                      "%d iterations each, %.1f s on one thread and %.1f s on %d worker processes (affinity %d "
                      "cores); extrapolated by the GPU's cold iteration count of every problem"
                      % (len(cs["idx"]), step, cs["iters"], cs["wall1"], cs["wallN"], cs["workers"], cs["cores"]),
            "one_thread": {"value": len(order) / t1, "seconds_to_residual": t1},
            "seconds_to_residual": tN, "parallel_speedup_of_sample": speedup}


def ragged_headline(U, ctx, dev, np, torch, steps, warmup):
    """The headline: warm start + batched solve of the 4096-problem ragged
    workload to residual 1e-6, against the cold batched solve and the plain
    cold single-problem solver."""
    from paper_1607_05816_amd import cloud_warmstart as CW
    if not os.path.exists(CW.WEIGHTS):
        raise RuntimeError("the trained cloud warm start is missing: %s" % CW.WEIGHTS)
    cw = CW.CloudWarmStart.load(CW.WEIGHTS, dev)
    probs = CW.ragged(0, B=RAGGED_B)
    Ns = np.array([p.x.shape[0] for p in probs], float)
    Ms = np.array([p.y.shape[0] for p in probs], float)
    pairs = Ns * Ms
    bp = CW.batch_problem(probs, dev)
    bp.workspace()

    def step():
        v0 = cw.v0(bp, ctx=ctx)
        return CW.solve(bp, v0=v0, ctx=ctx, rebalance_at=RAGGED_REBALANCE)[2]

    CW.solve(bp, ctx=ctx)                # the batch signature's one-time product tuning
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    infos = [step() for _ in range(steps)]
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    warm = infos[-1]
    it_warm = warm["iters"].astype(float)
    # warm start alone (features, network, v0)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(3):
        cw.v0(bp, ctx=ctx)
    torch.cuda.synchronize()
    ws_ms = (time.perf_counter() - t) / 3 * 1e3
    # cold batched
    cold_s = []
    for _ in range(2):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, cold = CW.solve(bp, ctx=ctx)
        torch.cuda.synchronize()
        cold_s.append(time.perf_counter() - t)
    it_cold = cold["iters"].astype(float)
    # the warm start's parts (start included in the time): the mass balance
    # without the network (at the start and again at RAGGED_REBALANCE), the
    # network without any balance, and the network with the balance at the
    # start only
    ablation = {}
    for name, start, reb in (("balance_only", lambda: CW.balanced_cold_v0(bp, ctx=ctx), RAGGED_REBALANCE),
                             ("network_only", lambda: cw.v0(bp, ctx=ctx, balance=False), 0),
                             ("no_rebalance", lambda: cw.v0(bp, ctx=ctx), 0)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        _, _, inf = CW.solve(bp, v0=start(), ctx=ctx, rebalance_at=reb)
        torch.cuda.synchronize()
        ablation[name] = {"seconds": time.perf_counter() - t, "iters_mean": float(inf["iters"].mean()),
                          "converged": int(inf["n_converged"]), "rebalance_at": reb}
    # plain: cold single-problem solves of a stratified sample (one per
    # N*M stratum), each after an untimed first solve of its shape (the
    # product tuning, kept out as the batch's tuning is)
    order = np.argsort(pairs, kind="stable")
    n_plain = 64
    stp = len(order) // n_plain
    sample = [int(order[stp // 2 + k * stp]) for k in range(n_plain)]
    T = lambda a: torch.tensor(np.asarray(a, np.float32), device=dev)
    F = U.KL(1.0)
    plain = []
    for k in sample:
        p = probs[k]
        pb = U.points_problem(T(p.x), T(p.y), T(p.p), T(p.q), T(p.dx), T(p.dy), F, F, layout="nd")
        pb.workspace()
        U.solve(pb, RAGGED_EPS, tol=1e-6, max_iter=20000, check_every=50, ctx=ctx)
        torch.cuda.synchronize()
        a = time.perf_counter()
        _, _, pi = U.solve(pb, RAGGED_EPS, tol=1e-6, max_iter=20000, check_every=50, ctx=ctx)
        torch.cuda.synchronize()
        plain.append(time.perf_counter() - a)
    plain_s = float(np.mean(plain)) * len(probs)
    # roofline of the batched product: one warm solve with every launch
    # between HIP events on the library stream (no graphs)
    v0 = cw.v0(bp, ctx=ctx)
    _, _, tk = CW.solve(bp, v0=v0, ctx=ctx, time_kernels=True, rebalance_at=RAGGED_REBALANCE)
    it_tk = tk["iters"].astype(float)
    launches = tk["kernel_launches"][0] + tk["kernel_launches"][1]
    kms = tk["kernel_ms"][0] + tk["kernel_ms"][1]
    work = 2.0 * float((pairs * it_tk).sum())          # pair evaluations, both half-steps
    avg_ms = kms / launches
    peak = exp_peak()
    kname = {1: "k_batch_lse", 4: "k_batch_mf"}.get(int(tk["product"]), str(tk["product"]))
    executed = float(tk["kernel_launches"][3])   # exp2 the matrix-core product issued (tiles left out)
    roof = {"bound": "alu", "kernel": kname, "kernel_avg_ms": avg_ms, "launches": int(launches),
            "work_per_launch": work / launches, "work_unit": "exp (one per pair; both half-steps)",
            "achieved": work / launches / (avg_ms * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "Texp/s",
            "frac": work / launches / (avg_ms * 1e-3) / peak,
            "exp_executed_per_launch": executed / launches if executed else None,
            "frac_executed": executed / launches / (avg_ms * 1e-3) / peak if executed else None,
            "traffic": None,
            "product_ms_total": kms, "control_ms_total": tk["kernel_ms"][2],
            "note": "average over every product launch of a warm solve (stopped problems leave the item lists)"}
    tr = batch_traffic(kname, int(tk["tile_rows"]))
    if tr is not None:
        # counters were read on full launches; the average launch carries
        # work_per_launch pairs, and the bytes scale with the pairs
        per_pair = (tr[0] + tr[1]) / tr[2]
        roof["traffic"] = per_pair * work / launches
        roof["traffic_full_launch"] = {"read": tr[0], "written": tr[1], "pairs": tr[2]}
        roof["traffic_note"] = "calibrated FETCH_SIZE + WRITE_SIZE of full launches, scaled by pairs"
    return {
        "value": len(probs) * steps / dt,
        "ms_per_step": dt / steps * 1e3,
        "warm": {"seconds": dt / steps, "iters_mean": float(it_warm.mean()), "iters_total": int(it_warm.sum()),
                 "converged": int(warm["n_converged"]), "warm_start_ms": ws_ms,
                 "problem_iters_per_s": float(it_warm.sum()) / (dt / steps),
                 "pair_evals_per_s": 2.0 * float((pairs * it_warm).sum()) / (dt / steps),
                 "latency_ms_p50": float(np.percentile(warm["latency_ms"], 50)),
                 "latency_ms_p99": float(np.percentile(warm["latency_ms"], 99)),
                 "product": kname, "tile_rows": int(warm["tile_rows"]), "blocks_per_cu": int(warm["blocks_per_cu"]),
                 "rebalance_at": RAGGED_REBALANCE},
        "cold_batched": {"seconds": min(cold_s), "iters_mean": float(it_cold.mean()),
                         "iters_total": int(it_cold.sum()), "converged": int(cold["n_converged"]),
                         "problem_iters_per_s": float(it_cold.sum()) / min(cold_s)},
        "plain": {"seconds_extrapolated": plain_s, "sample": n_plain, "ms_per_problem_mean": float(np.mean(plain)) * 1e3,
                  "kind": "cold single-problem solves, one after another"},
        "speedup_vs_plain": plain_s / (dt / steps),
        "speedup_batched_cold_vs_plain": plain_s / min(cold_s),
        "speedup_warm_vs_cold_batched": min(cold_s) / (dt / steps),
        "warm_start_parts": ablation,
        "iters_ratio_cold_over_warm": float(it_cold.sum() / it_warm.sum()),
        "roofline": roof,
        "iters_cold": it_cold,
    }


def warm_bary(U, ctx, dev, np, torch, seeds=(0, 1)):
    """The barycentre configuration: 8 blob images at 128 x 128, KL 0.5 on
    both sides, eps 2e-3, residual 1e-6.  Starts compared on the same
    schedule where they can be: cold with the paper's eps-scaling, cold
    without annealing (v^(0) = 0), the local estimate (no network, no
    annealing) and the network (no annealing); iterations and time to
    residual 1e-6 per seed, best of two runs."""
    from paper_1607_05816_amd import synth, warmstart as W
    from paper_1607_05816_amd.train_warmstart import load_weights
    net = load_weights(os.path.join(ROOT, "paper_1607_05816_amd", "data", "warmstart_mlp64.npz"), dev)
    out = {"workload": "barycentre of 8 blob images 128x128, KL 0.5, eps 2e-3, tol 1e-6, FP32"}
    for seed in seeds:
        pr = synth.bary_blobs(seed, n_marg=8, n=128)
        p = torch.tensor(pr.p, dtype=torch.float32, device=dev)
        res = {}
        for name in ("cold_eps_scaling", "cold", "local", "net"):
            best = None
            for rep in range(2):
                torch.cuda.synchronize()
                a = time.perf_counter()
                if name == "net":
                    v0 = W.barycenter_v0(net, p, pr.alpha, 128, ctx=ctx)
                elif name == "local":
                    v0 = W.barycenter_local_v0(p, pr.alpha, 128, ctx=ctx)
                else:
                    v0 = None
                _, _, _, bi = W.barycenter_solve(p, pr.alpha, 128, v0=v0, ctx=ctx,
                                                 eps0=W.EPS0 if name == "cold_eps_scaling" else None)
                torch.cuda.synchronize()
                ms = (time.perf_counter() - a) * 1e3
                if best is None or ms < best["ms"]:
                    best = {"iters": int(bi["iters"]), "ms": ms, "converged": bool(bi["converged"])}
            res[name] = best
        base = min(res["cold"]["iters"], res["local"]["iters"])
        res["net_iters_gain_vs_best_non_net"] = base / res["net"]["iters"]
        out["seed%d" % seed] = res
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
TRAFFIC_SOURCE_SHA256 = "d9b3651b18eab72e4f6947301386994449ffd7a674a62e3dfb3e752cbb12d178"
TRAFFIC_BYTES = {
    ('k_grid_tf<false, 4>', 1): (2251937, 259840),
    ('k_grid_tf<false, 4>', 256): (67279922, 67108864),
    ('k_grid_tf<true, 4>', 1): (3097137, 523671),
    ('k_grid_tf<true, 4>', 256): (406611194, 134348800),
}


# HBM bytes per launch (calibrated FETCH_SIZE read + WRITE_SIZE written) of
# the batched matrix-core product on the ragged workload, from the counter
# runs of `bench.py --pmc-workload batch`; valid for the source they were
# taken on (sha256 of the product's file and the headers it includes).
BATCH_TRAFFIC_SOURCES = ["uot_dense_mf.hip", "uot_epilogue.h", "uot_device.h", "uot_launch.h"]
BATCH_TRAFFIC_SHA256 = "86daf7ddf1869f35e617ac634e1a1fd373555e3f650af5956bd573c51650a9c6"
# (kernel, rows per item) -> (bytes read, bytes written, pair evaluations) of
# one launch that holds every problem (the counter workload: all 4096
# problems active, warm maxima)
BATCH_TRAFFIC_BYTES = {("k_batch_mf", 256): (281937227, 81684312, 3782323547)}


def _sha256(names):
    import hashlib
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_1607_05816_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def batch_traffic(kernel, tile_rows):
    """(bytes read, bytes written, pairs) of a full launch of the batched
    product, or None once its source changed."""
    if BATCH_TRAFFIC_SHA256 is None or _sha256(BATCH_TRAFFIC_SOURCES) != BATCH_TRAFFIC_SHA256:
        return None
    return BATCH_TRAFFIC_BYTES.get((kernel, tile_rows))


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
        if len(ms) > 2:
            # matrix-core products leave out tiles of negligible terms: the
            # exp2 they issue per launch, and that rate against the peak
            by[name]["exp_executed_per_launch"] = ms[2]
            by[name]["frac_executed"] = ms[2] / (ms[0] * 1e-3) / peak
    d = by["mfma_bf16x3"]
    return {"bound": "alu", "kernel": d["kernel"], "kernel_avg_ms": d["kernel_avg_ms"],
            "achieved": pairs / (d["kernel_avg_ms"] * 1e-3) / 1e12, "peak": peak / 1e12, "unit": "Texp/s",
            "frac": d["frac"], "work_per_launch": pairs, "work_unit": "exp (one per pair)",
            "exp_executed_per_launch": d.get("exp_executed_per_launch"), "frac_executed": d.get("frac_executed"),
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
    N = M = 20000, FP32): the same launch timed on the clouds as generated
    (spatially sorted), on the same clouds shuffled (the library puts both in
    Morton order itself, so the work lists of (row wave, column group) pairs
    within the cut are the same), and with the squared Euclidean cost.  Algorithmic work: the pairs within the cut (the
    non-zero kernel entries), each one exp and one log, priced at half the
    transcendental issue peak.  `merge_ms`: the merge of the units of each
    row and the epilogue."""
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
        t = U.time_half_step(pb, eps, v, reps=20, ctx=ctx)
        out[name + "_ms"] = t[0]
        if name == "sorted":
            out["merge_ms"] = t[1]
    peak = exp_peak() / 2
    ms = out["sorted_ms"]
    out.update({"bound": "alu", "kernel": "k_wf_lse<float, 2>", "kernel_avg_ms": ms,
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


def calibration_copy(torch, dev):
    """Three 256 MiB device copies: the kernel of known traffic the HBM
    counters are calibrated on."""
    src = torch.empty(64 << 20, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()


def pmc_workload_batch(U, torch, np, dev, ctx, iters=10):
    """The launches the batched product's counters are read on: a 256 MiB
    device copy (the calibration kernel of known size), then one batched
    solve of the 4096-problem ragged workload for a fixed `iters` iterations
    from the warm start (no tolerance, so every launch holds every problem),
    after the batch signature's tuning solve."""
    from paper_1607_05816_amd import cloud_warmstart as CW
    calibration_copy(torch, dev)
    cw = CW.CloudWarmStart.load(CW.WEIGHTS, dev)
    bp = CW.batch_problem(CW.ragged(0, B=RAGGED_B), dev)
    CW.solve(bp, ctx=ctx, tol=0.0, max_iter=4)
    v0 = cw.v0(bp, ctx=ctx)
    _, _, info = CW.solve(bp, v0=v0, ctx=ctx, tol=0.0, max_iter=iters, check_every=iters)
    torch.cuda.synchronize()
    print("pmc batch workload done: %d iterations, product %s, rows per item %d" % (
        int(info["iters"].max()), info["product"], int(info["tile_rows"])), flush=True)


BF16_MFMA_PEAK = 2.5e15     # MI355X dense BF16 MFMA, FLOP/s


def library_gemms(torch, dev, batch=256, reps=20):
    """Context for a kernel trace of the GEMM workload: the same four BF16
    products through torch's matmul (the platform BLAS), `reps` times each;
    their kernels appear in the trace beside the library's own."""
    g = torch.Generator(device="cpu")
    g.manual_seed(0)
    for M, N, K in ((batch, 256, 8192), (batch, 256, 4096), (256, 8192, batch), (batch, 4096, 256)):
        a = torch.randn(M, K, generator=g).to(dev).to(torch.bfloat16)
        b = torch.randn(K, N, generator=g).to(dev).to(torch.bfloat16)
        for _ in range(reps):
            torch.matmul(a, b)
    torch.cuda.synchronize()


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


def grid2d_bench(U, ctx, dev, np, torch, steps=5, warmup=1, seed=0):
    """The 2-D grid workload: 256 x 256 blob densities, separable kernel in
    log-domain 1-D passes, eps 1e-1 -> 1e-3 (10 stages of 100 iterations) to
    residual 1e-6, solved once with KL 0.1 and once with TV 0.05, each
    followed by the FP64 objective; iterations/s over `steps` steps, the
    roofline of its dominant pass (one field and 256 fields) and the mixed
    FP16/FP32 form."""
    from paper_1607_05816_amd import synth
    pr = synth.blobs2d(seed, n=N_GRID)
    t = lambda a: torch.tensor(np.asarray(a), dtype=torch.float32, device=dev)
    d = np.full(pr.size, pr.h[0] * pr.h[1])
    probs = []
    for name, lam in PENALTIES:
        F = U.KL(lam) if name == "KL" else U.TV(lam)
        probs.append((name, U.grid_problem(pr.shape, pr.h, t(pr.p), t(pr.q), t(d), t(d), F, F)))
    for _, pb in probs:
        pb.workspace()

    def step():
        out = []
        for name, pb in probs:
            u, v, info = U.solve(pb, EPS, eps0=EPS0, tol=TOL, max_iter=MAX_ITER, check_every=50, ctx=ctx)
            obj = U.objective(pb, EPS, u, v, ctx=ctx)
            out.append((name, info, obj, v))
        return out

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = 0
    last = None
    for _ in range(steps):
        last = step()
        iters += sum(o[1]["iters"] for o in last)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {
        "workload": "grid2d-256x256-blobs5-KL0.1+TV0.05-eps1e-1to1e-3-10x100-tol1e-6 FP32",
        "iters_per_s": iters / dt, "ms_per_step": dt / steps * 1e3, "steps": steps,
        "time_to_residual_ms": {o[0]: o[1]["elapsed_ms"] for o in last},
        "iters_per_solve": {o[0]: o[1]["iters"] for o in last},
        "converged": all(o[1]["converged"] for o in last),
        "gap": {o[0]: o[2]["gap"] for o in last},
        "roofline": grid_roofline(U, probs, last, ctx, torch, np),
        "mixed_fp16_fp32": mixed_precision(U, probs, last, ctx, torch),
    }, pr


METRIC = "Sinkhorn iters/s and time-to-residual 1e-6, warm+batched vs plain, 1 MI355X"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-grid", action="store_true")
    ap.add_argument("--no-warm-bary", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-gemm", action="store_true")
    ap.add_argument("--no-extensions", action="store_true")
    ap.add_argument("--pmc-workload", nargs="?", const="grid", choices=("grid", "dense", "batch", "gemm"),
                    help="only run the launches counters are read on: the grid passes (HBM traffic), "
                         "the dense products at 20000^2, the batched product of the ragged workload or the "
                         "training GEMMs of the warm-start net")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    # the oracle's CPU sample runs first, before anything touches the GPU
    # (its worker processes are forked)
    cs = None
    if not args.no_cpu_baseline and args.pmc_workload is None:
        cs = cpu_sample()

    import numpy as np
    import torch
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
    if args.pmc_workload == "batch":
        pmc_workload_batch(U, torch, np, dev, U.default_context())
        return
    if args.pmc_workload == "gemm":
        calibration_copy(torch, dev)
        print(json.dumps(gemm_roofline(U, torch, np, dev, U.default_context())), flush=True)
        library_gemms(torch, dev)
        return
    ctx = U.default_context()
    head = ragged_headline(U, ctx, dev, np, torch, args.steps, args.warmup)
    iters_cold = head.pop("iters_cold")
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "problems/s to residual 1e-6",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded ragged uniform point clouds)",
        "config": {"workload": "ragged-4096-clouds2d-NM-loguniform-64-4096-uniform-points-KL1-eps5e-3-tol1e-6",
                   "problems": RAGGED_B, "eps": RAGGED_EPS, "tol": TOL, "lambda": 1.0, "seed": 0,
                   "warm_start": "cloud MLP 16-64-64-64-1 (data/warmstart_cloud.npz)", "parallelism": "single-gpu"},
        "time_to_residual_1e-6_s": {"warm_batched": head["warm"]["seconds"],
                                    "cold_batched": head["cold_batched"]["seconds"],
                                    "plain_extrapolated": head["plain"]["seconds_extrapolated"]},
        "speedup_vs_plain": head["speedup_vs_plain"],
        "iters_per_s": head["warm"]["problem_iters_per_s"],
        "roofline": head["roofline"],
        "ragged": {k: v for k, v in head.items() if k not in ("value", "ms_per_step", "roofline")},
    }
    if not args.no_grid:
        line["grid2d_256"], pr = grid2d_bench(U, ctx, dev, np, torch, seed=args.seed)
    if not args.no_warm_bary:
        line["barycenter_warm_start"] = warm_bary(U, ctx, dev, np, torch)
    if not args.no_dense:
        line["roofline_dense"] = dense_roofline(U, torch, np, dev, ctx)
        line["dense_solve"] = dense_solve(U, torch, np, dev, ctx)
    if not args.no_gemm:
        line["roofline_gemm"] = gemm_roofline(U, torch, np, dev, ctx)
    if not args.no_extensions:
        from paper_1607_05816_amd import synth
        line["extensions"] = extensions(U, synth.blobs2d(args.seed, n=N_GRID), ctx, dev, np, torch)
        line["extensions"]["roofline_wf_dense"] = wf_dense_roofline(U, torch, np, dev, ctx)
        line["extensions"]["gradient_flows"] = flows_bench(U, torch, np, dev, ctx)
        line["extensions"]["colour_transfer"] = colour_transfer_bench(U, torch, np, dev, ctx)
    if cs is not None:
        line["cpu_baseline"] = cpu_baseline_ragged(cs, iters_cold, None, None)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
