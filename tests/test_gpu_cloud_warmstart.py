"""The warm start of ragged point-cloud batches: the batched Gibbs products
(uot_batch_gibbs) and the network's features (uot_cloud_features) against
the oracle's dense log-sum-exp products, element by element; v0's
composition (uot_cloud_v0); and what the trained network (data/
warmstart_cloud.npz) gains over the cold batched iteration on held-out
batches, landing on the same fixed point."""
import math
import os
import sys

import numpy as np
import pytest
import torch

from oracle import uot_oracle as O
from tests.helpers import rounded

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import cloud_warmstart as CW  # noqa: E402
from paper_1607_05816_amd import synth  # noqa: E402
from paper_1607_05816_amd import uot as U  # noqa: E402

DEV = torch.device("cuda:0")


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def small_batch(seed, dtype, B=11, lo=20, hi=700):
    probs = synth.ragged_batch(seed, B=B, lo=lo, hi=hi)
    npd = np.float32 if dtype == torch.float32 else np.float64
    for p in probs:
        for f in ("x", "y", "p", "q", "dx", "dy"):
            setattr(p, f, rounded(getattr(p, f), npd))
    cat = lambda f: torch.tensor(np.concatenate([f(p) for p in probs]), dtype=dtype, device=DEV)
    F = U.KL(1.0)
    bp = U.BatchProblem([p.x.shape[0] for p in probs], [p.y.shape[0] for p in probs], cat(lambda p: p.x),
                        cat(lambda p: p.y), cat(lambda p: p.p), cat(lambda p: p.q), cat(lambda p: p.dx),
                        cat(lambda p: p.dy), F, F, layout="nd")
    return probs, bp


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_batch_gibbs_matches_oracle(dtype):
    """out_r = LSE_c(w_c - |row_r - col_c|^2 / eps) per problem, all four
    (rows, cols) pairings, against the oracle's dense product.  Scale of the
    terms: max |w| + max C / eps; FP32 evaluates them to a few 2^-24 of that
    scale, FP64 to a few 2^-53."""
    probs, bp = small_batch(3, dtype)
    rng = np.random.default_rng(4)
    eps = 5e-3
    tol = 2e-6 if dtype == torch.float32 else 1e-13
    for rows in (0, 1):
        for cols in (0, 1):
            n_c = bp.totM if cols else bp.totN
            w = rounded(rng.uniform(-3, 1, n_c), np.float32 if dtype == torch.float32 else np.float64)
            say("case batch gibbs", dtype, rows, cols)
            out = U.batch_gibbs(bp, eps, rows, cols, torch.tensor(w, dtype=dtype, device=DEV)).cpu().numpy()
            offR = bp.offM if rows else bp.offN
            offC = bp.offM if cols else bp.offN
            for b, p in enumerate(probs):
                R = p.y if rows else p.x
                C = p.y if cols else p.x
                wb = w[offC[b]:offC[b + 1]]
                ref = O.PointsGeom(R, C).lse_x(wb, eps)
                scale = np.max(np.abs(wb)) + np.max(O.sq_dist(R, C)) / eps
                err = np.max(np.abs(out[offR[b]:offR[b + 1]] - ref)) / scale
                assert err < tol, (rows, cols, b, err)


def test_cloud_features_match_oracle_products():
    """The 16 features of every point of the second clouds against the same
    quantities from the oracle's dense products (FP32: the products to a few
    2^-24 of their term scale, times eps), then the normalisation."""
    probs, bp = small_batch(5, torch.float32)
    eps = 5e-3
    rng = np.random.default_rng(6)
    shift = rng.uniform(-0.1, 0.1, 16).astype(np.float32)
    scale = rng.uniform(0.5, 20.0, 16).astype(np.float32)
    say("case cloud features")
    x = U.cloud_features(bp, eps, shift, scale).cpu().numpy().astype(np.float64)
    prods = [(0, "pdx", a) for a in (0.5, 1, 2, 4)] + [(1, "qdy", a) for a in (0.5, 1, 2, 4)] + \
            [(0, "dx", a) for a in (0.5, 1, 2)] + [(1, "dy", 1)] + [(0, "pdx", None), (1, "qdy", None)]
    for b, p in enumerate(probs):
        c = np.zeros((p.y.shape[0], 16))
        c[:, 0] = eps * np.log(p.q)
        ws = {"pdx": np.log(p.p) + np.log(p.dx), "qdy": np.log(p.q) + np.log(p.dy), "dx": np.log(p.dx),
              "dy": np.log(p.dy)}
        tol = np.zeros(16)
        tol[0] = 1e-6 * eps * np.max(np.abs(np.log(p.q))) + 1e-9
        for k, (cols, inp, a) in enumerate(prods):
            C = p.y if cols else p.x
            if a is None:       # the problem's total mass: the log-sum of the input
                c[:, k + 1] = eps * O.lse(ws[inp], axis=0)
                tol[k + 1] = 4e-6 * eps * np.max(np.abs(ws[inp]))
                continue
            c[:, k + 1] = eps * O.PointsGeom(p.y, C).lse_x(ws[inp], a * eps)
            tol[k + 1] = 4e-6 * eps * (np.max(np.abs(ws[inp])) + np.max(O.sq_dist(p.y, C)) / (a * eps))
        c[:, 15] = eps * math.log(p.x.shape[0] / p.y.shape[0])
        tol[15] = 1e-6 * abs(c[0, 15]) + 1e-9
        ref = (c - shift) * scale
        got = x[bp.offM[b]:bp.offM[b + 1]]
        assert np.all(np.abs(got - ref) <= (tol + 2e-7 * np.abs(c - shift)) * scale + 1e-6 * np.abs(ref)), b


def test_cloud_v0_composition():
    rng = np.random.default_rng(8)
    q = rng.uniform(0.1, 1.0, 1000).astype(np.float32)
    y = rng.standard_normal(1000).astype(np.float32)
    say("case cloud v0")
    v0 = U.cloud_v0(torch.tensor(q, device=DEV), 0.004, torch.tensor(y, device=DEV), 0.02, -0.003).cpu().numpy()
    ref = 0.004 * np.log(q.astype(np.float64)) + 0.02 * y - 0.003
    assert np.max(np.abs(v0 - ref)) < 1e-8


def test_trained_cloud_warm_start_gains_over_cold_batch():
    """Held-out ragged batches (sizes as the workload's, fewer problems):
    the network's v^(0) needs fewer iterations in total than the cold start
    (v^(0) = 0) and than the pointwise part alone (v^(0) = z eps log q, no
    network), and the iteration lands on the same potentials (it decides the
    answer, to the accuracy the tolerance allows)."""
    if not os.path.exists(CW.WEIGHTS):
        pytest.fail("missing trained weights %s" % CW.WEIGHTS)
    cw = CW.CloudWarmStart.load(CW.WEIGHTS, DEV)
    ratios = []
    for seed in (7, 8):
        bp = CW.batch_problem(CW.ragged(seed, B=512), DEV)
        say("case cloud warm start seed", seed)
        _, vc, ic = CW.solve(bp)
        ones = torch.zeros(bp.totM, dtype=torch.float32, device=DEV)
        vp = U.cloud_v0(bp.q, CW.zeps(), ones, 1.0, 0.0)
        _, _, ip = CW.solve(bp, v0=vp)
        v0 = cw.v0(bp)
        _, vw, iw = CW.solve(bp, v0=v0)
        assert ic["n_converged"] == bp.B and ip["n_converged"] == bp.B and iw["n_converged"] == bp.B
        cold, point, warm = int(ic["iters"].sum()), int(ip["iters"].sum()), int(iw["iters"].sum())
        say("  total iterations: cold %d, pointwise part %d, network %d" % (cold, point, warm))
        ratios.append(min(cold, point) / warm)
        dv = float((vw - vc).abs().max() / vc.abs().max())
        assert dv < 1e-3, dv
    assert min(ratios) > 1.1, ratios
