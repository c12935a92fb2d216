"""Writes the stored oracle solutions that the full-size GPU parity tests
compare against.  Every value here comes from `oracle/` (FP64) on inputs from
the seeded generators; nothing is read from the GPU path.

    python tests/golden/make_golden.py grid256_kl grid256_tv bary8x128_kl

Cases (the workloads' own sizes):
  grid256_kl, grid256_tv: 256 x 256 blob images on [0,1]^2 (seed 0), KL 0.1
      or TV 0.05 on both marginals, eps 1e-1 -> 1e-3 by the eps-scaling of
      Sec. 4.4 (10 stages of 100 iterations), to residual 1e-6;
  bary8x128_kl: barycentre of 8 blob images of 128 x 128 (seed 0),
      alpha_k = 1/8, KL 0.5 on both sides of every coupling (Sec. 5.2,
      Table estimatebary (ii)), eps 2e-3 from a cold start, to residual 1e-6.

Inputs are rounded once to FP32, as the GPU tests round them, and the oracle
runs on those values.  The stored potentials are the oracle's FP64 results
rounded to FP32 (relative rounding 6e-8, far below the 1e-5 the tests use);
`iters` is the oracle's own stopping iteration and `res` its residual
history.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import uot_oracle as O  # noqa: E402
from paper_1607_05816_amd import synth  # noqa: E402


def f32(a):
    return np.asarray(a, np.float64).astype(np.float32).astype(np.float64)


def grid256(kind):
    pr = synth.blobs2d(0, n=256)
    p, q = f32(pr.p), f32(pr.q)
    d = f32(np.full(pr.size, pr.h[0] * pr.h[1]))
    F = O.KL(0.1) if kind == "kl" else O.TV(0.05)
    G = O.GridGeom(pr.shape, pr.h)
    r = O.solve(G, np.log(p), np.log(q), np.log(d), np.log(d), F, F, 1e-3, tol=1e-6, max_iter=5000, eps0=1e-1,
                n_stages=10, iters_per_stage=100)
    return dict(u=r["u"].astype(np.float32), v=r["v"].astype(np.float32), iters=r["iters"],
                converged=r["converged"], res=np.asarray(r["res"]))


def bary8x128():
    bp = synth.bary_blobs(0, n_marg=8, n=128)
    p = f32(bp.p)
    d = f32(np.full(128 * 128, (1.0 / 128) ** 2))
    G = O.GridGeom((128, 128), (1.0 / 128, 1.0 / 128))
    F = O.KL(0.5)
    r = O.barycenter(G, np.log(p), bp.alpha, np.log(d), np.log(d), F, F, 2e-3, tol=1e-6, max_iter=6000)
    return dict(u=r["u"].astype(np.float32), v=r["v"].astype(np.float32), logh=r["logh"].astype(np.float32),
                iters=r["iters"], converged=r["converged"], res=np.asarray(r["res"]))


CASES = {
    "grid256_kl": lambda: grid256("kl"),
    "grid256_tv": lambda: grid256("tv"),
    "bary8x128_kl": bary8x128,
}


def main(names):
    for name in names:
        t = time.time()
        out = CASES[name]()
        np.savez_compressed(os.path.join(HERE, name + ".npz"), **out)
        print("%s: %d iterations, converged %s, %.0f s" % (name, out["iters"], out["converged"], time.time() - t),
              flush=True)


if __name__ == "__main__":
    main(sys.argv[1:] or list(CASES))
