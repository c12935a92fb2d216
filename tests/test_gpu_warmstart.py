"""The trained warm-start network of barycentres (paper_1607_05816_amd/data/
warmstart_mlp64.npz) against the method without it, every start on the same
schedule (no eps-scaling): on 128 x 128 barycentres of 8 blob images (KL
0.5, eps 2e-3, tol 1e-6) over four seeds, the network's v^(0) must need
fewer iterations on average than the best start without a network: the cold
start (v^(0) = 0) and the local estimate (the one-point problem between p_k
and h0 at every cell, uot_bary_local_v0).  Every start lands on the same
fixed point (the iteration, not the network, decides the answer)."""
import os
import sys

import numpy as np
import pytest
import torch

from tests.helpers import pot_rel_err

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_1607_05816_amd import synth  # noqa: E402
from paper_1607_05816_amd import warmstart as W  # noqa: E402
from paper_1607_05816_amd.train_warmstart import load_weights  # noqa: E402

DEV = torch.device("cuda:0")
WEIGHTS = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1607_05816_amd", "data",
                       "warmstart_mlp64.npz")


def test_trained_net_gains_over_the_best_start_without_it():
    net = load_weights(WEIGHTS, DEV)
    iters = {"cold": [], "local": [], "net": []}
    for seed in (0, 1, 2, 3):
        print("case warm start seed", seed, flush=True)
        sys.stdout.flush()
        pr = synth.bary_blobs(seed, n_marg=8, n=128)
        p = torch.tensor(pr.p, dtype=torch.float32, device=DEV)
        starts = {"cold": None, "local": W.barycenter_local_v0(p, pr.alpha, 128),
                  "net": W.barycenter_v0(net, p, pr.alpha, 128)}
        hs = {}
        for name, v0 in starts.items():
            _, _, h, info = W.barycenter_solve(p, pr.alpha, 128, v0=None if v0 is None else v0.contiguous())
            assert info["converged"], (seed, name)
            iters[name].append(info["iters"])
            hs[name] = h.cpu().numpy().astype(np.float64)
        for name in ("local", "net"):
            assert pot_rel_err(hs[name], hs["cold"], 1.0) < 1e-3, (seed, name)
        print("  iterations: %s" % {k: v[-1] for k, v in iters.items()}, flush=True)
    mean = {k: float(np.mean(v)) for k, v in iters.items()}
    print("mean iterations: %s; gain of the network over the best start without it: %.3f" % (
        mean, min(mean["cold"], mean["local"]) / mean["net"]), flush=True)
    assert mean["net"] < min(mean["cold"], mean["local"]), mean
