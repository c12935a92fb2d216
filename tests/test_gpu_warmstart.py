"""The trained warm-start network (paper_1607_05816_amd/data) against the
method without it: on 128 x 128 barycentres of 8 blob images (KL 0.5,
eps 2e-3, tol 1e-6) the network's v^(0) must reach the tolerance in fewer
iterations than the plain cold start with eps-scaling, and land on the same
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


def test_trained_net_gains_over_cold_start():
    net = load_weights(WEIGHTS, DEV)
    gains = []
    for seed in (0, 3):
        print("case warm start seed", seed, flush=True)
        sys.stdout.flush()
        pr = synth.bary_blobs(seed, n_marg=8, n=128)
        p = torch.tensor(pr.p, dtype=torch.float32, device=DEV)
        uc, vc, hc, ic = W.barycenter_solve(p, pr.alpha, 128, eps0=W.EPS0)
        v0 = W.barycenter_v0(net, p, pr.alpha, 128)
        uw, vw, hw, iw = W.barycenter_solve(p, pr.alpha, 128, v0=v0.contiguous())
        assert ic["converged"] and iw["converged"]
        gains.append(ic["iters"] - iw["iters"])
        # same barycentre to the accuracy the tolerance allows
        assert pot_rel_err(hw.cpu(), hc.cpu().numpy().astype(np.float64), 1.0) < 1e-3
    assert min(gains) > 0, gains
