"""Shared test helpers: input marshalling for both sides and the parity metric."""
import numpy as np

from oracle import uot_oracle as O


def pot_rel_err(gpu, ref, eps):
    """max |u_gpu - u_ref| / max(||u_ref||_inf, eps) over finite entries; the
    -inf pattern (zero densities) must match exactly."""
    a = np.asarray(gpu, np.float64)
    b = np.asarray(ref, np.float64)
    assert a.shape == b.shape
    assert np.array_equal(np.isneginf(a), np.isneginf(b)), "-inf pattern differs"
    assert not np.isnan(a).any(), "NaN in GPU potentials"
    f = np.isfinite(b)
    if not f.any():
        return 0.0
    return float(np.max(np.abs(a[f] - b[f])) / max(np.max(np.abs(b[f])), eps))


def oracle_div(F):
    """Oracle divergence from a binding divergence."""
    from paper_1607_05816_amd import uot as U
    if F.kind == U.UOT_DIV_EQ:
        return O.EQ
    if F.kind == U.UOT_DIV_KL:
        return O.KL(F.lam)
    if F.kind == U.UOT_DIV_TV:
        return O.TV(F.lam)
    if F.kind == U.UOT_DIV_GROWTH:
        return O.GROWTH(F.lam)
    return O.RG(F.alpha, F.beta)


def rounded(a, dtype):
    """Round float64 draws once to the GPU dtype; both sides use these values."""
    return np.asarray(a, np.float64).astype(dtype).astype(np.float64)
