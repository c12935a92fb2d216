"""Plain FP64 CPU oracle for the generalized Sinkhorn scaling iteration of
entropic unbalanced optimal transport (Chizat, Peyre, Schmitzer, Vialard,
"Scaling algorithms for unbalanced optimal transport problems").

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module:
only the tests, the package smoke check and the CPU-baseline leg of the
benchmark do.  It shares no code with the HIP path; the two meet only in the
seeded input generators (which hold none of the method's arithmetic).

Conventions (discrete setting of Sec. 4 "Numerical algorithm for discrete
measures"):
  * X = {x_i}, Y = {y_j}, reference weights dx_i, dy_j > 0;
  * densities p = mu/dx, q = nu/dy (Sec. 5.1, eq. (UOT));
  * potentials u = eps log a, v = eps log b (Prop. "alternating"), so the plan
    w.r.t. dx (x) dy is R_ij = exp((u_i + v_j - C_ij)/eps) (Thm. "duality");
  * all arrays are float64 and log-densities carry -inf where the density is 0
    (convention 0/0 = 0 of Sec. 1 "Notation").

Functions without an independent pin in tests/ are flagged "parity unpinned"
in their docstring; at the time of writing every function is pinned.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, List, Optional, Sequence

import numpy as np

LOG2 = np.log(2.0)


# ---------------------------------------------------------------------------
# elementary helpers
# ---------------------------------------------------------------------------
def lse(a: np.ndarray, axis) -> np.ndarray:
    """log(sum(exp(a))) along `axis`; an all -inf slice gives -inf."""
    a = np.asarray(a, dtype=np.float64)
    m = np.max(a, axis=axis, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore", over="ignore", invalid="ignore"):
        s = np.sum(np.exp(a - m_safe), axis=axis, keepdims=True)
        out = np.log(s) + m_safe
    return np.squeeze(out, axis=axis)


def safe_log(x: np.ndarray) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.log(x)


# ---------------------------------------------------------------------------
# divergences: Sec. 2.1 (entropy functions, Examples KL / TV / = / RG)
# ---------------------------------------------------------------------------
@dataclass(frozen=True)
class Div:
    """A marginal functional F(s) = sum_i dx_i Dbar_phi(s_i | p_i) (eq.
    "divergencefunctions"), scaled by `lam` for KL and TV.

    kind: "eq" (equality constraint), "kl" (lam * KL), "tv" (lam * TV),
    "rg" (range constraint RG[alpha, beta], 0 <= alpha <= beta <= inf),
    "growth" (the growth functional of the WF gradient flow example of Sec.
    5.3: F(s) = inf_r KL(s|r) - lam r + iota_{r <= p}, lam = 2 tau alpha in
    [0, 1); p is the density cap, 1 in the paper's example).
    """
    kind: str
    lam: float = 1.0
    alpha: float = 0.0
    beta: float = np.inf


EQ = Div("eq")


def KL(lam):
    return Div("kl", lam=float(lam))


def TV(lam):
    return Div("tv", lam=float(lam))


def RG(alpha, beta):
    return Div("rg", alpha=float(alpha), beta=float(beta))


def GROWTH(lam):
    """Growth functional with incentive lam = 2 tau alpha (0 <= lam < 1)."""
    return Div("growth", lam=float(lam))


# ---------------------------------------------------------------------------
# proxdiv: Table "proximalexplicit" (Sec. 5.1), stabilized form of eq.
# (proxdiv) in Sec. 4.3.  proxdiv_F(s, u, eps) = prox^KL_{F/eps}(e^{-u/eps} s) / s
# ---------------------------------------------------------------------------
def proxdiv_log(F: Div, logp: np.ndarray, logs: np.ndarray, ubar, eps: float) -> np.ndarray:
    """Logarithm of the stabilized proxdiv of Table proximalexplicit, with
    absorbed offset `ubar` (0 gives the plain proxdiv of eq. (proxdiv_a)).

    Rows (log of the table's right column):
      =      : log p - log s
      lam KL : lam/(lam+eps) (log p - log s) - ubar/(lam+eps)
      lam TV : clamp(log p - log s, -(lam+ubar)/eps, (lam-ubar)/eps)
      RG     : min(log beta + log p - log s, max(log alpha + log p - log s, -ubar/eps))
      growth : min(-(ubar + log kappa)/eps, (log p - log s - ubar)/(1 + eps)),
               kappa = 1 - lam (the two branches of the tumour-growth example,
               Sec. 5.3, with the cap p; they meet where the paper switches)
    """
    logp = np.asarray(logp, dtype=np.float64)
    logs = np.asarray(logs, dtype=np.float64)
    ubar = np.broadcast_to(np.asarray(ubar, dtype=np.float64), logp.shape)
    with np.errstate(invalid="ignore"):
        # p = 0 gives ratio 0 even where s = 0 (0/0 = 0); s = 0 < p gives +inf
        d = np.where(np.isneginf(logp), -np.inf, logp - logs)
    if F.kind == "eq":
        return d
    if F.kind == "kl":
        z = F.lam / (F.lam + eps)
        return z * d - ubar / (F.lam + eps)
    if F.kind == "tv":
        lo = -(F.lam + ubar) / eps
        hi = (F.lam - ubar) / eps
        return np.minimum(np.maximum(d, lo), hi)
    if F.kind == "rg":
        lower = (np.log(F.alpha) + d) if F.alpha > 0 else np.full_like(d, -np.inf)
        inner = np.maximum(lower, -ubar / eps)
        if np.isinf(F.beta):
            return inner
        return np.minimum(np.log(F.beta) + d, inner)
    if F.kind == "growth":
        lk = np.log1p(-F.lam)
        return np.minimum(-(ubar + lk) / eps, (d - ubar) / (1.0 + eps))
    raise ValueError(F.kind)


def proxdiv_scaling(F: Div, p: np.ndarray, s: np.ndarray, ubar, eps: float) -> np.ndarray:
    """Table proximalexplicit, right column, evaluated in the scaling domain
    (plain exponentials; used by the literal Algorithms 1 and 2).  0/0 = 0."""
    p = np.asarray(p, dtype=np.float64)
    s = np.asarray(s, dtype=np.float64)
    ubar = np.broadcast_to(np.asarray(ubar, dtype=np.float64), p.shape)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where((p == 0) & (s == 0), 0.0, p / s)
    if F.kind == "eq":
        return ratio
    if F.kind == "kl":
        z = F.lam / (F.lam + eps)
        return ratio ** z * np.exp(-ubar / (F.lam + eps))
    if F.kind == "tv":
        return np.minimum(np.exp((F.lam - ubar) / eps), np.maximum(np.exp(-(F.lam + ubar) / eps), ratio))
    if F.kind == "rg":
        inner = np.maximum(F.alpha * ratio, np.exp(-ubar / eps))
        if np.isinf(F.beta):
            return inner
        return np.minimum(F.beta * ratio, inner)
    if F.kind == "growth":
        # first branch while s <= e^{u/eps} kappa^{(1+eps)/eps} p, else the second
        kap = 1.0 - F.lam
        with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
            low = s <= np.exp(ubar / eps) * kap ** ((1.0 + eps) / eps) * p
            first = (np.exp(ubar) * kap) ** (-1.0 / eps) * np.ones_like(s)
            second = np.where(p > 0, (p / (s * np.exp(ubar))) ** (1.0 / (1.0 + eps)), 0.0)
        return np.where(p > 0, np.where(low, first, second), 0.0)
    raise ValueError(F.kind)


# ---------------------------------------------------------------------------
# F and F* (Sec. 5.1 eq. (UOT); conjugates from the appendix "Properties of
# divergence functionals", phi* of each entropy function), dx-weighted.
# ---------------------------------------------------------------------------
def F_value(F: Div, s: np.ndarray, p: np.ndarray, dx: np.ndarray) -> float:
    """F(s) = sum_i dx_i Dbar_phi(s_i | p_i); set constraints give 0 or inf."""
    s = np.asarray(s, np.float64)
    p = np.asarray(p, np.float64)
    if F.kind == "kl":
        with np.errstate(divide="ignore", invalid="ignore"):
            t = np.where(s > 0, s * np.log(s / p), 0.0)
        t = np.where((p == 0) & (s > 0), np.inf, t)
        return float(F.lam * np.sum(dx * (t - s + p)))
    if F.kind == "tv":
        return float(F.lam * np.sum(dx * np.abs(s - p)))
    if F.kind == "eq":
        ok = np.allclose(s, p, rtol=1e-9, atol=1e-300)
        return 0.0 if ok else np.inf
    if F.kind == "rg":
        ok = np.all(s >= F.alpha * p * (1 - 1e-9)) and np.all(s <= F.beta * p * (1 + 1e-9))
        return 0.0 if ok else np.inf
    if F.kind == "growth":
        return float(np.sum(dx * growth_value(s, p, F.lam)))
    raise ValueError(F.kind)


def growth_value(s, p, lam):
    """Pointwise inf_{0 <= r <= p} [KL(s|r) - lam r] in closed form: the inner
    minimiser is r = min(s / kappa, p) (kappa = 1 - lam), giving s log kappa
    while s <= kappa p and s log(s/p) - s + kappa p beyond."""
    s = np.asarray(s, np.float64)
    p = np.asarray(p, np.float64)
    kap = 1.0 - lam
    with np.errstate(divide="ignore", invalid="ignore"):
        lo = s * np.log(kap)
        hi = np.where(s > 0, s * np.log(s / p), 0.0) - s + kap * p
    out = np.where(s <= kap * p, lo, hi)
    return np.where((p == 0) & (s > 0), np.inf, out)


def F_conj(F: Div, w: np.ndarray, p: np.ndarray, dx: np.ndarray) -> float:
    """F*(w) = sum_i dx_i p_i lam phi*(w_i/lam) (+ the domain constraint w <= lam phi'_inf).

      KL: phi*(t) = e^t - 1        TV: phi*(t) = max(t, -1), t <= 1
      =  : phi*(t) = t             RG: phi*(t) = max(alpha t, beta t)
    """
    w = np.asarray(w, np.float64)
    p = np.asarray(p, np.float64)
    if F.kind == "kl":
        with np.errstate(invalid="ignore", over="ignore"):
            t = np.where(p > 0, p * np.expm1(w / F.lam), 0.0)
        return float(np.sum(dx * F.lam * t))
    if F.kind == "tv":
        if np.any(w > F.lam * (1 + 1e-12) + 1e-300):
            return np.inf
        return float(np.sum(dx * p * np.maximum(w, -F.lam)))
    if F.kind == "eq":
        with np.errstate(invalid="ignore"):
            return float(np.sum(dx * np.where(p > 0, p * w, 0.0)))
    if F.kind == "rg":
        hi = np.where(w > 0, (F.beta * w if np.isfinite(F.beta) else np.where(p > 0, np.inf, 0.0)), F.alpha * w)
        with np.errstate(invalid="ignore"):
            t = np.where(p > 0, p * hi, 0.0)
        return float(np.sum(dx * t))
    if F.kind == "growth":
        # the pointwise F is C^1 with F' = log max(kappa, s/p): F*(w) = 0 for
        # w <= log kappa, p (e^w - kappa) beyond
        with np.errstate(over="ignore"):
            return float(np.sum(dx * p * np.maximum(np.exp(w) - (1.0 - F.lam), 0.0)))
    raise ValueError(F.kind)


# ---------------------------------------------------------------------------
# geometries: the Gibbs operators of eq. (gibbs-convolution) in log form
# ---------------------------------------------------------------------------
class DenseGeom:
    """Explicit cost matrix C (I x J).  lse_x(w) = log K(e^w) with
    (K e^w)_i = sum_j exp(-C_ij/eps + w_j); lse_y is the transposed product."""

    def __init__(self, C: np.ndarray):
        self.C = np.asarray(C, dtype=np.float64)
        self.N, self.M = self.C.shape

    def lse_x(self, w, eps):
        with np.errstate(invalid="ignore"):
            a = np.where(np.isinf(self.C), -np.inf, -self.C / eps + np.asarray(w)[None, :])
        return lse(a, axis=1)

    def lse_y(self, w, eps):
        with np.errstate(invalid="ignore"):
            a = np.where(np.isinf(self.C), -np.inf, -self.C / eps + np.asarray(w)[:, None])
        return lse(a, axis=0)

    def cost_moment_log(self, wx, wy, eps):
        """log sum_ij C_ij exp(wx_i + wy_j - C_ij/eps); pairs with C = inf
        (beyond a cut locus) carry no mass and contribute nothing."""
        with np.errstate(divide="ignore", invalid="ignore"):
            L = np.where(np.isfinite(self.C), np.log(self.C) - self.C / eps, -np.inf) \
                + np.asarray(wx)[:, None] + np.asarray(wy)[None, :]
        return float(lse(L.reshape(-1), axis=0))


def sq_dist(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """C_ij = |x_i - y_j|^2 computed as a sum of squared coordinate gaps."""
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    if x.ndim == 1:
        x = x[:, None]
    if y.ndim == 1:
        y = y[:, None]
    C = np.zeros((x.shape[0], y.shape[0]))
    for k in range(x.shape[1]):
        C += (x[:, k][:, None] - y[:, k][None, :]) ** 2
    return C


def wf_cost(d2: np.ndarray, cut: float) -> np.ndarray:
    """Cost of the Wasserstein-Fisher-Rao distance (Definition WF, eq.
    "logcost"): c = -log cos_+^2(theta), cos_+(z) = cos(min(z, pi/2)), with the
    distance rescaled so that theta = (pi/2) |x - y| / cut; c is +inf from
    |x - y| = cut on (the cut locus).  d2 holds squared distances."""
    d = np.sqrt(np.asarray(d2, np.float64))
    theta = 0.5 * np.pi * d / cut
    with np.errstate(divide="ignore"):
        c = -2.0 * np.log(np.cos(np.minimum(theta, 0.5 * np.pi)))
    return np.where(theta < 0.5 * np.pi, c, np.inf)


def make_cost(d2, cost: str, cut: Optional[float]):
    if cost == "sqeuclid":
        return np.asarray(d2, np.float64)
    if cost == "wf":
        return wf_cost(d2, cut)
    raise ValueError(cost)


class PointsGeom(DenseGeom):
    """Point clouds with the squared Euclidean cost (Sec. 2.3 GHK cost |x-y|^2)
    or, with cost="wf", the WF cost of eq. "logcost" with cut locus `cut`."""

    def __init__(self, x, y, cost: str = "sqeuclid", cut: Optional[float] = None):
        super().__init__(make_cost(sq_dist(x, y), cost, cut))


class GridGeom:
    """X = Y = a regular grid of cell centres with cost |x - y|^2, for which
    K is a tensor product of 1-D Gaussian kernels, applied by successive 1-D
    passes (Sec. 4.4, "Computing the matrix multiplications": separable
    kernel).  Each 1-D pass is evaluated as a log-sum-exp, which is the same
    sum as the paper's convolution written in the log domain."""

    def __init__(self, shape: Sequence[int], h: Sequence[float], cost: str = "sqeuclid",
                 cut: Optional[float] = None):
        self.shape = tuple(int(n) for n in shape)
        self.h = tuple(float(v) for v in h)
        self.cost, self.cut = cost, cut
        if cost != "sqeuclid" and len(self.shape) != 1:
            # -log cos^2 of a Euclidean distance is not a sum over axes
            raise ValueError("the WF cost is separable only on a 1-D grid")
        self.N = self.M = int(np.prod(self.shape))
        self.C1 = [make_cost(((np.arange(n)[:, None] - np.arange(n)[None, :]) * hh) ** 2, cost, cut)
                   for n, hh in zip(self.shape, self.h)]

    def _sep(self, w, logkers):
        t = np.asarray(w, np.float64).reshape(self.shape)
        for ax, L in enumerate(logkers):
            # out[..., i_ax, ...] = LSE_j (L[i_ax, j] + t[..., j, ...])
            t = np.moveaxis(t, ax, -1)                        # (..., n_ax)
            t = lse(t[..., None, :] + L, axis=-1)             # (..., n_ax[i])
            t = np.moveaxis(t, -1, ax)
        return t.reshape(-1)

    def lse_x(self, w, eps):
        return self._sep(w, [-C / eps for C in self.C1])

    lse_y = lse_x  # X = Y and C symmetric

    def cost_moment_log(self, wx, wy, eps):
        """log sum_ij C_ij exp(wx_i + wy_j - C_ij/eps) with C = sum_axes C^(a):
        axis a carries the kernel C^(a) e^{-C^(a)/eps}, the others e^{-C/eps}."""
        terms = []
        for a in range(len(self.shape)):
            kers = []
            for b, C in enumerate(self.C1):
                if a == b:
                    with np.errstate(divide="ignore", invalid="ignore"):
                        kers.append(np.where(np.isfinite(C), np.log(C) - C / eps, -np.inf))
                else:
                    kers.append(-C / eps)
            terms.append(lse(np.asarray(wx) + self._sep(wy, kers), axis=0))
        return float(lse(np.array(terms), axis=0))

    def dense(self) -> DenseGeom:
        axes = [(np.arange(n) + 0.5) * hh for n, hh in zip(self.shape, self.h)]
        mesh = np.meshgrid(*axes, indexing="ij")
        pts = np.stack([m.reshape(-1) for m in mesh], axis=1)
        return PointsGeom(pts, pts, self.cost, self.cut)


# ---------------------------------------------------------------------------
# residual: relative L1 violation of the X marginal against its prox target
# (stopping criterion, which the paper leaves unspecified in Alg. 1 / 2)
# ---------------------------------------------------------------------------
def expo(pot, prev, logd, eps):
    """Exponent pot/eps + log d with which a potential enters the next Gibbs
    product.  Where the product it was computed from vanished (prev = -inf:
    K b = 0 at that point, which exact zeros of K beyond a cut locus allow),
    the row of the plan is zero whatever the potential, and every b_j that
    a_i K_ij could reach is already 0 (q_j = 0), so the point is left out
    (-inf) instead of carrying an infinite potential into the sum."""
    pot = np.asarray(pot, np.float64)
    with np.errstate(invalid="ignore"):
        w = pot / eps + logd
    if prev is None:
        return w
    return np.where(np.isneginf(prev), -np.inf, w)


def marginal_residual(S, u_old, u_new, logdx, eps) -> float:
    """r = sum_i dx_i |e^{S_i + u_old_i/eps} - e^{S_i + u_new_i/eps}|
           / sum_i dx_i e^{S_i + u_new_i/eps}  (terms with S_i = -inf are 0)."""
    la = S + expo(u_old, S, logdx, eps)
    lb = S + expo(u_new, S, logdx, eps)
    m = np.max(lb)
    if m == -np.inf:
        # the marginal vanishes: 0/0 = 0 if the old one did too
        return 0.0 if np.all(np.isneginf(la)) else np.inf
    with np.errstate(over="ignore", invalid="ignore"):
        ea = np.exp(la - m)
        eb = np.exp(lb - m)
        num = np.where(np.isneginf(la) & np.isneginf(lb), 0.0, np.abs(ea - eb))
    den = np.sum(eb)
    return float(np.sum(num) / den)


# ---------------------------------------------------------------------------
# the scaling iteration (S) / Algorithm 1, in the log domain (Algorithm 2 with
# an absorption after every half-step), with the eps-scaling heuristic of
# Sec. 4.4 ("Gradually decreasing eps")
# ---------------------------------------------------------------------------
def eps_schedule(eps: float, eps0: Optional[float], n_stages: int = 10, iters_per_stage: int = 100):
    """List of (eps_k, n_iter_k) annealing stages before the final eps; empty
    when eps0 is None.  eps_k = eps0 * f^k, f = (eps/eps0)^(1/n_stages)."""
    if eps0 is None or n_stages <= 0:
        return []
    f = (eps / eps0) ** (1.0 / n_stages)
    return [(eps0 * f ** k, iters_per_stage) for k in range(n_stages)]


def solve(geom, logp, logq, logdx, logdy, F1: Div, F2: Div, eps: float,
          tol: float = 1e-6, max_iter: int = 10000, v0=None, u0=None,
          eps0: Optional[float] = None, n_stages: int = 10, iters_per_stage: int = 100,
          record: bool = False, rebalance_at: Optional[int] = None):
    """Scaling iterations (S): each iteration is an X half-step
        S = log K(b (.) dy),  u <- eps log proxdiv_F1(e^S)
    followed by a Y half-step
        T = log K^T(a (.) dx), v <- eps log proxdiv_F2(e^T),
    all in the log domain.  Stops after the first iteration (from the second
    on: the first residual compares with the arbitrary initial u) whose
    residual r <= tol at the final eps (annealing iterations count), or at
    max_iter.

    rebalance_at = K (KL penalties on both marginals): the v that starts
    iteration K is replaced by v - s with s the mass-balance shift of
    `mass_balance_shift` (Prop. "alternating": only v enters the iterates, so
    this is a restart from a better start, and the fixed point is unchanged).
    As u is affine in a constant shift of v (KL row of Table
    proximalexplicit), the restart is taken after the X half-step of
    iteration K: u <- u + theta1 s, with P from that u and Q from the v it was
    computed from.  The residual of iteration K is that of the unshifted u,
    and an iteration that stops is not shifted.

    Returns dict(u, v, iters, res (list), converged, hist, S) with S the last X product.
    """
    if rebalance_at is not None and (F1.kind != "kl" or F2.kind != "kl"):
        raise ValueError("the mass balance takes KL penalties on both marginals")
    N = len(logp)
    M = len(logq)
    v = np.zeros(M) if v0 is None else np.array(v0, np.float64)
    u = np.zeros(N) if u0 is None else np.array(u0, np.float64)
    stages = eps_schedule(eps, eps0, n_stages, iters_per_stage)
    res = []
    hist = []
    it = 0
    plan = [(e, n, False) for e, n in stages] + [(eps, None, True)]
    T = S = None
    for e, n_it, final in plan:
        k = 0
        while True:
            if it >= max_iter:
                return dict(u=u, v=v, iters=it, res=res, converged=False, hist=hist, S=S)
            if n_it is not None and k >= n_it:
                break
            S = geom.lse_x(expo(v, T, logdy, e), e)
            u_new = e * proxdiv_log(F1, logp, S, 0.0, e)
            r = marginal_residual(S, u, u_new, logdx, e)
            if rebalance_at is not None and it + 1 == rebalance_at and not (final and r <= tol and it + 1 >= 2):
                with np.errstate(invalid="ignore"):
                    tp = np.where(np.isneginf(logp), -np.inf, logp - u_new / F1.lam + logdx)
                    tq = np.where(np.isneginf(logq), -np.inf, logq - v / F2.lam + logdy)
                lP, lQ = lse(tp, 0), lse(tq, 0)
                if np.isfinite(lP) and np.isfinite(lQ):
                    th1 = F1.lam / (F1.lam + e)
                    u_new = u_new + th1 * (lP - lQ) / (th1 / F1.lam + 1.0 / F2.lam)
            u = u_new
            T = geom.lse_y(expo(u, S, logdx, e), e)
            v = e * proxdiv_log(F2, logq, T, 0.0, e)
            it += 1
            k += 1
            res.append(r)
            if record:
                hist.append((u.copy(), v.copy()))
            # the first residual compares with the arbitrary initial u and
            # certifies nothing: it is recorded, not used to stop
            if final and r <= tol and it >= 2:
                return dict(u=u, v=v, iters=it, res=res, converged=True, hist=hist, S=S)
    raise AssertionError("unreachable")


def half_step_x(geom, logp, logdx, logdy, F1: Div, eps, u_old, v):
    """One X half-step from a given state: returns (S, u_new, r)."""
    S = geom.lse_x(v / eps + logdy, eps)
    u_new = eps * proxdiv_log(F1, logp, S, 0.0, eps)
    return S, u_new, marginal_residual(S, u_old, u_new, logdx, eps)


def half_step_y(geom, logq, logdx, F2: Div, eps, u):
    T = geom.lse_y(u / eps + logdx, eps)
    return T, eps * proxdiv_log(F2, logq, T, 0.0, eps)


# ---------------------------------------------------------------------------
# objectives: (P_eps), (D_eps) of Thm. "duality", discrete form with the
# dx dy-weighted entropy; gap in Fenchel-Young form
# ---------------------------------------------------------------------------
def objective(geom, p, q, dx, dy, F1: Div, F2: Div, eps, u, v) -> dict:
    """Primal, dual, gap, transport cost and marginals at the plan
    R_ij = exp((u_i + v_j - C_ij)/eps) (w.r.t. dx dy).

      pi1 = R dy = e^{u/eps + S(v)},  pi2 = R^T dx = e^{v/eps + T(u)}
      P = F1(pi1) + F2(pi2) + <u,pi1>_dx + <v,pi2>_dy - eps m(pi1) + eps m(K)
      D = -F1*(-u) - F2*(-v) - eps m(pi1) + eps m(K)
      gap = [F1(pi1) + F1*(-u) + <u,pi1>] + [F2(pi2) + F2*(-v) + <v,pi2>]
    """
    p = np.asarray(p, np.float64)
    q = np.asarray(q, np.float64)
    dx = np.asarray(dx, np.float64)
    dy = np.asarray(dy, np.float64)
    logdx, logdy = np.log(dx), np.log(dy)
    S = geom.lse_x(v / eps + logdy, eps)
    T = geom.lse_y(u / eps + logdx, eps)
    with np.errstate(invalid="ignore"):
        pi1 = np.exp(S + expo(u, S, 0.0, eps))
        pi2 = np.exp(T + expo(v, T, 0.0, eps))
    pi1 = np.nan_to_num(pi1, nan=0.0)
    pi2 = np.nan_to_num(pi2, nan=0.0)
    m1 = float(np.sum(dx * pi1))
    m2 = float(np.sum(dy * pi2))
    mK = float(np.exp(lse(logdx + geom.lse_x(logdy, eps), axis=0)))
    with np.errstate(invalid="ignore"):
        up = float(np.sum(np.where(pi1 > 0, dx * u * pi1, 0.0)))
        vp = float(np.sum(np.where(pi2 > 0, dy * v * pi2, 0.0)))
    f1 = F_value(F1, pi1, p, dx)
    f2 = F_value(F2, pi2, q, dy)
    c1 = F_conj(F1, -u, p, dx)
    c2 = F_conj(F2, -v, q, dy)
    primal = f1 + f2 + up + vp - eps * m1 + eps * mK
    dual = -c1 - c2 - eps * m1 + eps * mK
    gap = (f1 + c1 + up) + (f2 + c2 + vp)
    with np.errstate(invalid="ignore"):
        wx = np.where(np.isneginf(u), -np.inf, expo(u, S, logdx, eps))
        wy = np.where(np.isneginf(v), -np.inf, expo(v, T, logdy, eps))
    cost = float(np.exp(geom.cost_moment_log(wx, wy, eps)))
    return dict(primal=primal, dual=dual, gap=gap, transport_cost=cost,
                mass=m1, mass2=m2, pi1=pi1, pi2=pi2, mK=mK)


def dual_value(geom, p, q, dx, dy, F1, F2, eps, u, v) -> float:
    """(D_eps) at (u, v)."""
    o = objective(geom, p, q, dx, dy, F1, F2, eps, u, v)
    return o["dual"]


# ---------------------------------------------------------------------------
# literal Algorithm 1 (ScalingAlgo) and Algorithm 2 (ScalingAlgo2), dense
# kernels; used to cross-check the log-domain iteration above
# ---------------------------------------------------------------------------
def scaling_algo(C, p, q, dx, dy, F1, F2, eps, n_iter, b0=None):
    """Algorithm 1: b = 1; repeat a = proxdiv_F1(K(b dy)), b = proxdiv_F2(K^T(a dx)).
    Returns the potentials (eps log a, eps log b) after each iteration."""
    K = np.exp(-np.asarray(C, np.float64) / eps)
    b = np.ones(len(q)) if b0 is None else np.asarray(b0, np.float64)
    out = []
    for _ in range(n_iter):
        a = proxdiv_scaling(F1, p, K @ (b * dy), 0.0, eps)
        b = proxdiv_scaling(F2, q, K.T @ (a * dx), 0.0, eps)
        with np.errstate(divide="ignore"):
            out.append((eps * np.log(a), eps * np.log(b)))
    return out


def scaling_algo2(C, p, q, dx, dy, F1, F2, eps, n_iter, tau, eps0=None, n_stages=10, iters_per_stage=100):
    """Algorithm 2 with absorption when max |log a~|, |log b~| > tau, and the
    eps-scaling heuristic (absorb, then change eps, then rebuild K~).
    Returns total potentials (u + eps log a~, v + eps log b~) per iteration."""
    C = np.asarray(C, np.float64)
    N, M = C.shape
    stages = eps_schedule(eps, eps0, n_stages, iters_per_stage)
    eps_of_iter = []
    for e, n in stages:
        eps_of_iter += [e] * n
    e = eps_of_iter[0] if eps_of_iter else eps
    u = np.zeros(N)
    v = np.zeros(M)
    at = np.ones(N)
    bt = np.ones(M)
    Kt = np.exp(-C / e)
    out = []
    for it in range(n_iter):
        e_it = eps_of_iter[it] if it < len(eps_of_iter) else eps
        if e_it != e:
            # absorption, then the new eps, then the rebuilt stabilized kernel
            u = u + e * np.log(at)
            v = v + e * np.log(bt)
            e = e_it
            Kt = np.exp((u[:, None] + v[None, :] - C) / e)
            at = np.ones(N)
            bt = np.ones(M)
        at = proxdiv_scaling(F1, p, Kt @ (bt * dy), u, e)
        bt = proxdiv_scaling(F2, q, Kt.T @ (at * dx), v, e)
        with np.errstate(divide="ignore"):
            la, lb = np.log(at), np.log(bt)
        out.append((u + e * la, v + e * lb))
        big = max(np.max(np.abs(la[np.isfinite(la)]), initial=0.0), np.max(np.abs(lb[np.isfinite(lb)]), initial=0.0))
        if big > tau:
            u = u + e * la
            v = v + e * lb
            Kt = np.exp((u[:, None] + v[None, :] - C) / e)
            at = np.ones(N)
            bt = np.ones(M)
    return out


# ---------------------------------------------------------------------------
# barycentres: Sec. 5.2 (weighted KL, K_k = exp(-c_k/(alpha_k eps)) with
# c_k = alpha_k c so that every K_k = K; Table estimatebary rows (i) and (ii))
# ---------------------------------------------------------------------------
# ---------------------------------------------------------------------------
# Algorithm 4 (Sec. 4.4, generalization to a function of the total mass):
# min F1(P^X R) + F2(P^Y R) + F3(m R) + eps KL(R|K), with m R the total mass
# of the plan and F3 a divergence on the one-point space (reference measure
# 1, "density" m0): F3(sigma) = D(sigma | m0).  Its proxdiv is the row of
# Table proximalexplicit with p = m0.
# ---------------------------------------------------------------------------
def mass_scaling_algo(C, p, q, dx, dy, F1, F2, F3, m0, eps, n_iter):
    """Algorithm 4 in the scaling domain: b = 1, z = 1; repeat
        a = proxdiv_F1(z K(b dy)),  b = proxdiv_F2(z K^T(a dx)),
        z = proxdiv_F3(<a dx, K(b dy)>);
    the plan is z a_i K_ij b_j.  Returns (eps log a, eps log b, log z) after
    each iteration."""
    K = np.exp(-np.asarray(C, np.float64) / eps)
    b = np.ones(len(q))
    z = 1.0
    out = []
    m0a = np.array([float(m0)])
    for _ in range(n_iter):
        a = proxdiv_scaling(F1, p, z * (K @ (b * dy)), 0.0, eps)
        b = proxdiv_scaling(F2, q, z * (K.T @ (a * dx)), 0.0, eps)
        z = float(proxdiv_scaling(F3, m0a, np.array([(a * dx) @ (K @ (b * dy))]), 0.0, eps)[0])
        with np.errstate(divide="ignore"):
            out.append((eps * np.log(a), eps * np.log(b), np.log(z)))
    return out


def solve_mass(geom, logp, logq, logdx, logdy, F1: Div, F2: Div, F3: Div, log_m0: float, eps: float,
               tol: float = 1e-6, max_iter: int = 10000, eps0: Optional[float] = None, n_stages: int = 10,
               iters_per_stage: int = 100):
    """Algorithm 4 in the log domain (zeta = log z, potentials u, v): per
    iteration
        S = log K(b dy);  u <- eps log proxdiv_F1(e^{S + zeta})   (residual r as in solve, on S + zeta)
        T = log K^T(a dx); v <- eps log proxdiv_F2(e^{T + zeta})
        log m = LSE_j(T_j + v_j/eps + log dy_j);  zeta <- log proxdiv_F3(e^{log m})  (p = m0)
    with the eps schedule of solve.  Returns dict(u, v, zeta, iters, res)."""
    N = len(logp)
    M = len(logq)
    v = np.zeros(M)
    u = np.zeros(N)
    zeta = 0.0
    stages = eps_schedule(eps, eps0, n_stages, iters_per_stage)
    res = []
    it = 0
    plan = [(e, n, False) for e, n in stages] + [(eps, None, True)]
    lm0 = np.array([float(log_m0)])
    T = None
    for e, n_it, final in plan:
        k = 0
        while True:
            if it >= max_iter:
                return dict(u=u, v=v, zeta=zeta, iters=it, res=res, converged=False)
            if n_it is not None and k >= n_it:
                break
            S = geom.lse_x(expo(v, T, logdy, e), e) + zeta
            u_new = e * proxdiv_log(F1, logp, S, 0.0, e)
            r = marginal_residual(S, u, u_new, logdx, e)
            u = u_new
            T = geom.lse_y(expo(u, S, logdx, e), e)
            v = e * proxdiv_log(F2, logq, T + zeta, 0.0, e)
            logm = float(lse(T + expo(v, T, logdy, e), axis=0))
            zeta = float(proxdiv_log(F3, lm0, np.array([logm]), 0.0, e)[0])
            it += 1
            k += 1
            res.append(r)
            if final and r <= tol and it >= 2:
                return dict(u=u, v=v, zeta=zeta, iters=it, res=res, converged=True)
    raise AssertionError("unreachable")


def pwl_root_inf(f, breaks: np.ndarray) -> np.ndarray:
    """Per column j: inf{x : f(x)[j] >= 0} for a function f, non-decreasing in
    x and linear between consecutive finite entries of breaks[:, j], that is
    negative left of the first breakpoint and >= 0 at the last one.  f takes
    an array of shape (m, J) of evaluation points and returns the same shape.
    The root is the linear interpolation on the segment where f first
    becomes >= 0 (the first breakpoint itself when f is already >= 0 there)."""
    b = np.sort(np.where(np.isfinite(breaks), breaks, np.inf), axis=0)
    fb = f(b)
    ok = np.isfinite(b) & (fb >= 0)
    i = np.argmax(ok, axis=0)                     # first breakpoint with f >= 0
    J = np.arange(b.shape[1])
    x1, f1 = b[i, J], fb[i, J]
    im = np.maximum(i - 1, 0)
    x0, f0 = b[im, J], fb[im, J]
    with np.errstate(invalid="ignore", divide="ignore"):
        x = x0 + (0.0 - f0) * (x1 - x0) / (f1 - f0)
    return np.where(i == 0, x1, x)


def bary_logh(T: np.ndarray, alpha: np.ndarray, eps: float, F2: Div) -> np.ndarray:
    """log h from Table estimatebary, given T_k = log s_k (shape (n, J)).

      (i)   =       : h = (prod_k s_k^alpha_k)^(1/sum alpha)
      (ii)  lam KL  : h = (sum_k alpha_k s_k^(eps/(eps+lam)) / sum alpha)^((eps+lam)/eps)
      (iii) lam TV  : with I+ = {k : s_k > 0}, h = 0 if the weight off I+ is at
                      least the weight on I+; otherwise log h is the root of
                      sum_{k not in I+} alpha_k + sum_{k in I+} alpha_k
                        clamp((eps/lam) log(h/s_k), -1, 1)
      (iv)  RG[b1,b2]: h = 0 if some s_k = 0; otherwise log h is the root of
                      sum_k alpha_k [b2 min(log(b2 h/s_k), 0) + b1 max(log(b1 h/s_k), 0)]
    (iii) and (iv) are non-decreasing and piecewise linear in log h with
    breakpoints log s_k -+ lam/eps (TV) and log s_k - log b_i (RG); where
    their zero set is an interval the smallest root is taken (for (iv) that
    interval is [max log s_k - log b2, min log s_k - log b1] when every s_k
    fits one band, and its left end is returned exactly).
    """
    alpha = np.asarray(alpha, np.float64)
    T = np.asarray(T, np.float64)
    A = alpha.sum()
    if F2.kind == "eq":
        return np.sum(alpha[:, None] * T, axis=0) / A
    if F2.kind == "kl":
        g = eps / (eps + F2.lam)
        return (lse(np.log(alpha)[:, None] + g * T, axis=0) - np.log(A)) / g
    al = alpha[:, None, None]
    if F2.kind == "tv":
        pos = np.isfinite(T)
        a0 = np.sum(np.where(pos, 0.0, alpha[:, None]), axis=0)
        a1 = np.sum(np.where(pos, alpha[:, None], 0.0), axis=0)
        d = F2.lam / eps
        Tp = np.where(pos, T, np.nan)

        def f(x):   # x: (m, J)
            t = np.clip((x[None, :, :] - Tp[:, None, :]) / d, -1.0, 1.0)
            return a0[None, :] + np.nansum(np.where(pos[:, None, :], al * t, 0.0), axis=0)
        br = np.concatenate([np.where(pos, T - d, np.inf), np.where(pos, T + d, np.inf)], axis=0)
        x = pwl_root_inf(f, br)
        return np.where(a0 >= a1, -np.inf, x)
    if F2.kind == "rg":
        b1, b2 = F2.alpha, F2.beta
        if not np.isfinite(b2):
            raise ValueError("a range barycentre needs a finite upper bound")
        zero = np.any(np.isneginf(T), axis=0)
        Tz = np.where(np.isneginf(T), 0.0, T)
        lb1 = np.log(b1) if b1 > 0 else -np.inf

        def f(x):
            y = x[None, :, :] - Tz[:, None, :]
            lo = b1 * np.maximum(y + lb1, 0.0) if b1 > 0 else 0.0
            return np.sum(al * (b2 * np.minimum(y + np.log(b2), 0.0) + lo), axis=0)
        br = [Tz - np.log(b2)]
        if b1 > 0:
            br.append(Tz - lb1)
        x = pwl_root_inf(f, np.concatenate(br, axis=0))
        # every input within one band [b1 h, b2 h]: the function is zero on
        # [max log s_k - log b2, min log s_k - log b1]; its left end is taken
        # exactly (evaluated at a breakpoint, the sum may round to -0)
        left = np.max(Tz, axis=0) - np.log(b2)
        band = left <= (np.min(Tz, axis=0) - lb1 if b1 > 0 else np.inf)
        return np.where(zero, -np.inf, np.where(band, left, x))
    raise ValueError("barycentre F2 kind %s is not supported" % F2.kind)


def barycenter(geom, logp, alpha, logdx, logdy, F1: Div, F2: Div, eps: float,
               tol: float = 1e-6, max_iter: int = 10000, v0=None):
    """Multi-coupling scaling iterations for the barycentre (Sec. 4.4 "Multiple
    couplings", Sec. 5.2).  For each k: S_k = log K(b_k dy),
    u_k = eps log proxdiv_F1(p_k)(e^S_k); T_k = log K^T(a_k dx); h from Table
    estimatebary; v_k = eps log proxdiv_F2(h)(e^T_k).  The residual is the
    relative L1 X-marginal violation aggregated over all k.
    Returns dict(u, v, logh, iters, res)."""
    logp = np.asarray(logp, np.float64)
    n, N = logp.shape
    M = len(logdy)
    v = np.zeros((n, M)) if v0 is None else np.array(v0, np.float64)
    u = np.zeros((n, N))
    res = []
    logh = None
    T = None
    for it in range(1, max_iter + 1):
        S = np.stack([geom.lse_x(expo(v[k], None if T is None else T[k], logdy, eps), eps) for k in range(n)])
        u_new = eps * proxdiv_log(F1, logp, S, 0.0, eps)
        # aggregated over every coupling
        r = marginal_residual(S, u, u_new, logdx, eps)
        u = u_new
        T = np.stack([geom.lse_y(expo(u[k], S[k], logdx, eps), eps) for k in range(n)])
        logh = bary_logh(T, alpha, eps, F2)
        v = eps * proxdiv_log(F2, np.broadcast_to(logh, T.shape), T, 0.0, eps)
        res.append(r)
        if r <= tol and it >= 2:
            return dict(u=u, v=v, logh=logh, iters=it, res=res, converged=True)
    return dict(u=u, v=v, logh=logh, iters=max_iter, res=res, converged=False)


# ---------------------------------------------------------------------------
# gradient flows (Sec. 5.3): each time step is one problem of the generic
# form, solved by the scaling iteration; the next density is read off the
# optimal coupling
# ---------------------------------------------------------------------------
def second_marginal_log(geom, u, v, logdx, eps, S=None):
    """log pi2 = log(R^T dx) = v/eps + T(u), the density of P^2_# R w.r.t. dy
    (S: the product u was computed from, for the vanishing-product rule)."""
    T = geom.lse_y(expo(u, S, logdx, eps), eps)
    return T + expo(v, T, 0.0, eps)


def growth_joint_pot(T, logq, lam, eps):
    """Y update of the multi-species growth step (Sec. 5.3, several species).
    The paper's joint proxdiv is e^{-u_k/eps} / beta(sum_k s_k e^{-u_k/eps})
    with beta(Z) = max(Z^{1/(1+eps)}, kappa^{1/eps}), kappa = 1 - lam, for the
    cap 1; with a cap q, Z is replaced by Z/q.  In potentials (u = 0 form):
    v = -eps log beta, the same for every species.  T: (S, M), T_k = log s_k."""
    T = np.atleast_2d(np.asarray(T, np.float64))
    logq = np.asarray(logq, np.float64)
    L = lse(T, axis=0)
    lk = np.log1p(-lam)
    with np.errstate(invalid="ignore"):
        logbeta = np.maximum((L - logq) / (1.0 + eps), lk / eps)
    v = np.where(np.isneginf(logq), -np.inf, -eps * logbeta)
    return np.broadcast_to(v, T.shape).copy()


def growth_next_log(logy, logq, lam):
    """Next densities of the growth flow from the second marginals y_k of the
    optimal couplings: the minimiser r_k of sum_k KL(y_k|r_k) - lam sum_k r_k
    under sum_k r_k <= q, i.e. r_k = y_k / max(kappa, sum_k y_k / q) (for one
    species min(y / kappa, q), as Sec. 5.3 states)."""
    logy = np.atleast_2d(np.asarray(logy, np.float64))
    logq = np.asarray(logq, np.float64)
    L = lse(logy, axis=0)
    with np.errstate(invalid="ignore"):
        den = np.maximum(np.log1p(-lam), L - logq)
    out = logy - den
    return np.where(np.isneginf(logq) | np.isneginf(logy), -np.inf, out)


def solve_species(geom, logp, logq, logdx, logdy, lam, eps, tol=1e-6, max_iter=10000, v0=None,
                  F1: Optional[Div] = None):
    """Scaling iterations of one step of the multi-species WF growth flow
    (Sec. 5.3; the several-couplings iteration of Sec. 4.4): S couplings R_k,
    F1 = KL(.|p_k) (lambda 1 unless given) on each first marginal and the joint
    growth functional of incentive lam and cap q on the sum of the second
    marginals.  Per iteration: S_k = log K(b_k dy), u_k = eps log
    proxdiv_F1(p_k)(e^{S_k}) for every k; then T_k = log K^T(a_k dx) and the
    joint v (growth_joint_pot).  The residual aggregates the X-marginal
    violations of all couplings; the first one never stops the loop.
    Returns dict(u, v, iters, res, converged)."""
    F1 = KL(1.0) if F1 is None else F1
    logp = np.atleast_2d(np.asarray(logp, np.float64))
    n, N = logp.shape
    M = len(logdy)
    v = np.zeros((n, M)) if v0 is None else np.array(np.broadcast_to(v0, (n, M)), np.float64)
    u = np.zeros((n, N))
    res = []
    T = None
    for it in range(1, max_iter + 1):
        S = np.stack([geom.lse_x(expo(v[k], None if T is None else T[k], logdy, eps), eps) for k in range(n)])
        u_new = eps * proxdiv_log(F1, logp, S, 0.0, eps)
        # aggregated over every coupling
        r = marginal_residual(S, u, u_new, logdx, eps)
        u = u_new
        T = np.stack([geom.lse_y(expo(u[k], S[k], logdx, eps), eps) for k in range(n)])
        v = growth_joint_pot(T, logq, lam, eps)
        res.append(r)
        if r <= tol and it >= 2:
            return dict(u=u, v=v, iters=it, res=res, converged=True, S=S)
    return dict(u=u, v=v, iters=max_iter, res=res, converged=False, S=S)


def flow(geom, kind: str, p0, q, dx, tau: float, eps: float, n_steps: int, iters: int,
         alpha: float = 0.0, tol: float = 0.0):
    """A time-discretised gradient flow (Sec. 5.3): n_steps steps, each solved
    by the scaling iteration (`iters` iterations, or to tol), warm-started with
    the previous step's v.  X = Y, dx = dy.
      "heat"  : F1 = iota_=(. | p_k), F2 = 2 tau KL(. | q): Wasserstein flow of
                KL(. | q dx); next density = pi2
      "crowd" : F1 = iota_=(. | p_k), F2 = iota_{<= q}: the projection step of
                the congested crowd model (its free evolution is another
                algorithm and not part of this); next density = pi2
      "growth": WF flow of -alpha mu(X) + iota_{<= q}: per species F1 = KL(. |
                p_k), the joint growth functional with lam = 2 tau alpha on the
                second marginals; next densities from growth_next_log
    p0: (S, N) initial densities (S = 1 unless kind is "growth").
    Returns (list of n_steps + 1 arrays (S, N), list of per-step info dicts)."""
    p = np.atleast_2d(np.asarray(p0, np.float64))
    q = np.asarray(q, np.float64)
    dx = np.asarray(dx, np.float64)
    logdx = np.log(dx)
    logq = safe_log(q)
    n = p.shape[0]
    if kind != "growth" and n != 1:
        raise ValueError("several species only for the growth flow")
    out = [p.copy()]
    infos = []
    v = None
    for _ in range(n_steps):
        logp = safe_log(p)
        if kind == "growth":
            lam = 2.0 * tau * alpha
            r = solve_species(geom, logp, logq, logdx, logdx, lam, eps, tol=tol, max_iter=iters, v0=v)
            logy = np.stack([second_marginal_log(geom, r["u"][k], r["v"][k], logdx, eps, r["S"][k])
                             for k in range(n)])
            p = np.exp(growth_next_log(logy, logq, lam))
            v = r["v"]
        else:
            F2 = KL(2.0 * tau) if kind == "heat" else RG(0.0, 1.0)
            r = solve(geom, logp[0], logq, logdx, logdx, EQ, F2, eps, tol=tol, max_iter=iters,
                      v0=None if v is None else v[0])
            p = np.exp(second_marginal_log(geom, r["u"], r["v"], logdx, eps, r["S"]))[None, :]
            v = r["v"][None, :]
        out.append(p.copy())
        infos.append(dict(iters=r["iters"], res=r["res"], converged=r["converged"]))
    return out, infos


# ---------------------------------------------------------------------------
# barycentric projection (colour transfer, Sec. 5.1): the approximate
# transport map T_i = sum_j R_ij dy_j y_j / sum_j R_ij dy_j
# ---------------------------------------------------------------------------
def barycentric_map_dense(C, Y, v, logdy, eps, rows=None):
    """T (len(rows) x d) straight from the plan's definition: row i of the plan
    w.r.t. dx is R_ij dy_j = exp((u_i + v_j - C_ij)/eps + log dy_j) and u_i
    cancels in the ratio.  C: cost rows (len(rows) x M) or the full matrix;
    Y: (M, d) coordinates of the points of Y.  A row with no mass gives NaN."""
    C = np.atleast_2d(np.asarray(C, np.float64))
    Y = np.asarray(Y, np.float64).reshape(C.shape[1], -1)
    with np.errstate(invalid="ignore"):
        L = np.where(np.isinf(C), -np.inf, (np.asarray(v)[None, :] - C) / eps + np.asarray(logdy)[None, :])
    m = np.max(L, axis=1, keepdims=True)
    with np.errstate(invalid="ignore"):
        W = np.exp(L - np.where(np.isfinite(m), m, 0.0))
        den = W.sum(axis=1, keepdims=True)
        return (W @ Y) / den


def grid_points(shape, h):
    """Cell centres (i + 1/2) h of a grid, (size, ndim), row-major."""
    axes = [(np.arange(n) + 0.5) * hh for n, hh in zip(shape, h)]
    mesh = np.meshgrid(*axes, indexing="ij")
    return np.stack([m.reshape(-1) for m in mesh], axis=1)


def barycentric_map_rows(geom, v, logdy, eps, rows):
    """T for the given rows of X on a grid or point geometry, one cost row at a
    time (no N x M matrix): the definition above, for large problems."""
    if isinstance(geom, GridGeom):
        P = grid_points(geom.shape, geom.h)
        Y = P
        d2 = ((P[rows][:, None, :] - P[None, :, :]) ** 2).sum(-1)
        C = make_cost(d2, geom.cost, geom.cut)
    else:
        raise TypeError("use barycentric_map_dense with the cost matrix")
    return barycentric_map_dense(C, Y, v, logdy, eps)


# ---------------------------------------------------------------------------
# batches: independent problems, one after the other
# ---------------------------------------------------------------------------
def mass_balance_shift(geom, logp, logq, logdx, logdy, F1: Div, F2: Div, eps: float, v0) -> float:
    """Constant shift s of a starting potential v0 (to be replaced by v0 - s)
    that balances the two estimates of the plan's total mass, for KL penalties
    on both marginals.  A refinement of a warm start: by Prop. "alternating"
    only v^(0) enters the iterates, so the iteration and its fixed point are
    unchanged.

    KL row of Table proximalexplicit: a = (p / K b)^theta1, theta1 =
    lam1/(lam1+eps), so the plan's first marginal a (K b) equals
    p a^(-eps/lam1) = p e^(-u/lam1); likewise at the fixed point the second
    marginal is q e^(-v/lam2), and both carry the plan's mass.  From v0, one
    X half-step gives u1 and
        P = sum_i p_i e^(-u1_i/lam1) dx_i,   Q = sum_j q_j e^(-v0_j/lam2) dy_j.
    Replacing v0 by v0 - s turns u1 into u1 + theta1 s (log K(b e^(-s/eps))
    = log K b - s/eps), P into P e^(-theta1 s/lam1) and Q into Q e^(s/lam2);
    they agree for s = log(P/Q) / (theta1/lam1 + 1/lam2).  Returns 0 when P
    or Q is 0.
    """
    if F1.kind != "kl" or F2.kind != "kl":
        raise ValueError("the mass balance takes KL penalties on both marginals")
    logp = np.asarray(logp, np.float64)
    logq = np.asarray(logq, np.float64)
    v0 = np.asarray(v0, np.float64)
    S = geom.lse_x(v0 / eps + logdy, eps)
    u1 = eps * proxdiv_log(F1, logp, S, 0.0, eps)
    with np.errstate(invalid="ignore"):
        tp = np.where(np.isneginf(logp), -np.inf, logp - u1 / F1.lam + logdx)
        tq = np.where(np.isneginf(logq), -np.inf, logq - v0 / F2.lam + logdy)
    lP, lQ = lse(tp, 0), lse(tq, 0)
    if not (np.isfinite(lP) and np.isfinite(lQ)):
        return 0.0
    th1 = F1.lam / (F1.lam + eps)
    return float((lP - lQ) / (th1 / F1.lam + 1.0 / F2.lam))


def solve_batch(problems, F1, F2, eps, tol, max_iter, **kw):
    """problems: iterable of (x, y, p, q, dx, dy); dense squared-Euclidean cost."""
    out = []
    for (x, y, p, q, dx, dy) in problems:
        g = PointsGeom(x, y)
        out.append(solve(g, safe_log(p), safe_log(q), np.log(dx), np.log(dy), F1, F2, eps, tol, max_iter, **kw))
    return out
