"""Seeded synthetic inputs for entropic unbalanced OT workloads.

This module only draws and shapes input data (point clouds, histograms,
reference weights).  It holds none of the scaling method's arithmetic, so both
the GPU path and the CPU oracle can take their inputs from it.

Every generator uses ``numpy.random.default_rng(seed)`` (PCG64) in float64.
Densities are returned with respect to the reference weights ``dx`` / ``dy``
(p = mu / dx), which is the convention of the paper's UOT section (Sec. 5.1,
p = d mu / dx).  Float32 workloads round the float64 draws once; both sides
then read the same rounded values.

The paper's own marginals and images exist only as figures, so the recipes
below stand in for them with the shapes of its experiments (1-D grids,
2-D grids, point clouds, barycentres of blob images).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np


# ---------------------------------------------------------------------------
# containers
# ---------------------------------------------------------------------------
@dataclass
class GridProblem:
    """Two densities on the same regular grid of cell centres.

    shape: grid shape (n1,) / (n1, n2) / (n1, n2, n3); h: spacing per axis;
    p, q: densities w.r.t. the cell weights dx = dy = prod(h), row-major.
    """
    shape: tuple
    h: tuple
    p: np.ndarray
    q: np.ndarray

    @property
    def size(self) -> int:
        return int(np.prod(self.shape))

    def coords(self) -> np.ndarray:
        """Cell-centre coordinates, shape (size, ndim), row-major order."""
        axes = [(np.arange(n) + 0.5) * hh for n, hh in zip(self.shape, self.h)]
        mesh = np.meshgrid(*axes, indexing="ij")
        return np.stack([m.reshape(-1) for m in mesh], axis=1)

    def cell_weight(self) -> float:
        return float(np.prod(self.h))


@dataclass
class CloudProblem:
    """Two weighted point clouds.  x: (N, d), y: (M, d); p, q densities w.r.t.
    dx, dy (arrays of positive reference weights)."""
    x: np.ndarray
    y: np.ndarray
    p: np.ndarray
    q: np.ndarray
    dx: np.ndarray
    dy: np.ndarray


@dataclass
class BaryProblem:
    """n densities on one regular grid, with barycentre weights alpha."""
    shape: tuple
    h: tuple
    p: np.ndarray          # (n, size)
    alpha: np.ndarray      # (n,)


# ---------------------------------------------------------------------------
# building blocks (sampling only)
# ---------------------------------------------------------------------------
def _gauss_mixture_1d(rng, centres, n_comp, mean_lo, mean_hi, sig_lo, sig_hi):
    means = rng.uniform(mean_lo, mean_hi, n_comp)
    sig = rng.uniform(sig_lo, sig_hi, n_comp)
    w = rng.uniform(0.5, 1.5, n_comp)
    w = w / w.sum()
    g = np.zeros_like(centres)
    for k in range(n_comp):
        g += w[k] * np.exp(-0.5 * ((centres - means[k]) / sig[k]) ** 2) / (sig[k] * np.sqrt(2 * np.pi))
    return g


def _blobs_2d(rng, shape, n_blobs, floor):
    n1, n2 = shape
    c1 = (np.arange(n1) + 0.5) / n1
    c2 = (np.arange(n2) + 0.5) / n2
    X1, X2 = np.meshgrid(c1, c2, indexing="ij")
    g = np.full(shape, floor, dtype=np.float64)
    for _ in range(n_blobs):
        m = rng.uniform(0.15, 0.85, 2)
        s = rng.uniform(0.03, 0.1)
        a = rng.uniform(0.5, 1.5)
        g += a * np.exp(-0.5 * ((X1 - m[0]) ** 2 + (X2 - m[1]) ** 2) / s ** 2)
    return g


def _to_density(g, cell_w, mass):
    """Scale a nonnegative profile so that sum(p * cell_w) == mass."""
    return g * (mass / (g.sum() * cell_w))


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def hist1d(seed: int, n: int = 256, masses=(1.0, 1.5)) -> GridProblem:
    """1-D UOT between two 3-component Gaussian mixtures on n cell centres of
    [0, 1] (dx = 1/n).  Means U[0.1, 0.9], sigma U[0.02, 0.1], component weights
    U[0.5, 1.5] normalised; total masses 1.0 and 1.5.  No floor: densities may
    underflow to exact zeros far from every component."""
    rng = np.random.default_rng(seed)
    centres = (np.arange(n) + 0.5) / n
    h = 1.0 / n
    gp = _gauss_mixture_1d(rng, centres, 3, 0.1, 0.9, 0.02, 0.1)
    gq = _gauss_mixture_1d(rng, centres, 3, 0.1, 0.9, 0.02, 0.1)
    return GridProblem((n,), (h,), _to_density(gp, h, masses[0]), _to_density(gq, h, masses[1]))


def blobs2d(seed: int, n: int = 256, n_blobs: int = 5, floor: float = 1e-6) -> GridProblem:
    """2-D grid UOT: n x n cell centres on [0,1]^2; each side is a sum of 5
    Gaussian blobs (centres U[0.15,0.85]^2, sigma U[0.03,0.1], amplitude
    U[0.5,1.5]) plus a 1e-6 floor, scaled to a total mass U[0.5, 2]."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    gp = _blobs_2d(rng, (n, n), n_blobs, floor)
    gq = _blobs_2d(rng, (n, n), n_blobs, floor)
    mp, mq = rng.uniform(0.5, 2.0, 2)
    cw = h * h
    return GridProblem((n, n), (h, h), _to_density(gp, cw, mp).reshape(-1),
                       _to_density(gq, cw, mq).reshape(-1))


def clouds3d(seed: int, N: int = 20000, M: int = 20000, n_comp: int = 8,
             shift=(0.15, 0.0, 0.0)) -> CloudProblem:
    """Dense point-cloud UOT in R^3: X from an 8-component isotropic Gaussian
    mixture (means U[0.2,0.8]^3, sigma U[0.03,0.1], weights U[0.5,1.5]
    normalised); Y from the same means shifted by `shift` with fresh sigmas and
    weights.  Point masses U[0.5,1.5]/N with dx = 1/N, so p = U[0.5,1.5]."""
    rng = np.random.default_rng(seed)
    means = rng.uniform(0.2, 0.8, (n_comp, 3))

    def draw(n, mu):
        sig = rng.uniform(0.03, 0.1, n_comp)
        w = rng.uniform(0.5, 1.5, n_comp)
        w /= w.sum()
        comp = rng.choice(n_comp, size=n, p=w)
        return mu[comp] + sig[comp, None] * rng.standard_normal((n, 3))

    x = draw(N, means)
    y = draw(M, means + np.asarray(shift)[None, :])
    p = rng.uniform(0.5, 1.5, N)
    q = rng.uniform(0.5, 1.5, M)
    return CloudProblem(x, y, p, q, np.full(N, 1.0 / N), np.full(M, 1.0 / M))


def uniform_clouds(rng, N: int, M: int, d: int = 2) -> CloudProblem:
    """Uniform points in [0,1]^d with densities U[0.1, 1] w.r.t. dx = 1/N."""
    x = rng.uniform(0.0, 1.0, (N, d))
    y = rng.uniform(0.0, 1.0, (M, d))
    p = rng.uniform(0.1, 1.0, N)
    q = rng.uniform(0.1, 1.0, M)
    return CloudProblem(x, y, p, q, np.full(N, 1.0 / N), np.full(M, 1.0 / M))


def ragged_batch(seed: int, B: int = 4096, lo: int = 64, hi: int = 4096, d: int = 2) -> List[CloudProblem]:
    """B independent problems, sizes N, M ~ log-uniform on [lo, hi] (rounded),
    uniform points in [0,1]^d with densities U[0.1,1] w.r.t. dx = 1/N."""
    rng = np.random.default_rng(seed)
    Ns = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), B))).astype(np.int64)
    Ms = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), B))).astype(np.int64)
    return [uniform_clouds(rng, int(n), int(m), d) for n, m in zip(Ns, Ms)]


def ragged_sizes(seed: int, B: int = 4096, lo: int = 64, hi: int = 4096):
    """Only the (N, M) sizes that `ragged_batch` would draw for the same seed."""
    rng = np.random.default_rng(seed)
    Ns = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), B))).astype(np.int64)
    Ms = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), B))).astype(np.int64)
    return Ns, Ms


def bary_blobs(seed: int, n_marg: int = 8, n: int = 128, n_blobs: int = 5,
               floor: float = 1e-6) -> BaryProblem:
    """n_marg blob images on an n x n grid of [0,1]^2 (recipe of `blobs2d`),
    each scaled to a mass U[0.5, 2]; barycentre weights alpha_k = 1/n_marg."""
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    cw = h * h
    ps = []
    for _ in range(n_marg):
        g = _blobs_2d(rng, (n, n), n_blobs, floor)
        ps.append(_to_density(g, cw, rng.uniform(0.5, 2.0)).reshape(-1))
    return BaryProblem((n, n), (h, h), np.stack(ps), np.full(n_marg, 1.0 / n_marg))


def pair_blobs(seed: int, n: int = 64) -> GridProblem:
    """One training pair for the warm-start network: two n x n blob images."""
    return blobs2d(seed, n=n)


# ---------------------------------------------------------------------------
# spatially coherent point order (for kernels with exact zeros beyond a cut
# locus, whose tiles can only be skipped when nearby points sit together)
# ---------------------------------------------------------------------------
def morton_order(x: np.ndarray, bits: int = 10) -> np.ndarray:
    """Indices sorting points x (N, d) of [0, 1]^d along a Z-order (Morton)
    curve: coordinates quantised to 2^bits levels, bits interleaved."""
    x = np.atleast_2d(np.asarray(x, np.float64))
    N, d = x.shape
    q = np.clip((x * (1 << bits)).astype(np.int64), 0, (1 << bits) - 1)
    code = np.zeros(N, np.int64)
    for b in range(bits):
        for k in range(d):
            code |= ((q[:, k] >> b) & 1) << (b * d + k)
    return np.argsort(code, kind="stable")


def clusters_sorted(seed: int, N: int = 20000, M: int = 20000, d: int = 2, n_comp: int = 12,
                    sig_lo: float = 0.03, sig_hi: float = 0.12) -> CloudProblem:
    """Two clouds of Gaussian clusters in [0, 1]^d (clipped), each stored in
    Morton order; uniform reference weights 1/N, 1/M and densities
    U[0.5, 1.5] times the masses 1 and 1.3."""
    rng = np.random.default_rng(seed)

    def cloud(n):
        c = rng.uniform(0.15, 0.85, (n_comp, d))
        s = rng.uniform(sig_lo, sig_hi, n_comp)
        lab = rng.integers(0, n_comp, n)
        pts = np.clip(c[lab] + s[lab, None] * rng.standard_normal((n, d)), 0.0, 1.0)
        return pts[morton_order(pts)]

    x, y = cloud(N), cloud(M)
    dx, dy = np.full(N, 1.0 / N), np.full(M, 1.0 / M)
    p = rng.uniform(0.5, 1.5, N)
    q = rng.uniform(0.5, 1.5, M) * 1.3
    return CloudProblem(x, y, p, q, dx, dy)


# ---------------------------------------------------------------------------
# gradient flows on [0, 1] (Sec. 5.3 experiments: n uniform cells)
# ---------------------------------------------------------------------------
def growth_profile_1d(seed: int, n: int = 3000, species: int = 1, floor: float = 1e-3) -> np.ndarray:
    """Initial densities (species, n) for the growth flows, w.r.t. the cell
    width 1/n: a plateau at the cap 1 with smooth shoulders and a few smaller
    bumps (the shape of the tumour example's initial profile), at least
    `floor`.  Several species split the profile with smooth random weights
    (their sum keeps the shape)."""
    rng = np.random.default_rng(seed)
    t = (np.arange(n) + 0.5) / n
    a, b = np.sort(rng.uniform(0.25, 0.55, 2))
    w = rng.uniform(0.02, 0.05)
    plateau = 0.5 * (np.tanh((t - a) / w) - np.tanh((t - b - 0.1) / w))
    bumps = sum(rng.uniform(0.2, 0.6) * np.exp(-0.5 * ((t - rng.uniform(0.1, 0.9)) / rng.uniform(0.02, 0.06)) ** 2)
                for _ in range(3))
    prof = np.clip(np.maximum(plateau, bumps), floor, 1.0)
    if species == 1:
        return prof[None, :]
    raw = np.stack([1.0 + 0.8 * np.sin(2 * np.pi * (rng.uniform(0.5, 2.0) * t + rng.uniform())) for _ in range(species)])
    wts = raw / raw.sum(axis=0)
    return np.maximum(prof[None, :] * wts, floor / species)


# ---------------------------------------------------------------------------
# colour histograms (colour-transfer experiment, Sec. 5.1): the colours of an
# image in a cube X = [0, 1]^3 (luminance, two chrominances), binned on a
# 64 x 32 x 32 grid with unit reference mass per bin
# ---------------------------------------------------------------------------
def colour_histograms(seed: int, shape=(64, 32, 32), n_pixels: int = 512 * 512, n_modes: int = 6) -> GridProblem:
    """Two synthetic images' colour histograms.  Each image's pixel colours
    come from a mixture of n_modes anisotropic Gaussians (luminance spread
    widely, chrominance tightly, as in natural images), clipped to the cube
    and binned; p, q = bin counts / n_pixels (mass 1 each) w.r.t. dx = dy = 1.
    Most bins are empty, as in real colour histograms."""
    rng = np.random.default_rng(seed)
    shape = tuple(int(s) for s in shape)
    h = tuple(1.0 / s for s in shape)

    def hist():
        w = rng.dirichlet(np.full(n_modes, 2.0))
        lab = rng.choice(n_modes, n_pixels, p=w)
        mu = np.column_stack([rng.uniform(0.15, 0.85, n_modes), rng.uniform(0.3, 0.7, (n_modes, 2))])
        sd = np.column_stack([rng.uniform(0.05, 0.15, n_modes), rng.uniform(0.01, 0.04, (n_modes, 2))])
        c = np.clip(mu[lab] + sd[lab] * rng.standard_normal((n_pixels, 3)), 0.0, 1.0 - 1e-9)
        idx = [np.minimum((c[:, k] * shape[k]).astype(np.int64), shape[k] - 1) for k in range(3)]
        flat = np.ravel_multi_index(idx, shape)
        return np.bincount(flat, minlength=int(np.prod(shape))).astype(np.float64) / n_pixels

    return GridProblem(shape, h, hist(), hist())
