"""Synthetic coefficient fields and right-hand sides.

Array conventions (shared by every consumer):

* The unknowns sit at the interior grid points x = (x_1, ..., x_d), 1 <= x_k <= s, of a
  uniform grid with spacing h = 1/(s+1) on the unit cube; x = 0 and x = s+1 are the zero
  Dirichlet ghosts. The linear DOF index is sum_k (x_k - 1) s^(k-1), so x_1 runs fastest.
  A length-N vector reshaped with ``.reshape((s,)*d)`` is indexed [x_d-1, ..., x_1-1].
* The diffusion coefficient a is piecewise constant on the (s+1)^d grid cells; cell
  (c_1, ..., c_d), 0 <= c_k <= s, spans [c_k h, (c_k+1) h] in each direction. It is stored
  as an array of shape (s+1,)*d indexed [c_d, ..., c_1], so its C-order flattening again
  has c_1 fastest.
* Random numbers come from ``numpy.random.default_rng(seed)``; the coefficient field is
  drawn first and the right-hand side f second, from the same generator.

The fields follow the workloads of the numerical section of the paper (a high-contrast
random medium) and the synthetic log-normal media used to exercise the solver at scale.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy import ndimage


@dataclass
class Problem:
    """One SPD finite-difference problem  -div(a grad u) + b u = f  on (0,1)^d."""

    name: str
    d: int
    s: int                      # interior points per axis; N = s**d
    a_cells: np.ndarray         # (s+1,)*d cell coefficients, indexed [c_d, ..., c_1]
    b: Optional[np.ndarray]     # (N,) reaction term or None for b = 0
    f: np.ndarray               # (N,) right-hand side
    leaf: int                   # leaf cell width m (cells span m grid steps at level 0)
    eps: float                  # ID relative precision
    precond: int = 1            # 1 = recursively preconditioned (PHIF), 0 = plain HIF
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return self.s ** self.d

    @property
    def h(self) -> float:
        return 1.0 / (self.s + 1)


def two_valued_field(rng: np.random.Generator, d: int, s: int, lo: float, hi: float) -> np.ndarray:
    """iid per cell: ``lo`` with probability 1/2, else ``hi``."""
    u = rng.random((s + 1,) * d)
    return np.where(u < 0.5, lo, hi)


def gaussian_random_field(rng: np.random.Generator, d: int, s: int, corr_len: float) -> np.ndarray:
    """Standardized smooth Gaussian field on the (s+1)^d cells.

    White noise is convolved with an isotropic Gaussian kernel of standard deviation
    corr_len/sqrt(2) cells (so the field covariance decays like exp(-r^2 / (2 corr_len^2))),
    with reflecting ends, and then shifted and scaled to sample mean 0 and sample std 1.
    """
    z = rng.standard_normal((s + 1,) * d)
    g = ndimage.gaussian_filter(z, sigma=corr_len / np.sqrt(2.0), mode="reflect", truncate=4.0)
    g = g - g.mean()
    sd = g.std()
    return g / sd if sd > 0 else g


def quantized_paper_field(rng: np.random.Generator, d: int, s: int, lo=1e-2, hi=1e2, width_cells=4.0):
    """The high-contrast medium of the paper's numerical section: uniform samples, smoothed
    by an isotropic Gaussian of width 4h, then thresholded at the median to two values."""
    u = rng.random((s + 1,) * d)
    g = ndimage.gaussian_filter(u, sigma=width_cells, mode="reflect", truncate=4.0)
    mu = np.median(g)
    return np.where(g <= mu, lo, hi)


def _rhs(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.standard_normal(n)


def make_problem(kind: str, d: int, s: int, seed: int, leaf: int, eps: float, *,
                 lo: float = 1e-2, hi: float = 1e2, sigma: float = 3.0, corr_len: float = 8.0,
                 b_const: float = 0.0, precond: int = 1, name: Optional[str] = None) -> Problem:
    """Build a seeded problem.

    kind: "two_valued" (iid lo/hi per cell), "lognormal" (a = exp(sigma * GRF)),
          "paper" (quantized smoothed field), "constant" (a = 1).
    """
    rng = np.random.default_rng(seed)
    if kind == "two_valued":
        a = two_valued_field(rng, d, s, lo, hi)
    elif kind == "lognormal":
        a = np.exp(sigma * gaussian_random_field(rng, d, s, corr_len))
    elif kind == "paper":
        a = quantized_paper_field(rng, d, s, lo, hi)
    elif kind == "constant":
        a = np.ones((s + 1,) * d)
    else:
        raise ValueError(f"unknown field kind {kind!r}")
    n = s ** d
    f = _rhs(rng, n)
    b = np.full(n, float(b_const)) if b_const != 0.0 else None
    return Problem(name=name or f"{kind}-{d}d-{s}", d=d, s=s, a_cells=a, b=b, f=f,
                   leaf=leaf, eps=eps, precond=precond,
                   meta=dict(kind=kind, seed=seed, lo=lo, hi=hi, sigma=sigma,
                             corr_len=corr_len, b_const=b_const))


def _cfg1():
    return make_problem("two_valued", 2, 64, seed=0, leaf=8, eps=1e-3, lo=1e-2, hi=1e2,
                        name="2d-64-twovalued-eps1e-3")


def _cfg2(eps=1e-6):
    return make_problem("lognormal", 2, 512, seed=1, leaf=16, eps=eps, sigma=3.0, corr_len=8.0,
                        name=f"2d-512-lognormal-s3-eps{eps:g}")


def _cfg3():
    return make_problem("two_valued", 3, 64, seed=2, leaf=4, eps=1e-3, lo=1e-3, hi=1e3,
                        b_const=1e-2, name="3d-64-twovalued-eps1e-3")


def batch_problem(k: int, eps: float = 1e-4) -> Problem:
    """Problem k of the batch of uneven 2D problems: its side is drawn first from
    default_rng(k), then its field and its right-hand side."""
    rng = np.random.default_rng(k)
    s = int(rng.choice([128, 192, 256, 384, 512]))
    a = np.exp(2.0 * gaussian_random_field(rng, 2, s, 8.0))
    f = _rhs(rng, s * s)
    return Problem(name=f"batch{k}-2d-{s}", d=2, s=s, a_cells=a, b=None, f=f, leaf=16, eps=eps,
                   meta=dict(kind="lognormal", seed=k, sigma=2.0, corr_len=8.0))


CONFIGS = {
    "cfg1": _cfg1,
    "cfg2": _cfg2,
    "cfg3": _cfg3,
}
