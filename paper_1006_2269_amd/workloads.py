"""Seeded synthetic point sets and charges.

This module only draws random numbers: it holds none of the method's
arithmetic, and it is the one piece that both the GPU path and the CPU oracle
use, so that both see bit-identical inputs.  Every generator takes a seed and
uses ``numpy.random.Generator(PCG64(seed))``.

The paper's own workloads are synthetic point clouds (Section 5): uniform and
1/r-radial densities in the unit disc for the error-vs-p experiment, and
normal / "layer" layouts forced into the unit square by rejection for the
adaptivity and robustness experiments.  The named workloads below follow the
same style at the sizes this library is measured on:

* ``uniform_10k``       10,000 points uniform in [0,1]^2, charges U[-1,1].
* ``mixed_1m``          500,000 uniform plus 4 x 125,000 Gaussian points
                        (sigma 0.1, 0.03, 0.01, 0.003), charges U[-1,1].
* ``clustered_10m``     1,000,000 uniform plus 3 x 3,000,000 Gaussian points
                        (sigma 1e-3, 1e-2, 1e-1), charges +-1.
* ``ring_4m``           2,000,000 points on a noisy circle (radius 0.4,
                        radial noise sd 1e-3) plus 2,000,000 uniform.
* ``random_mixture``    1-8 Gaussian clusters with sigma in [1e-3, 1e-1],
                        Dirichlet(1) weights (parameter-selector layouts).

Cluster centres are drawn from U[0.2, 0.8]^2 and Gaussian samples falling
outside the unit square are redrawn (rejection, as in Section 5).  Every
workload also scales down by a factor (``scale``) keeping its mixture
fractions, so that the same recipe gives test-sized inputs.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


@dataclass
class PointSet:
    name: str
    x: np.ndarray  # float64 [n]
    y: np.ndarray  # float64 [n]
    q: np.ndarray  # float64 [n]

    @property
    def n(self) -> int:
        return int(self.x.shape[0])


def _uniform_square(g, n):
    return g.random(n), g.random(n)


def _gaussian_in_square(g, n, mu, sigma):
    """n samples of N(mu, sigma^2 I) restricted to [0,1]^2 by rejection."""
    xs = np.empty(n)
    ys = np.empty(n)
    filled = 0
    while filled < n:
        m = max(16, int(1.3 * (n - filled)) + 16)
        px = g.normal(mu[0], sigma, m)
        py = g.normal(mu[1], sigma, m)
        ok = (px >= 0.0) & (px <= 1.0) & (py >= 0.0) & (py <= 1.0)
        px, py = px[ok], py[ok]
        take = min(n - filled, px.shape[0])
        xs[filled:filled + take] = px[:take]
        ys[filled:filled + take] = py[:take]
        filled += take
    return xs, ys


def _charges_uniform(g, n):
    return g.uniform(-1.0, 1.0, n)


def _charges_sign(g, n):
    return np.where(g.random(n) < 0.5, -1.0, 1.0)


def _shuffle(g, x, y):
    order = g.permutation(x.shape[0])
    return x[order], y[order]


def uniform(n: int, seed: int = 1, name: str = "uniform") -> PointSet:
    g = rng(seed)
    x, y = _uniform_square(g, n)
    return PointSet(name, x, y, _charges_uniform(g, n))


def uniform_10k(scale: float = 1.0, seed: int = 1001) -> PointSet:
    n = max(16, int(round(10_000 * scale)))
    return uniform(n, seed, "uniform_10k")


def mixed_1m(scale: float = 1.0, seed: int = 1002) -> PointSet:
    g = rng(seed)
    nu = int(round(500_000 * scale))
    nc = int(round(125_000 * scale))
    xs, ys = [], []
    x, y = _uniform_square(g, nu)
    xs.append(x); ys.append(y)
    for sigma in (0.1, 0.03, 0.01, 0.003):
        mu = g.uniform(0.2, 0.8, 2)
        x, y = _gaussian_in_square(g, nc, mu, sigma)
        xs.append(x); ys.append(y)
    x, y = _shuffle(g, np.concatenate(xs), np.concatenate(ys))
    return PointSet("mixed_1m", x, y, _charges_uniform(g, x.shape[0]))


def clustered_10m(scale: float = 1.0, seed: int = 1003) -> PointSet:
    g = rng(seed)
    nu = int(round(1_000_000 * scale))
    nc = int(round(3_000_000 * scale))
    xs, ys = [], []
    x, y = _uniform_square(g, nu)
    xs.append(x); ys.append(y)
    for sigma in (1e-3, 1e-2, 1e-1):
        mu = g.uniform(0.2, 0.8, 2)
        x, y = _gaussian_in_square(g, nc, mu, sigma)
        xs.append(x); ys.append(y)
    x, y = _shuffle(g, np.concatenate(xs), np.concatenate(ys))
    return PointSet("clustered_10m", x, y, _charges_sign(g, x.shape[0]))


def ring_4m(scale: float = 1.0, seed: int = 1004) -> PointSet:
    g = rng(seed)
    nr = int(round(2_000_000 * scale))
    nu = int(round(2_000_000 * scale))
    ang = g.uniform(0.0, 2.0 * np.pi, nr)
    rad = 0.4 + g.normal(0.0, 1e-3, nr)
    xr = 0.5 + rad * np.cos(ang)
    yr = 0.5 + rad * np.sin(ang)
    xu, yu = _uniform_square(g, nu)
    x, y = _shuffle(g, np.concatenate([xr, xu]), np.concatenate([yr, yu]))
    return PointSet("ring_4m", x, y, _charges_uniform(g, x.shape[0]))


def random_mixture(n: int, seed: int) -> PointSet:
    """1-8 Gaussian clusters, sigma = 10^U[-3,-1], Dirichlet(1) weights."""
    g = rng(seed)
    k = int(g.integers(1, 9))
    sig = 10.0 ** g.uniform(-3.0, -1.0, k)
    w = g.dirichlet(np.ones(k))
    counts = np.floor(w * n).astype(np.int64)
    counts[0] += n - counts.sum()
    xs, ys = [], []
    for c in range(k):
        if counts[c] == 0:
            continue
        mu = g.uniform(0.2, 0.8, 2)
        x, y = _gaussian_in_square(g, int(counts[c]), mu, float(sig[c]))
        xs.append(x); ys.append(y)
    x, y = _shuffle(g, np.concatenate(xs), np.concatenate(ys))
    return PointSet("random_mixture", x, y, _charges_uniform(g, n))


def selector_layout(seed: int, log10_lo: float = 4.0, log10_hi: float = 6.3) -> PointSet:
    """Layouts for training and testing the parameter selector: N =
    round(10^U[lo, hi]), a random_mixture of 1-8 Gaussian clusters, and with
    probability 1/2 a uniform background holding a U[0.2, 0.8] share of the
    points (the benchmark sets mix clusters with a uniform background)."""
    g = rng(2 * seed + 1)
    n = int(round(10.0 ** g.uniform(log10_lo, log10_hi)))
    share = g.uniform(0.2, 0.8) if g.random() < 0.5 else 0.0
    nu = int(round(share * n))
    ps = random_mixture(n - nu, seed) if n - nu > 0 else None
    if nu == 0:
        return PointSet("selector_layout", ps.x, ps.y, ps.q)
    xu, yu = _uniform_square(g, nu)
    x = np.concatenate([ps.x, xu]) if ps is not None else xu
    y = np.concatenate([ps.y, yu]) if ps is not None else yu
    x, y = _shuffle(g, x, y)
    return PointSet("selector_layout", x, y, _charges_uniform(g, n))


def unit_disc(n: int, seed: int, radial_inverse: bool = False) -> PointSet:
    """Unit-disc layouts of the error-vs-p experiment: uniform density, or
    radial density proportional to 1/r (radius uniform in [0,1]).  Total
    mass 1 (equal positive charges)."""
    g = rng(seed)
    ang = g.uniform(0.0, 2.0 * np.pi, n)
    rad = g.random(n) if radial_inverse else np.sqrt(g.random(n))
    x = rad * np.cos(ang)
    y = rad * np.sin(ang)
    return PointSet("disc_1r" if radial_inverse else "disc_uniform", x, y, np.full(n, 1.0 / n))


def normal_corner(n: int, seed: int, sigma: float = 0.1) -> PointSet:
    """The 'normal' layout of Section 5's second and third experiments:
    N(0, sigma^2 I) forced into the unit square by rejection, so the points
    cluster at the origin corner.  Charges U[-1,1]."""
    g = rng(seed)
    x, y = _gaussian_in_square(g, n, (0.0, 0.0), sigma)
    return PointSet("normal", x, y, _charges_uniform(g, n))


def layer(n: int, seed: int, sigma: float = 0.1) -> PointSet:
    """The 'layer' layout of the same experiments: x uniform in [0,1] and y
    from N(0, sigma^2) forced into [0,1] by rejection, so the points cluster
    along the x-axis.  Charges U[-1,1]."""
    g = rng(seed)
    x = g.random(n)
    y = np.empty(n)
    filled = 0
    while filled < n:
        m = max(16, int(2.2 * (n - filled)) + 16)
        py = g.normal(0.0, sigma, m)
        py = py[(py >= 0.0) & (py <= 1.0)]
        take = min(n - filled, py.shape[0])
        y[filled:filled + take] = py[:take]
        filled += take
    return PointSet("layer", x, y, _charges_uniform(g, n))


def grid(levels: int, per_axis_factor: int = 2, seed: int = 7) -> PointSet:
    """Cell centres ((i + 1/2) / m, (j + 1/2) / m) of an m x m grid with
    m = per_axis_factor * 2^levels, listed in a seeded random order, with
    charges U[-1,1]."""
    m = per_axis_factor * (2 ** levels)
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    x = (i.ravel() + 0.5) / m
    y = (j.ravel() + 0.5) / m
    g = rng(seed)
    x, y = _shuffle(g, x, y)
    return PointSet("grid", x, y, _charges_uniform(g, x.shape[0]))


WORKLOADS = {
    "uniform_10k": uniform_10k,
    "mixed_1m": mixed_1m,
    "clustered_10m": clustered_10m,
    "ring_4m": ring_4m,
}


def sample_targets(n: int, m: int, seed: int = 4242) -> np.ndarray:
    """m distinct target indices drawn without replacement (all when m >= n)."""
    if m >= n:
        return np.arange(n, dtype=np.int64)
    g = rng(seed)
    return np.sort(g.choice(n, size=m, replace=False)).astype(np.int64)
