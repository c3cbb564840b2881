"""Seeded inputs for the GPU parity tests: the named workloads at test sizes,
plus adversarial layouts (ties, duplicates, degenerate lines, extreme
scales, exact and ragged powers of four)."""
import numpy as np

from paper_1006_2269_amd import workloads as W


def _ties(n, seed):
    g = W.rng(seed)
    x = np.round(g.random(n), 2)
    y = np.round(g.random(n), 2)
    return W.PointSet("ties", x, y, g.uniform(-1, 1, n))


def _duplicates(n, seed):
    g = W.rng(seed)
    base = g.random((n // 8, 2))
    idx = g.integers(0, base.shape[0], n)
    return W.PointSet("duplicates", base[idx, 0].copy(), base[idx, 1].copy(), g.uniform(-1, 1, n))


def _vertical(n, seed):
    g = W.rng(seed)
    return W.PointSet("vertical", np.full(n, 0.25), g.random(n), g.uniform(-1, 1, n))


def _scales(n, seed):
    g = W.rng(seed)
    x = np.sign(g.uniform(-1, 1, n)) * 10.0 ** g.uniform(-12, 12, n)
    y = np.sign(g.uniform(-1, 1, n)) * 10.0 ** g.uniform(-12, 12, n)
    return W.PointSet("scales", x, y, g.uniform(-1, 1, n))


def _negative_zero(n, seed):
    ps = W.uniform(n, seed)
    ps.x[: n // 10] = 0.0
    ps.x[n // 10: n // 5] = -0.0
    ps.y[: n // 7] = -0.0
    return ps


# name -> (maker, levels)
TREE_CASES = {
    "uniform_1k_L3": (lambda: W.uniform(1000, 3), 3),
    "ties_3k_L4": (lambda: _ties(3000, 4), 4),
    "grid_L4": (lambda: W.grid(4), 4),
    "exact_4pow5": (lambda: W.uniform(4 ** 5, 5), 5),
    "ragged_4pow5_plus1": (lambda: W.uniform(4 ** 5 + 1, 6), 5),
    "prime_10007_L5": (lambda: W.uniform(10007, 7), 5),
    "duplicates_4k_L4": (lambda: _duplicates(4000, 8), 4),
    "vertical_2k_L3": (lambda: _vertical(2000, 9), 3),
    "scales_3k_L4": (lambda: _scales(3000, 10), 4),
    "negzero_2k_L4": (lambda: _negative_zero(2000, 11), 4),
    "single_box_L0": (lambda: W.uniform(7, 12), 0),
    "uniform_10k_L5": (lambda: W.uniform_10k(), 5),
    # fine depths finished in LDS from depth 3 (odd: the x split lines of
    # depth 2 come from the global passes)
    "uniform_20k_L5": (lambda: W.uniform(20000, 13), 5),
    # leaves of 50 and 63 points: the FP32 near field in four chunks of 16
    # targets per leaf (one block of four wavefronts per list segment)
    "uniform_3200_L3": (lambda: W.uniform(3200, 14), 3),
    # leaves of 39 points: the pair-once near field with 4 chunks of 10
    # targets per leaf
    "uniform_2500_L3": (lambda: W.uniform(2500, 16), 3),
    # leaves of 45 and 46 points: 4 chunks of 12 targets
    "uniform_2900_L3": (lambda: W.uniform(2900, 17), 3),
    "duplicates_4k_L3": (lambda: _duplicates(4000, 8), 3),
    # leaves of 125 points: more than one point per lane in the
    # wavefront-per-leaf multipole kernel
    "uniform_2000_L2": (lambda: W.uniform(2000, 15), 2),
    "mixed_scaled_20k_L6": (lambda: W.mixed_1m(scale=0.02), 6),
    "clustered_scaled_20k_L6": (lambda: W.clustered_10m(scale=0.002), 6),
    "clustered_scaled_30k_L6": (lambda: W.clustered_10m(scale=0.003, seed=2003), 6),
    "ring_scaled_20k_L6": (lambda: W.ring_4m(scale=0.005), 6),
}
