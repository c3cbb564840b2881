"""The relaxed criterion's bins: the least grid threshold at which
Criterion 2.1 holds (the oracle's definition, a scan from the lowest) is
what a bisection over the grid finds (the GPU's search) as long as the
binary64 criterion is monotone in t along the grid: once true, true for
every larger threshold.  Checked with the oracle's own criterion on every
candidate pair of three trees and on pairs placed at the thresholds (theta_i
= R / (d - r) equal to a grid value, or one rounding either side of it).
"""
import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


def grid(theta, theta_max, k0=16, k1=16):
    return [theta * float(k + 1) / float(k0) for k in range(k0)] + \
        [theta + (theta_max - theta) * float(k + 1) / float(k1) for k in range(k1)]


def check_pair(orc, tk, gb, gc):
    seq = [orc.theta_test(t, gb, gc) for t in tk]
    first = seq.index(True) if True in seq else len(seq)
    assert all(seq[first:]), "criterion true at a threshold and false at a larger one"
    lo, hi = 0, len(tk)
    while lo < hi:  # the GPU's bisection
        mid = (lo + hi) // 2
        if seq[mid]:
            hi = mid
        else:
            lo = mid + 1
    assert lo == first
    return first


@pytest.mark.parametrize("maker,L", [(lambda: W.clustered_10m(scale=2e-4), 3),
                                     (lambda: W.ring_4m(scale=4e-4), 4),
                                     (lambda: W.mixed_1m(scale=1.5e-3), 3)])
@pytest.mark.parametrize("theta,theta_max", [(0.5, 0.9), (0.35, 0.8)])
def test_candidates_of_real_trees(orc, maker, L, theta, theta_max):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists(t, 0.3)  # a small theta: many strong pairs, so many candidates
    tk = grid(theta, theta_max)
    seen = 0
    for l in range(1, L + 1):
        G = t.level_geom(l)
        sp, si = ls.sptr[l - 1], ls.sidx[l - 1]
        for b in range(4 ** l):
            for q in si[sp[b // 4]:sp[b // 4 + 1]]:
                for c in range(4 * q, 4 * q + 4):
                    check_pair(orc, tk, G[b], G[c])
                    seen += 1
    assert seen > 1000


def test_pairs_placed_at_the_thresholds(orc):
    rng = np.random.default_rng(3)
    tk = grid(0.5, 0.9)
    for k, t in enumerate(tk):
        for _ in range(40):
            R = float(rng.uniform(0.1, 2.0)) * 2.0 ** int(rng.integers(-20, 20))
            r = R * float(rng.uniform(0.05, 1.0))
            d = R / t + r  # theta_i = t in exact arithmetic
            ang = float(rng.uniform(0, 2 * np.pi))
            gb = np.array([0.3, -0.7, R])
            for dd in (np.nextafter(d, 0), d, np.nextafter(d, np.inf)):
                gc = np.array([0.3 + dd * np.cos(ang), -0.7 + dd * np.sin(ang), r])
                first = check_pair(orc, tk, gb, gc)
                assert abs(first - k) <= 1  # lands on its own threshold or a neighbour
