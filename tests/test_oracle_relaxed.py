"""Pins of the oracle's locally relaxed theta-criterion (Section 4, last
paragraph: differing theta_i are admitted while the mean of theta_i^(p+1)
over the observed values stays at most theta^(p+1)).

* With theta_max = theta the relaxed lists are the plain ones.
* Brute force in exact rational arithmetic, written here on its own: each
  candidate's bin is the least grid threshold for which Criterion 2.1 holds
  exactly on the binary64 geometry, the admitted bin range is the longest
  one whose exact mean of t^(p+1) stays within theta^(p+1), and the lists of
  every level follow from the brute force's own strong lists of the level
  above.  Counts, admitted range and lists must agree with the oracle.
* The mean condition holds with each weak pair's own theta_i = R / (d - r)
  (the grid only over-estimates it), and the next bin would break it.
* Relaxation only moves pairs from strong to weak: every strong list is a
  subset of the plain one, and every (target leaf, source leaf) pair is
  still served exactly once.
* The FMM on relaxed lists keeps the a-priori model's bound
  0.1 theta^(p+1) / (1 - theta)^2 and, where that bound is below rounding
  (theta <= 1/2 at p = 60), reproduces the direct sum to rounding;
  promoting every candidate up to theta_max without the mean condition
  does not (so the condition is what keeps the error).
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


def _rows(ptr, idx, b):
    return idx[ptr[b]:ptr[b + 1]].tolist()


def grid(theta, theta_max, k0, k1):
    # the thresholds as binary64 expressions, evaluated as stated
    return [theta * float(k + 1) / float(k0) for k in range(k0)] + \
        [theta + (theta_max - theta) * float(k + 1) / float(k1) for k in range(k1)]


def passes_exact(t, gb, gc):
    """Criterion 2.1, R + t r <= t d, in exact arithmetic (d > 0)."""
    t = Fraction(t)
    xb, yb, rb = (Fraction(v) for v in gb)
    xc, yc, rc = (Fraction(v) for v in gc)
    R, r = max(rb, rc), min(rb, rc)
    d2 = (xb - xc) ** 2 + (yb - yc) ** 2
    lhs = R + t * r
    return d2 > 0 and lhs * lhs <= t * t * d2


def bin_exact(tk, gb, gc):
    """Least k with the criterion true at tk[k] (len(tk) if none).  In exact
    arithmetic the criterion is monotone in t, so a bisection finds it."""
    lo, hi = 0, len(tk)
    while lo < hi:
        mid = (lo + hi) // 2
        if passes_exact(tk[mid], gb, gc):
            hi = mid
        else:
            lo = mid + 1
    return lo


def brute_relaxed(t, theta, theta_max, p, k0, k1):
    tk = grid(theta, theta_max, k0, k1)
    nbin = k0 + k1
    strong = {0: [0]}  # level 0: the root is strong to itself
    out = []
    for l in range(1, t.levels + 1):
        G = t.level_geom(l)
        cand = {b: [4 * q + k for q in strong[b // 4] for k in range(4)] for b in range(4 ** l)}
        bins = {b: [bin_exact(tk, G[b], G[c]) for c in cs] for b, cs in cand.items()}
        count = [0] * nbin
        for bs in bins.values():
            for k in bs:
                if k < nbin:
                    count[k] += 1
        e = [Fraction(v) ** (p + 1) for v in tk]
        eth = Fraction(theta) ** (p + 1)
        K = k0 - 1
        for k in range(k0, nbin):
            n = sum(count[:k + 1])
            if sum(count[j] * e[j] for j in range(k + 1)) <= eth * n:
                K = k
            else:
                break
        Wl = {b: [c for c, k in zip(cand[b], bins[b]) if k <= K] for b in cand}
        Sl = {b: [c for c, k in zip(cand[b], bins[b]) if k > K] for b in cand}
        out.append((count, K, Wl, Sl))
        strong = Sl
    return out


CASES = [
    ("clustered", lambda: W.clustered_10m(scale=2e-4), 3),
    ("mixed", lambda: W.mixed_1m(scale=1.5e-3), 3),
    ("ring", lambda: W.ring_4m(scale=4e-4), 4),
]


@pytest.mark.parametrize("name,maker,L", CASES)
@pytest.mark.parametrize("theta", [0.35, 0.5, 0.7])
def test_theta_max_equal_theta_is_plain(orc, name, maker, L, theta):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    pl = orc.lists(t, theta)
    for p in (3, 12):
        r = orc.lists_relaxed(t, theta, theta, p)
        for l in range(L + 1):
            assert np.array_equal(r.sptr[l], pl.sptr[l]) and np.array_equal(r.sidx[l], pl.sidx[l])
            assert np.array_equal(r.wptr[l], pl.wptr[l]) and np.array_equal(r.widx[l], pl.widx[l])


@pytest.mark.parametrize("name,maker,L", CASES)
@pytest.mark.parametrize("theta,theta_max,p,k0,k1", [
    (0.5, 0.9, 10, 16, 16), (0.5, 0.75, 4, 8, 4), (0.35, 0.8, 16, 16, 16), (0.7, 0.95, 6, 4, 8)])
def test_relaxed_lists_match_exact_brute_force(orc, name, maker, L, theta, theta_max, p, k0, k1):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    r = orc.lists_relaxed(t, theta, theta_max, p, k0, k1)
    bf = brute_relaxed(t, theta, theta_max, p, k0, k1)
    promoted = 0
    for l in range(1, L + 1):
        count, K, Wl, Sl = bf[l - 1]
        assert r.count[l].tolist() == count
        assert r.kmax[l] == K
        promoted += sum(count[k0:K + 1])
        for b in range(4 ** l):
            assert _rows(r.wptr[l], r.widx[l], b) == Wl[b]
            assert _rows(r.sptr[l], r.sidx[l], b) == Sl[b]
    assert promoted > 0  # the cases do admit pairs above theta


def own_theta(gb, gc):
    """theta_i = R / (d - r), the least theta for which the pair passes."""
    R, r = max(gb[2], gc[2]), min(gb[2], gc[2])
    d = float(np.hypot(gb[0] - gc[0], gb[1] - gc[1]))
    return R / (d - r)


@pytest.mark.parametrize("name,maker,L", CASES)
@pytest.mark.parametrize("theta,theta_max,p", [(0.5, 0.9, 10), (0.35, 0.8, 16), (0.7, 0.95, 4)])
def test_mean_condition_with_own_theta_and_next_bin_breaks_it(orc, name, maker, L, theta, theta_max, p):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    r = orc.lists_relaxed(t, theta, theta_max, p)
    tk = grid(theta, theta_max, r.k0, r.k1)
    for l in range(1, L + 1):
        G = t.level_geom(l)
        vals = [own_theta(G[b], G[c]) ** (p + 1)
                for b in range(4 ** l) for c in _rows(r.wptr[l], r.widx[l], b)]
        if vals:
            assert np.mean(vals) <= theta ** (p + 1) * (1 + 1e-9)
            assert max(own_theta(G[b], G[c]) for b in range(4 ** l)
                       for c in _rows(r.wptr[l], r.widx[l], b)) <= tk[r.kmax[l]] * (1 + 1e-12)
        K = r.kmax[l]
        if K + 1 < r.k0 + r.k1 and r.count[l][K + 1] > 0:
            n = int(r.count[l][:K + 2].sum())
            s = sum(int(r.count[l][j]) * Fraction(tk[j]) ** (p + 1) for j in range(K + 2))
            assert s > Fraction(theta) ** (p + 1) * n


@pytest.mark.parametrize("name,maker,L", CASES)
def test_relaxed_strong_subset_and_exact_cover(orc, name, maker, L):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    pl = orc.lists(t, 0.5)
    r = orc.lists_relaxed(t, 0.5, 0.9, 8)
    for l in range(1, L + 1):
        for b in range(4 ** l):
            assert set(_rows(r.sptr[l], r.sidx[l], b)) <= set(_rows(pl.sptr[l], pl.sidx[l], b))
    assert r.sidx[L].shape[0] < pl.sidx[L].shape[0]
    nleaf = 4 ** L
    cover = np.zeros((nleaf, nleaf), dtype=np.int64)
    for l in range(1, L + 1):
        s = 4 ** (L - l)
        for b in range(4 ** l):
            for c in _rows(r.wptr[l], r.widx[l], b):
                cover[b * s:(b + 1) * s, c * s:(c + 1) * s] += 1
    for b in range(nleaf):
        for c in _rows(r.sptr[L], r.sidx[L], b):
            cover[b, c] += 1
    assert np.all(cover == 1)


@pytest.mark.parametrize("maker", [lambda: W.clustered_10m(scale=4e-4),
                                   lambda: W.ring_4m(scale=1e-3)])
def test_relaxed_fmm_within_model_and_exact_at_high_order(orc, maker):
    ps = maker()
    ex = orc.direct(ps.x, ps.y, ps.q)
    t = orc.tree(ps.x, ps.y, 4)
    for theta in (0.35, 0.5, 0.7):
        for p in (4, 10, 16):
            r = orc.lists_relaxed(t, theta, 0.9, p)
            e, _ = orc.rel_errors(orc.fmm_eval(ps.x, ps.y, ps.q, t, r, p), ex)
            assert e <= 0.1 * theta ** (p + 1) / (1 - theta) ** 2
        # p = 60: the model bound is below rounding for theta <= 1/2
        # (0.4 * 0.5^61 ~ 2e-19), not at 0.7 (4e-10), where the pairs
        # admitted above theta sit close to it
        r = orc.lists_relaxed(t, theta, 0.9, 60)
        e, e2 = orc.rel_errors(orc.fmm_eval(ps.x, ps.y, ps.q, t, r, 60), ex)
        assert e <= max(0.1 * theta ** 61 / (1 - theta) ** 2, 1e-13)
        if theta <= 0.5:
            assert e <= 1e-13 and e2 <= 1e-13


def test_without_mean_condition_the_error_leaves_the_model(orc):
    # every candidate up to theta_max admitted: the lists of theta_max itself
    ps = W.clustered_10m(scale=4e-4)
    ex = orc.direct(ps.x, ps.y, ps.q)
    t = orc.tree(ps.x, ps.y, 4)
    theta, p = 0.5, 16
    e_all, _ = orc.rel_errors(orc.fmm_eval(ps.x, ps.y, ps.q, t, orc.lists(t, 0.9), p), ex)
    e_rel, _ = orc.rel_errors(orc.fmm_eval(ps.x, ps.y, ps.q, t, orc.lists_relaxed(t, theta, 0.9, p), p), ex)
    bound = 0.1 * theta ** (p + 1) / (1 - theta) ** 2
    assert e_rel <= bound < e_all


def test_argument_checks(orc):
    ps = W.ring_4m(scale=1e-4)
    t = orc.tree(ps.x, ps.y, 2)
    for bad in [(0.5, 0.4, 4, 16, 16), (0.5, 1.0, 4, 16, 16), (0.5, 0.9, -1, 16, 16),
                (0.5, 0.9, 4, 0, 16), (0.5, 0.9, 4, 200, 57)]:
        with pytest.raises(ValueError):
            orc.lists_relaxed(t, *bad)
