"""Pins of the selector oracle (oracle/select.py): brute force, closed forms,
invariants, and the a-priori rule against the truncation bound of Section 3."""
import math

import numpy as np
import pytest

from oracle import select as S
from paper_1006_2269_amd import workloads as W


def brute_features(x, y, tol):
    """Point-by-point loops over the definition (small or sampled inputs)."""
    n_all = len(x)
    xs = [float(v) + 0.0 for v in x]
    ys = [float(v) + 0.0 for v in y]
    stride = -(-n_all // 2 ** 18) if n_all > 2 ** 18 else 1

    def cell(v, lo, hi):
        ext = hi - lo
        s = 1024.0 / ext if ext > 0.0 else 0.0
        t = (v - lo) * s
        if not t >= 0.0:
            t = 0.0
        if not t < 1024.0:
            t = 1023.0
        return int(t)

    xl, xh, yl, yh = min(xs), max(xs), min(ys), max(ys)   # box of all points
    fine = [(cell(xs[i], xl, xh), cell(ys[i], yl, yh)) for i in range(0, n_all, stride)]
    n = len(fine)
    out = [math.log10(n_all), math.log10(tol)]
    for l in range(1, 11):
        counts = {}
        for cx, cy in fine:
            key = (cx >> (10 - l), cy >> (10 - l))
            counts[key] = counts.get(key, 0) + 1
        out.append(len(counts) / 4.0 ** l)
        hist = [0] * 8
        for c in counts.values():
            r = c * 4 ** l / n          # exact rational comparison below
            k = sum(1 for j in range(1, 8) if c * 4 ** l * 16 >= n * 2 ** j)
            assert k == sum(1 for e in (1 / 8, 1 / 4, 1 / 2, 1, 2, 4, 8) if r >= e)
            hist[k] += c
        out.extend(h / n for h in hist)
    return np.array(out, dtype=np.float32)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_features_match_brute_force(seed):
    ps = W.random_mixture(400, seed)
    f = S.features(ps.x, ps.y, 1e-6)
    b = brute_features(ps.x, ps.y, 1e-6)
    assert f.shape == (S.NFEAT,)
    np.testing.assert_array_equal(f, b)


@pytest.mark.slow
def test_features_sampled_match_brute_force():
    # above 2^18 points the cells are counted over every ceil(n / 2^18)-th point
    ps = W.random_mixture(300_000, 4)
    assert S.sample_stride(ps.n) == 2
    np.testing.assert_array_equal(S.features(ps.x, ps.y, 1e-5), brute_features(ps.x, ps.y, 1e-5))


def test_features_regular_grid_closed_form():
    # 32 x 32 cell centres: every level-5 cell holds one point, so levels
    # 1..5 are fully occupied at relative density 1 (bin 4); at level 6 a
    # quarter of the cells are occupied at density 4 (bin 6), deeper levels
    # at density >= 16 (bin 7).
    g = (np.arange(32) + 0.5) / 32
    X, Y = np.meshgrid(g, g)
    f = S.features(X.ravel(), Y.ravel(), 1e-3)
    assert f[0] == np.float32(math.log10(1024)) and f[1] == np.float32(-3.0)
    for l in range(1, 11):
        base = 2 + 9 * (l - 1)
        occ, hist = f[base], f[base + 1: base + 9]
        assert occ == np.float32(min(1.0, 1024 / 4 ** l))
        k = 4 if l <= 5 else (6 if l == 6 else 7)
        expect = np.zeros(8, dtype=np.float32)
        expect[k] = 1.0
        np.testing.assert_array_equal(hist, expect)


def test_features_single_cluster_closed_form():
    # all points at one location plus two corners fixing the bounding box:
    # at every level 3 cells are occupied and n - 2 points sit in one cell
    n = 1000
    x = np.full(n, 0.3)
    y = np.full(n, 0.7)
    x[0], y[0], x[1], y[1] = 0.0, 0.0, 1.0, 1.0
    f = S.features(x, y, 1e-6)
    for l in range(1, 11):
        base = 2 + 9 * (l - 1)
        assert f[base] == np.float32(3 / 4 ** l)
        # the corner cells hold 1 point: density 4^l / n
        k1 = sum(1 for j in range(1, 8) if 4 ** l * 16 >= n * 2 ** j)
        kc = sum(1 for j in range(1, 8) if (n - 2) * 4 ** l * 16 >= n * 2 ** j)
        expect = np.zeros(8)
        expect[k1] += 2 / n
        expect[kc] += (n - 2) / n
        np.testing.assert_array_equal(f[base + 1: base + 9], expect.astype(np.float32))


def test_features_invariants():
    ps = W.random_mixture(5000, 7)
    f = S.features(ps.x, ps.y, 1e-5)
    perm = np.random.default_rng(0).permutation(ps.n)
    np.testing.assert_array_equal(f, S.features(ps.x[perm], ps.y[perm], 1e-5))
    for l in range(1, 11):
        base = 2 + 9 * (l - 1)
        assert abs(float(f[base + 1: base + 9].astype(np.float64).sum()) - 1.0) < 1e-6
        if l > 1:
            assert f[base] <= f[base - 9] + 1e-7   # finer grid: smaller occupied fraction
    # degenerate extent: every point in cell 0 at every level
    g = S.features(np.zeros(50), np.zeros(50), 1e-5)
    for l in range(1, 11):
        base = 2 + 9 * (l - 1)
        assert g[base] == np.float32(1 / 4 ** l)
        # the one cell has relative density 4^l: bin 6 (4 >= 4) at level 1, 7 beyond
        assert g[base + 1 + (6 if l == 1 else 7)] == 1.0


@pytest.mark.parametrize("n,tol", [(10 ** 6, 1e-6), (20000, 1e-3), (4 ** 7 * 20, 1e-9), (300, 0.5)])
def test_rule_meets_bound(n, tol):
    L, p, theta = S.rule(n, tol)
    assert theta == 0.5
    bound = lambda q: 0.1 * theta ** (q + 1) / (1 - theta) ** 2
    assert bound(p) <= tol and (p == 1 or bound(p - 1) > tol)
    assert 1 <= L <= S.levels_max(n) and 4 ** L <= n
    assert abs(L - math.log(max(n / 20, 1), 4)) <= 0.5 or L in (1, S.levels_max(n))


def test_rule_values():
    assert S.rule(10 ** 6, 1e-6) == (8, 18, 0.5)
    # n / 20 = 4^7 exactly: log4 is 7, no rounding question
    assert S.rule(20 * 4 ** 7, 1e-6)[0] == 7
    # half-way case log4(n / 20) = 0.5 rounds up
    assert S.rule(40, 1e-3)[0] == 1


def _blob(mean3, std3, rng=(3.0, 7.0, -9.0, -3.0)):
    b = np.zeros(S.HEADER + 10, dtype=np.float32)
    b[2 * S.NFEAT: 2 * S.NFEAT + 3] = mean3
    b[2 * S.NFEAT + 3: 2 * S.NFEAT + 6] = std3
    b[2 * S.NFEAT + 6: 2 * S.NFEAT + 10] = rng
    return b


def test_decide_decoding():
    b = _blob((1.0, -1.3, 0.52), (1.0, 1.0, 1.0))
    # log4(1e6 / 16) = 7.966, + 1 -> levels 9 (= floor(log4 1e6)); theta
    # 0.52 -> 0.55; p = ceil((-6 - log10 2 + 1.3) / log10 0.55) - 1
    #                 = ceil(19.26) - 1 = 19
    assert S.decide(np.zeros(3), b, 10 ** 6, 1e-6) == (9, 19, 0.55, True)
    # the model's error at p is <= tol / 2, one order less is not
    C, th = 10 ** -1.3, 0.55
    assert C * th ** 20 <= 1e-6 / 2 < C * th ** 19
    b2 = _blob((0.0, -2.0, 0.5), (2.0, 4.0, 0.1))
    # outputs (-1, 0.25, -1.2): dl = -2 (7.966 - 2 -> 6), log10 C = -1, theta 0.38 -> 0.35;
    # p = ceil((-5 - log10 2) / log10 0.35) - 1 = ceil(11.63) - 1 = 11
    assert S.decide(np.array([-1.0, 0.25, -1.2]), b2, 10 ** 6, 1e-6) == (6, 11, 0.35, True)
    assert 0.1 * 0.35 ** 12 <= 1e-6 / 2 < 0.1 * 0.35 ** 11
    # the offset is from log4(N / 16) itself, not from its rounding: at
    # N = 4e5, log4(25000) = 7.305, so dl = 0.3 gives 7.605 -> 8 levels and
    # dl = 0.15 gives 7.455 -> 7
    b3 = _blob((0.0, -1.3, 0.55), (1.0, 1.0, 1.0))
    assert S.decide(np.array([0.3, 0.0, 0.0]), b3, 400000, 1e-6)[0] == 8
    assert S.decide(np.array([0.15, 0.0, 0.0]), b3, 400000, 1e-6)[0] == 7
    # outside the trained range -> the rule
    assert S.decide(np.zeros(3), b, 10 ** 8, 1e-6)[3] is False
    assert S.decide(np.zeros(3), b, 10 ** 6, 1e-10)[:3] == S.rule(10 ** 6, 1e-10)
    assert S.decide(np.array([np.nan, 0, 0]), b, 10 ** 6, 1e-6)[3] is False
