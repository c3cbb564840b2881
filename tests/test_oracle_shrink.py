"""Pins of the shrink-to-points geometry: the ball of each box of Criterion
2.1 drawn around its points (their bounding box) instead of its tiling
rectangle.

* Each box's bounding box equals a point-by-point loop over its members, every
  point lies in its box's ball, each ball is no larger than the tiling
  rectangle's, and parents' boxes contain their children's.
* Regular grid: the interior boxes' balls and the interior leaves' strong and
  weak list sizes follow an exact rational enumeration of the recursive rule
  on the stencil (ancestors at every level with their own point spans).
* The FMM on the shrunk geometry stays within the a-priori error model and
  reaches the direct sum to rounding at high order, plain and with the
  structural options.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


@pytest.mark.parametrize("maker,L", [(lambda: W.clustered_10m(scale=3e-4), 4),
                                     (lambda: W.random_mixture(1500, 3), 3),
                                     (lambda: W.uniform(700, 4), 2)])
def test_point_boxes_and_balls(orc, maker, L):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ts = orc.shrink(t, ps.x, ps.y)
    pr = orc.point_rects(t, ps.x, ps.y)
    for l in range(L + 1):
        span = 4 ** (L - l)
        for b in range(4 ** l):
            members = t.perm[t.leaf_start[b * span]:t.leaf_start[(b + 1) * span]]
            lo_x = hi_x = ps.x[members[0]]
            lo_y = hi_y = ps.y[members[0]]
            for j in members[1:]:
                lo_x, hi_x = min(lo_x, ps.x[j]), max(hi_x, ps.x[j])
                lo_y, hi_y = min(lo_y, ps.y[j]), max(hi_y, ps.y[j])
            g = orc.level_offset(l) + b
            assert tuple(pr[g]) == (lo_x, hi_x, lo_y, hi_y)
            cx, cy, r = ts.geom[g]
            d = np.hypot(ps.x[members] - cx, ps.y[members] - cy)
            # the centre is rounded at the scale of the coordinates, not of the box
            assert d.max() <= r + 4 * np.finfo(float).eps * max(abs(cx), abs(cy), r)
            assert r <= t.geom[g, 2] * (1 + 1e-15)
            if l < L:
                kids = pr[orc.level_offset(l + 1) + 4 * b: orc.level_offset(l + 1) + 4 * b + 4]
                assert pr[g, 0] == kids[:, 0].min() and pr[g, 1] == kids[:, 1].max()
                assert pr[g, 2] == kids[:, 2].min() and pr[g, 3] == kids[:, 3].max()


def test_grid_stencil_exact(orc):
    L, theta = 5, Fraction(1, 2)
    ps = W.grid(L)             # 2 x 2 points per leaf at the cell centres of a 64 x 64 grid
    t = orc.tree(ps.x, ps.y, L)
    ts = orc.shrink(t, ps.x, ps.y)
    ls = orc.lists(ts, 0.5)
    k = 2 ** L

    def coords(b, lv):
        ix = iy = 0
        for lev in range(lv):
            digit = (b >> (2 * (lv - 1 - lev))) & 3
            ix = 2 * ix + (digit >> 1)
            iy = 2 * iy + (digit & 1)
        return ix, iy

    # in units of the leaf side h: the grid spacing is h/2, a box of level m
    # has side s_m = 2^(L-m) and its points span (2^(L-m+1) - 1) h/2 per
    # axis, so its ball has radius r_m = span sqrt(2)/2; interior boxes keep
    # the tiling centres
    def sep(m, off):  # ancestors at level m with offset `off` (in boxes of that level)
        s = Fraction(2 ** (L - m))
        span = Fraction(2 ** (L - m + 1) - 1, 2)
        d2 = (off[0] ** 2 + off[1] ** 2) * s * s
        # (R + theta r)^2 <= theta^2 d^2 with R = r = span sqrt(2) / 2
        return (1 + theta) ** 2 * span * span / 2 <= theta * theta * d2 and d2 > 0

    def expected(ix, iy):
        ns = nw = 0
        for dx in range(-8, 9):
            for dy in range(-8, 9):
                cx, cy = ix + dx, iy + dy
                anc = [((cx >> (L - m)) - (ix >> (L - m)), (cy >> (L - m)) - (iy >> (L - m))) for m in range(1, L + 1)]
                if any(sep(m, anc[m - 1]) for m in range(1, L)):
                    continue
                if sep(L, anc[L - 1]):
                    nw += 1
                else:
                    ns += 1
        return ns, nw

    # interior leaves: their ball is half the tiling one (exact)
    checked = 0
    for b in range(4 ** L):
        ix, iy = coords(b, L)
        if min(ix, iy, k - 1 - ix, k - 1 - iy) < 8:
            continue
        g = orc.level_offset(L) + b
        assert ts.geom[g, 2] == t.geom[g, 2] / 2
        ns, nw = expected(ix, iy)
        assert ls.sptr[L][b + 1] - ls.sptr[L][b] == ns
        assert ls.wptr[L][b + 1] - ls.wptr[L][b] == nw
        checked += 1
    assert checked == (k - 16) ** 2


@pytest.mark.parametrize("opt", [False, True])
def test_fmm_on_shrunk_geometry(orc, opt):
    ps = W.clustered_10m(scale=4e-4)
    ex = orc.direct(ps.x, ps.y, ps.q)
    ts = orc.shrink(orc.tree(ps.x, ps.y, 4), ps.x, ps.y)
    for theta in (0.35, 0.5, 0.7):
        if opt:
            ls = orc.lists_opt(ts, theta, parent=True, swap_levels=range(1, 5))
            ev = lambda p: orc.fmm_eval_opt(ps.x, ps.y, ps.q, ts, ls, p)
        else:
            ls = orc.lists(ts, theta)
            ev = lambda p: orc.fmm_eval(ps.x, ps.y, ps.q, ts, ls, p)
        for p in (4, 10, 16):
            e, _ = orc.rel_errors(ev(p), ex)
            assert e <= max(0.1 * theta ** (p + 1) / (1 - theta) ** 2, 1e-14)
        e, e2 = orc.rel_errors(ev(60), ex)
        assert e <= 1e-13 and e2 <= 1e-13
