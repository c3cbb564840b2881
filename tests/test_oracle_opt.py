"""Pins of the oracle's structural optimisations (Section 4): interaction via
the parent box, and exchanged roles (P2L / M2P) for strongly coupled boxes of
very different radii.

* Every entry of the optimised lists is re-decided in exact rational
  arithmetic on the binary64 geometry: V entries (via the parent) pass the
  criterion against the parent and all four of its children; X entries fail
  the criterion but pass it with the radii exchanged, on disjoint balls; W
  and S entries are what is left of each candidate group.
* Exact cover: every (target leaf, source leaf) pair is served exactly once
  by W, V, X at some level or by the finest S.
* With the exchange at the finest level only, the optimised lists are a
  regrouping of the plain ones (S = S' + X, W = W' + children of V).
* Regular grid: exchanged pairs only with a box on the root border (the
  interior boxes are congruent squares), and the number of
  parent interactions of an interior box equals an exact enumeration of the
  stencil.
* P2L: the local expansion of far sources obeys the logarithm's tail bound.
* The FMM with the optimised lists stays within the a-priori model and
  reproduces the direct sum to rounding at p = 60.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


def _exact(g):
    return Fraction(g[0]), Fraction(g[1]), Fraction(g[2])


def separated_exact(theta, gb, gc):
    t = Fraction(theta)
    xb, yb, rb = _exact(gb)
    xc, yc, rc = _exact(gc)
    R, r = max(rb, rc), min(rb, rc)
    d2 = (xb - xc) ** 2 + (yb - yc) ** 2
    lhs = R + t * r
    return lhs * lhs <= t * t * d2 and d2 > 0


def exchanged_exact(theta, gb, gc):
    """r + theta R <= theta d with the balls disjoint (d > R + r)."""
    t = Fraction(theta)
    xb, yb, rb = _exact(gb)
    xc, yc, rc = _exact(gc)
    R, r = max(rb, rc), min(rb, rc)
    d2 = (xb - xc) ** 2 + (yb - yc) ** 2
    lhs = r + t * R
    return lhs * lhs <= t * t * d2 and d2 > (R + r) ** 2


def _rows(ptr, idx, b):
    return idx[ptr[b]:ptr[b + 1]].tolist()


CASES = [
    ("clustered", lambda: W.clustered_10m(scale=3e-4), 4, 0.5),
    ("mixed", lambda: W.mixed_1m(scale=3e-3), 4, 0.5),
    ("mixture", lambda: W.random_mixture(2500, 11), 4, 0.35),
    ("ring", lambda: W.ring_4m(scale=6e-4), 4, 0.7),
]
FLAGS = [(True, "finest"), (False, "finest"), (True, "all"), (False, "all"), (True, "none")]


def _opt(orc, t, theta, parent, swap):
    levels = {"finest": (t.levels,), "all": tuple(range(1, t.levels + 1)), "none": ()}[swap]
    return orc.lists_opt(t, theta, parent=parent, swap_levels=levels)


@pytest.mark.parametrize("name,maker,L,theta", CASES)
@pytest.mark.parametrize("parent,swap", FLAGS)
def test_opt_lists_decided_exactly(orc, name, maker, L, theta, parent, swap):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ls = _opt(orc, t, theta, parent, swap)
    for l in range(1, L + 1):
        G, Gp = t.level_geom(l), t.level_geom(l - 1)
        on = l in ls.swap_levels
        for b in range(4 ** l):
            cand = [4 * q + k for q in _rows(ls.sptr[l - 1], ls.sidx[l - 1], b // 4) for k in range(4)]
            S = _rows(ls.sptr[l], ls.sidx[l], b)
            Wl = _rows(ls.wptr[l], ls.widx[l], b)
            V = _rows(ls.vptr[l], ls.vidx[l], b)
            X = _rows(ls.xptr[l], ls.xidx[l], b)
            assert S == sorted(S) and Wl == sorted(Wl) and V == sorted(V) and X == sorted(X)
            # every candidate lands in exactly one list (V takes a whole group)
            served = S + Wl + X + [4 * q + k for q in V for k in range(4)]
            assert sorted(served) == cand
            for q in V:
                assert parent
                assert separated_exact(theta, G[b], Gp[q])
                assert all(separated_exact(theta, G[b], G[4 * q + k]) for k in range(4))
            for c in Wl:
                assert separated_exact(theta, G[b], G[c])
                q = c // 4
                grouped = all(separated_exact(theta, G[b], G[4 * q + k]) for k in range(4)) and \
                    separated_exact(theta, G[b], Gp[q])
                assert not (parent and grouped)
            for c in X:
                assert on and not separated_exact(theta, G[b], G[c]) and exchanged_exact(theta, G[b], G[c])
            for c in S:
                assert not separated_exact(theta, G[b], G[c])
                assert not (on and exchanged_exact(theta, G[b], G[c]))


@pytest.mark.parametrize("name,maker,L,theta", CASES)
@pytest.mark.parametrize("parent,swap", FLAGS)
def test_opt_lists_exact_cover(orc, name, maker, L, theta, parent, swap):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ls = _opt(orc, t, theta, parent, swap)
    nleaf = 4 ** L
    cover = np.zeros((nleaf, nleaf), dtype=np.int64)

    def add(l_t, b, l_s, c):
        st, ss = 4 ** (L - l_t), 4 ** (L - l_s)
        cover[b * st:(b + 1) * st, c * ss:(c + 1) * ss] += 1

    for l in range(1, L + 1):
        for b in range(4 ** l):
            for c in _rows(ls.wptr[l], ls.widx[l], b):
                add(l, b, l, c)
            for q in _rows(ls.vptr[l], ls.vidx[l], b):
                add(l, b, l - 1, q)
            for c in _rows(ls.xptr[l], ls.xidx[l], b):
                add(l, b, l, c)
    for b in range(nleaf):
        for c in _rows(ls.sptr[L], ls.sidx[L], b):
            add(L, b, L, c)
    assert np.all(cover == 1)


@pytest.mark.parametrize("name,maker,L,theta", CASES)
def test_finest_exchange_regroups_plain_lists(orc, name, maker, L, theta):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    plain = orc.lists(t, theta)
    ls = orc.lists_opt(t, theta, parent=True, swap_levels=(L,))
    for l in range(1, L + 1):
        for b in range(4 ** l):
            S = _rows(ls.sptr[l], ls.sidx[l], b)
            X = _rows(ls.xptr[l], ls.xidx[l], b)
            Wl = _rows(ls.wptr[l], ls.widx[l], b)
            V = _rows(ls.vptr[l], ls.vidx[l], b)
            assert sorted(S + X) == _rows(plain.sptr[l], plain.sidx[l], b)
            assert sorted(Wl + [4 * q + k for q in V for k in range(4)]) == _rows(plain.wptr[l], plain.widx[l], b)
            if l < L:
                assert not X


def test_grid_no_exchange_and_parent_count(orc):
    L, theta = 5, 0.5
    ps = W.grid(L)
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists_opt(t, theta, parent=True, swap_levels=range(1, L + 1))
    # exact enumeration on the stencil, in units of the leaf side h: leaf
    # centre (i + 1/2, j + 1/2), radius sqrt(2)/2; parent-level box (I, J)
    # centre (2I + 1, 2J + 1), radius sqrt(2).  Radii are multiples of
    # sqrt(2), so the squared criterion is rational.
    th = Fraction(1, 2)

    def sep(c1, r1sq2, c2, r2sq2):  # radii given as multiples of sqrt(2)
        R, r = max(r1sq2, r2sq2), min(r1sq2, r2sq2)
        d2 = (c1[0] - c2[0]) ** 2 + (c1[1] - c2[1]) ** 2
        return 2 * (R + th * r) ** 2 <= th * th * d2 and d2 > 0

    def expected(i, j):
        P = (i // 2, j // 2)
        half = Fraction(1, 2)
        cb = (i + half, j + half)
        nv = nw = 0
        for dI in range(-3, 4):
            for dJ in range(-3, 4):
                Q = (P[0] + dI, P[1] + dJ)
                # strong at the parent level: congruent boxes of side 2h
                cP, cQ = (2 * P[0] + 1, 2 * P[1] + 1), (2 * Q[0] + 1, 2 * Q[1] + 1)
                if sep(cP, 1, cQ, 1):
                    continue
                kids = [(2 * Q[0] + a + half, 2 * Q[1] + bb + half) for a in (0, 1) for bb in (0, 1)]
                weak = [sep(cb, half, ck, half) for ck in kids]
                if all(weak) and sep(cb, half, cQ, 1):
                    nv += 1
                else:
                    nw += sum(weak)
        return nv, nw

    k = 2 ** L

    def coords(b, lv=L):
        ix = iy = 0
        for lev in range(lv):
            digit = (b >> (2 * (lv - 1 - lev))) & 3
            ix = 2 * ix + (digit >> 1)
            iy = 2 * iy + (digit & 1)
        return ix, iy

    # interior boxes are congruent squares, where the exchanged criterion is
    # the plain one: exchanged pairs occur only with a box on the root border
    # (narrower by half a grid step, the root being the tight bounding box)
    for lv in range(1, L + 1):
        kl = 2 ** lv
        on_border = lambda a: min(a[0], a[1], kl - 1 - a[0], kl - 1 - a[1]) == 0
        for b in range(4 ** lv):
            for c in _rows(ls.xptr[lv], ls.xidx[lv], b):
                assert on_border(coords(b, lv)) or on_border(coords(c, lv))

    checked = 0
    for b in range(4 ** L):
        ix, iy = coords(b)
        if min(ix, iy, k - 1 - ix, k - 1 - iy) < 6:
            continue
        nv, nw = expected(ix, iy)
        assert len(_rows(ls.vptr[L], ls.vidx[L], b)) == nv
        assert len(_rows(ls.wptr[L], ls.widx[L], b)) == nw
        assert nw + 4 * nv == 39
        checked += 1
    assert checked == (k - 12) ** 2
    assert expected(10, 10)[0] > 0  # the grouping does occur on the grid


@pytest.mark.parametrize("ratio", [2.0, 3.0, 6.0])
def test_p2l_tail_bound(orc, ratio):
    g = np.random.Generator(np.random.PCG64(12))
    c, s = (0.3, -0.2), 0.4
    # sources on and outside the circle of radius ratio * s, targets inside s
    rad = ratio * s * (1 + g.random(60))
    ang = g.uniform(0, 2 * np.pi, 60)
    xs, ys = c[0] + rad * np.cos(ang), c[1] + rad * np.sin(ang)
    q = g.uniform(-1, 1, 60)
    rt = s * np.sqrt(g.random(30))
    at = g.uniform(0, 2 * np.pi, 30)
    xt, yt = c[0] + rt * np.cos(at), c[1] + rt * np.sin(at)
    ex = np.array([np.sum(q * np.log(np.hypot(xt[i] - xs, yt[i] - ys))) for i in range(30)])
    for p in (1, 4, 9, 18, 30):
        B = orc.p2l(xs, ys, q, c, s, p)
        err = np.abs(orc.l2p(B, c, s, xt, yt) - ex).max()
        bound = np.abs(q).sum() * ratio ** -(p + 1) / ((p + 1) * (1 - 1 / ratio))
        assert err <= bound * (1 + 1e-9) + 1e-14


@pytest.mark.parametrize("parent,swap", [(True, "finest"), (True, "all"), (False, "all")])
def test_opt_fmm_within_bound_and_exact_at_high_order(orc, parent, swap):
    ps = W.clustered_10m(scale=4e-4)
    ex = orc.direct(ps.x, ps.y, ps.q)
    t = orc.tree(ps.x, ps.y, 4)
    for theta in (0.35, 0.5, 0.7):
        ls = _opt(orc, t, theta, parent, swap)
        for p in (4, 10, 16):
            e, _ = orc.rel_errors(orc.fmm_eval_opt(ps.x, ps.y, ps.q, t, ls, p), ex)
            assert e <= max(0.1 * theta ** (p + 1) / (1 - theta) ** 2, 1e-14)
        # truncation theta^(p+1) below rounding: p = 60 (0.7^61 ~ 4e-10 x 0.1 / 0.09)
        e, e2 = orc.rel_errors(orc.fmm_eval_opt(ps.x, ps.y, ps.q, t, ls, 60), ex)
        assert e <= 1e-13 and e2 <= 1e-13
