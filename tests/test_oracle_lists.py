"""Pins of the oracle's strong/weak connectivity (Section 4) under the
theta-criterion (Criterion 2.1).

* The criterion itself is re-decided in exact rational arithmetic.
* The recursive rule is checked against its closed (non-recursive) meaning: c
  is strongly coupled to b at level l iff no pair of ancestors of (b, c) at
  levels 1..l is well separated; c is weakly coupled iff (b, c) is well
  separated while no pair of their ancestors at levels 1..l-1 is.
* Symmetry, self-coupling, exact cover of all sources, the separation
  inequalities (2.2), and the 13/39 stencil of a regular grid.
"""
from fractions import Fraction

import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


def separated_exact(theta, gb, gc):
    """R + theta r <= theta d for disjoint balls, decided exactly on the
    binary64 inputs."""
    t = Fraction(theta)
    rb, rc = Fraction(gb[2]), Fraction(gc[2])
    R, r = max(rb, rc), min(rb, rc)
    dx = Fraction(gb[0]) - Fraction(gc[0])
    dy = Fraction(gb[1]) - Fraction(gc[1])
    lhs = R + t * r
    d2 = dx * dx + dy * dy
    return lhs * lhs <= t * t * d2 and d2 > 0


def test_criterion_boundary_cases(orc):
    # two unit balls at distance d: separated iff 1 + theta <= theta d
    th = 0.5
    assert orc.theta_test(th, [0.0, 0.0, 1.0], [3.0, 0.0, 1.0])          # equality
    assert not orc.theta_test(th, [0.0, 0.0, 1.0], [2.9999999, 0.0, 1.0])
    # unequal radii: R = 2, r = 1, theta = 0.5: need d >= 5
    assert orc.theta_test(th, [0.0, 0.0, 2.0], [3.0, 4.0, 1.0])
    assert orc.theta_test(th, [3.0, 4.0, 1.0], [0.0, 0.0, 2.0])          # symmetric
    assert not orc.theta_test(th, [0.0, 0.0, 2.0], [3.0, 3.99, 1.0])
    # two zero-size balls at one point are not disjoint: never separated;
    # at distinct points they are
    assert not orc.theta_test(th, [0.5, 0.5, 0.0], [0.5, 0.5, 0.0])
    assert orc.theta_test(th, [0.5, 0.5, 0.0], [0.5, 0.5000001, 0.0])
    # a smaller theta is stricter
    assert not orc.theta_test(0.25, [0.0, 0.0, 2.0], [3.0, 4.0, 1.0])
    g = np.random.Generator(np.random.PCG64(3))
    for _ in range(2000):
        a = [g.normal(), g.normal(), abs(g.normal()) * 0.3]
        b = [g.normal(), g.normal(), abs(g.normal()) * 0.3]
        th = float(g.uniform(0.05, 0.95))
        assert orc.theta_test(th, a, b) == separated_exact(th, a, b)


def ancestor(b, l_from, l_to):
    return b >> (2 * (l_from - l_to))


@pytest.mark.parametrize("n,L,theta,seed", [(300, 3, 0.5, 1), (700, 3, 0.35, 2), (1100, 4, 0.7, 3)])
def test_lists_match_ancestor_definition(orc, n, L, theta, seed):
    ps = W.random_mixture(n, seed=seed)
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists(t, theta)
    sep = {}
    for l in range(1, L + 1):
        G = t.level_geom(l)
        nb = 4 ** l
        sep[l] = np.array([[separated_exact(theta, G[b], G[c]) for c in range(nb)] for b in range(nb)])
    for l in range(1, L + 1):
        nb = 4 ** l
        for b in range(nb):
            strong_anc = [c for c in range(nb)
                          if not any(sep[m][ancestor(b, l, m), ancestor(c, l, m)] for m in range(1, l))]
            want_s = [c for c in strong_anc if not sep[l][b, c]]
            want_w = [c for c in strong_anc if sep[l][b, c]]
            got_s = ls.sidx[l][ls.sptr[l][b]:ls.sptr[l][b + 1]].tolist()
            got_w = ls.widx[l][ls.wptr[l][b]:ls.wptr[l][b + 1]].tolist()
            assert got_s == want_s
            assert got_w == want_w


@pytest.mark.parametrize("maker,L,theta", [(lambda: W.uniform(5000, 4), 5, 0.5),
                                           (lambda: W.clustered_10m(scale=4e-4), 5, 0.5),
                                           (lambda: W.ring_4m(scale=1e-3), 5, 0.3),
                                           (lambda: W.random_mixture(3000, 9), 4, 0.75)])
def test_list_invariants(orc, maker, L, theta):
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists(t, theta)
    cover = np.zeros((4 ** L, 4 ** L), dtype=np.int64)
    for l in range(1, L + 1):
        nb = 4 ** l
        G = t.level_geom(l)
        S = [set(ls.sidx[l][ls.sptr[l][b]:ls.sptr[l][b + 1]].tolist()) for b in range(nb)]
        Wl = [set(ls.widx[l][ls.wptr[l][b]:ls.wptr[l][b + 1]].tolist()) for b in range(nb)]
        for b in range(nb):
            assert b in S[b]
            assert not (S[b] & Wl[b])
            for c in S[b]:
                assert b in S[c]
            for c in Wl[b]:
                assert b in Wl[c]
                # (2.2): r/(d-R) <= R/(d-r) <= theta on every accepted pair
                d = np.hypot(G[b, 0] - G[c, 0], G[b, 1] - G[c, 1])
                R, r = max(G[b, 2], G[c, 2]), min(G[b, 2], G[c, 2])
                assert r / (d - R) <= R / (d - r) * (1 + 1e-12)
                assert R / (d - r) <= theta * (1 + 1e-12)
                # exact cover bookkeeping at leaf granularity
                span = 4 ** (L - l)
                cover[b * span:(b + 1) * span, c * span:(c + 1) * span] += 1
        if l == L:
            for b in range(nb):
                for c in S[b]:
                    cover[b, c] += 1
    assert np.all(cover == 1)


def test_grid_stencil_13_39(orc):
    L, theta = 5, 0.5
    ps = W.grid(L)
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists(t, theta)
    k = 2 ** L

    def coords(b):
        ix = iy = 0
        for lev in range(L):
            digit = (b >> (2 * (L - 1 - lev))) & 3
            ix = 2 * ix + (digit >> 1)
            iy = 2 * iy + (digit & 1)
        return ix, iy

    strong_offsets = {(0, 0), (1, 0), (-1, 0), (0, 1), (0, -1), (1, 1), (1, -1), (-1, 1), (-1, -1),
                      (2, 0), (-2, 0), (0, 2), (0, -2)}
    checked = 0
    for b in range(4 ** L):
        ix, iy = coords(b)
        if min(ix, iy, k - 1 - ix, k - 1 - iy) < 6:
            continue
        S = ls.sidx[L][ls.sptr[L][b]:ls.sptr[L][b + 1]]
        Wl = ls.widx[L][ls.wptr[L][b]:ls.wptr[L][b + 1]]
        offs = {(coords(c)[0] - ix, coords(c)[1] - iy) for c in S.tolist()}
        assert offs == strong_offsets
        assert len(Wl) == 39
        checked += 1
    assert checked == (k - 12) ** 2
