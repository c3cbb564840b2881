"""Pins of the oracle's uniform quadtree (the non-adaptive subdivision that
Section 5's second experiment compares the asymmetric adaptive tree with).

* Uniformity and tiling: the four children of a box are its four quarters
  (equal halves in each coordinate, up to one rounding of the midpoint), so
  every box of a level has the root's width and height over 2^l.
* Every point lies in exactly one leaf rectangle (half-open, closed on the
  root's upper edges), found by brute force over all leaves, and that leaf
  is the one the tree lists it in; the listing is a permutation, by (x,
  index) inside each leaf.
* On a regular grid of 2^L x 2^L cell centres: one point per leaf, and the
  same leaves and listing as the median tree (whose deeper split lines lie
  between points, not on the rectangles' midpoints).
* Degenerate sets: one point, all points at one location.
* The FMM on the uniform tree (empty leaves, leaves of hundreds of points)
  keeps the a-priori model's bound and reaches the direct sum to rounding
  at high order.
"""
import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


def _leaf_of_points(t):
    leaf = np.empty(t.n, dtype=np.int64)
    for b in range(4 ** t.levels):
        leaf[t.perm[t.leaf_start[b]:t.leaf_start[b + 1]]] = b
    return leaf


MAKERS = {
    "clustered": (lambda: W.clustered_10m(scale=2e-4), 4),
    "normal": (lambda: W.normal_corner(3000, 5, sigma=0.05), 4),
    "layer": (lambda: W.layer(3000, 6, sigma=0.02), 3),
    "uniform": (lambda: W.uniform(2000, 9), 3),
}


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_boxes_are_quarters_and_congruent(orc, name):
    maker, L = MAKERS[name]
    ps = maker()
    t = orc.tree_midpoint(ps.x, ps.y, L)
    root = t.rects[0]
    W0, H0 = root[1] - root[0], root[3] - root[2]
    for l in range(L):
        R, C = t.level_rects(l), t.level_rects(l + 1)
        for b in range(4 ** l):
            xlo, xhi, ylo, yhi = R[b]
            ch = C[4 * b:4 * b + 4]
            # the x split is shared by children (0, 1) | (2, 3), the y split by (0, 2) | (1, 3)
            mx, my = ch[0][1], ch[0][3]
            assert ch[1][1] == mx and ch[2][0] == mx and ch[3][0] == mx
            assert ch[2][3] == my and ch[1][2] == my and ch[3][2] == my
            assert tuple(ch[0][[0, 2]]) == (xlo, ylo) and tuple(ch[3][[1, 3]]) == (xhi, yhi)
            assert abs((mx - xlo) - (xhi - mx)) <= 2 * np.spacing(max(abs(xlo), abs(xhi), 1e-300))
            assert abs((my - ylo) - (yhi - my)) <= 2 * np.spacing(max(abs(ylo), abs(yhi), 1e-300))
        w = C[:, 1] - C[:, 0]
        h = C[:, 3] - C[:, 2]
        assert np.allclose(w, W0 / 2 ** (l + 1), rtol=0, atol=8 * np.spacing(W0))
        assert np.allclose(h, H0 / 2 ** (l + 1), rtol=0, atol=8 * np.spacing(H0))


@pytest.mark.parametrize("name", sorted(MAKERS))
def test_points_in_their_leaf_by_brute_force(orc, name):
    maker, L = MAKERS[name]
    ps = maker()
    t = orc.tree_midpoint(ps.x, ps.y, L)
    assert sorted(t.perm.tolist()) == list(range(ps.n))
    assert t.leaf_start[0] == 0 and t.leaf_start[-1] == ps.n and np.all(np.diff(t.leaf_start) >= 0)
    R = t.level_rects(L)
    root = t.rects[0]
    x, y = ps.x[:, None], ps.y[:, None]
    inx = (R[None, :, 0] <= x) & ((x < R[None, :, 1]) | ((R[None, :, 1] == root[1]) & (x == root[1])))
    iny = (R[None, :, 2] <= y) & ((y < R[None, :, 3]) | ((R[None, :, 3] == root[3]) & (y == root[3])))
    inside = inx & iny
    assert np.all(inside.sum(axis=1) == 1)  # exactly one leaf holds each point
    assert np.array_equal(np.argmax(inside, axis=1), _leaf_of_points(t))
    for b in range(4 ** L):
        idx = t.perm[t.leaf_start[b]:t.leaf_start[b + 1]]
        keys = list(zip(ps.x[idx].tolist(), idx.tolist()))
        assert keys == sorted(keys)


@pytest.mark.parametrize("L", [2, 3, 4])
def test_regular_grid_equals_median_tree(orc, L):
    ps = W.grid(L, per_axis_factor=1)
    t = orc.tree_midpoint(ps.x, ps.y, L)
    m = orc.tree(ps.x, ps.y, L)
    assert np.all(np.diff(t.leaf_start) == 1)
    assert np.array_equal(t.leaf_start, m.leaf_start) and np.array_equal(t.perm, m.perm)
    # the first split lines agree (both at the root's midpoint); deeper ones
    # differ: the median tree's lie between the straddling points
    assert np.array_equal(t.rects[:5], m.rects[:5])


def test_degenerate_sets(orc):
    t = orc.tree_midpoint(np.array([0.3]), np.array([0.7]), 2)
    assert t.leaf_start[-1] == 1 and np.count_nonzero(np.diff(t.leaf_start)) == 1
    n = 50
    x, y = np.full(n, 0.25), np.full(n, -0.5)
    q = np.linspace(-1, 1, n)
    t = orc.tree_midpoint(x, y, 3)
    # a zero-size root: every split line is the point itself, which goes high
    assert t.leaf_start[-2] == 0 and t.leaf_start[-1] == n
    phi = orc.fmm_eval(x, y, q, t, orc.lists(t, 0.5), 6)
    assert np.all(phi == 0.0)  # coincident points do not interact


@pytest.mark.parametrize("name", ["clustered", "normal", "layer"])
def test_fmm_on_uniform_tree_within_model(orc, name):
    maker, L = MAKERS[name]
    ps = maker()
    t = orc.tree_midpoint(ps.x, ps.y, L)
    sizes = np.diff(t.leaf_start)
    assert sizes.max() > 2 * ps.n / 4 ** L  # unbalanced leaves
    ex = orc.direct(ps.x, ps.y, ps.q)
    for theta in (0.35, 0.5, 0.7):
        ls = orc.lists(t, theta)
        for p in (4, 10, 16):
            e, _ = orc.rel_errors(orc.fmm_eval(ps.x, ps.y, ps.q, t, ls, p), ex)
            assert e <= 0.1 * theta ** (p + 1) / (1 - theta) ** 2
    e, e2 = orc.rel_errors(orc.fmm_eval(ps.x, ps.y, ps.q, t, orc.lists(t, 0.5), 50), ex)
    assert e <= 1e-13 and e2 <= 1e-13
