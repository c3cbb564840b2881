"""Pins of the oracle's balanced median-split pyramid (Section 4, Fig. 1.1).

The brute force here decides membership by counting (a point goes low when
fewer than floor(n/2) box members precede it in (coordinate, index) order),
which is a different algorithm from the oracle's sorting.  The grid layout has
closed-form split lines."""
import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


def brute_tree(x, y, L):
    """Returns leaf member lists (in (x, index) order) and rects per level."""
    n = x.shape[0]
    boxes = [np.arange(n)]
    rects = [[(x.min(), x.max(), y.min(), y.max())]]
    for _ in range(L):
        nb, nr = [], []
        for b, mem in enumerate(boxes):
            R = rects[-1][b]
            m = mem.shape[0]
            # rank of each member by (x, index), by counting
            rx = np.array([np.sum((x[mem] < x[i]) | ((x[mem] == x[i]) & (mem < i))) for i in mem])
            lo, hi = mem[rx < m // 2], mem[rx >= m // 2]
            sx = 0.5 * (x[lo].max() + x[hi].min())
            for side, part in ((0, lo), (1, hi)):
                k = part.shape[0]
                ry = np.array([np.sum((y[part] < y[i]) | ((y[part] == y[i]) & (part < i))) for i in part])
                ylo, yhi = part[ry < k // 2], part[ry >= k // 2]
                sy = 0.5 * (y[ylo].max() + y[yhi].min())
                x0, x1 = (R[0], sx) if side == 0 else (sx, R[1])
                nb += [ylo, yhi]
                nr += [(x0, x1, R[2], sy), (x0, x1, sy, R[3])]
        boxes, rects = nb, rects + [nr]
    leaves = [sorted(mem.tolist(), key=lambda i: (x[i], i)) for mem in boxes]
    return leaves, rects


@pytest.mark.parametrize("n,L,seed", [(16, 2, 1), (67, 2, 2), (200, 3, 3), (64, 3, 4), (97, 1, 5)])
def test_tree_matches_counting_brute_force(orc, n, L, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    x = g.random(n)
    y = g.random(n)
    # a few exact ties in each coordinate exercise the index tie-break
    x[: n // 5] = np.round(x[: n // 5], 1)
    y[n // 3: n // 2] = 0.5
    t = orc.tree(x, y, L)
    leaves, rects = brute_tree(x, y, L)
    for b, mem in enumerate(leaves):
        got = t.perm[t.leaf_start[b]:t.leaf_start[b + 1]].tolist()
        assert got == mem
    for l in range(L + 1):
        want = np.array(rects[l], dtype=np.float64)
        assert np.array_equal(t.level_rects(l), want)


@pytest.mark.parametrize("n,L", [(1000, 3), (4 ** 4, 4), (4 ** 4 + 1, 4), (9973, 5)])
def test_leaf_counts_and_containment(orc, n, L):
    ps = W.uniform(n, seed=n)
    t = orc.tree(ps.x, ps.y, L)
    counts = np.diff(t.leaf_start)
    assert counts.min() >= n // 4 ** L and counts.max() <= -(-n // 4 ** L)
    assert sorted(t.perm.tolist()) == list(range(n))
    R = t.level_rects(L)
    for b in range(4 ** L):
        mem = t.perm[t.leaf_start[b]:t.leaf_start[b + 1]]
        assert np.all((ps.x[mem] >= R[b, 0]) & (ps.x[mem] <= R[b, 1]))
        assert np.all((ps.y[mem] >= R[b, 2]) & (ps.y[mem] <= R[b, 3]))
    # children tile their parent
    for l in range(L):
        P = t.level_rects(l)
        C = t.level_rects(l + 1).reshape(-1, 4, 4)
        assert np.array_equal(C[:, 0, 0], P[:, 0]) and np.array_equal(C[:, 3, 1], P[:, 1])
        assert np.array_equal(C[:, 0, 1], C[:, 2, 0])           # shared x split
        assert np.array_equal(C[:, 0, 3], C[:, 1, 2])           # y split, low x half
        assert np.array_equal(C[:, 2, 3], C[:, 3, 2])           # y split, high x half
        assert np.array_equal(C[:, 0, 2], P[:, 2]) and np.array_equal(C[:, 1, 3], P[:, 3])


def test_count_rule_is_data_independent(orc):
    # n -> (floor(floor(n/2)/2), ceil(floor(n/2)/2), floor(ceil(n/2)/2), ceil(ceil(n/2)/2))
    n, L = 1237, 3
    u = W.uniform(n, seed=1)
    c = W.random_mixture(n, seed=2)
    a = orc.tree(u.x, u.y, L)
    b = orc.tree(c.x, c.y, L)
    sizes = [n]
    for _ in range(L):
        nxt = []
        for m in sizes:
            lo, hi = m // 2, m - m // 2
            nxt += [lo // 2, lo - lo // 2, hi // 2, hi - hi // 2]
        sizes = nxt
    assert np.diff(a.leaf_start).tolist() == sizes
    assert np.diff(b.leaf_start).tolist() == sizes


@pytest.mark.parametrize("L", [2, 4])
def test_grid_split_lines_closed_form(orc, L):
    ps = W.grid(L)  # m = 2^(L+1) cells per axis, two points per leaf per axis
    m = 2 ** (L + 1)
    t = orc.tree(ps.x, ps.y, L)
    lo_edge, hi_edge = 0.5 / m, 1.0 - 0.5 / m
    for l in range(L + 1):
        R = t.level_rects(l)
        k = 2 ** l
        for b in range(4 ** l):
            # box b at level l: x index from bits 1,3,5..., y from bits 0,2,4...
            ix = iy = 0
            for lev in range(l):
                digit = (b >> (2 * (l - 1 - lev))) & 3
                ix = 2 * ix + (digit >> 1)
                iy = 2 * iy + (digit & 1)
            want = [ix / k, (ix + 1) / k, iy / k, (iy + 1) / k]
            want[0] = lo_edge if ix == 0 else want[0]
            want[1] = hi_edge if ix == k - 1 else want[1]
            want[2] = lo_edge if iy == 0 else want[2]
            want[3] = hi_edge if iy == k - 1 else want[3]
            assert R[b].tolist() == want


def test_prefix_property(orc):
    ps = W.mixed_1m(scale=0.004)
    deep = orc.tree(ps.x, ps.y, 4)
    for l in range(4):
        shallow = orc.tree(ps.x, ps.y, l)
        assert np.array_equal(deep.rects[:shallow.rects.shape[0]], shallow.rects)
        # same members per level-l box
        per = 4 ** (4 - l)
        for b in range(4 ** l):
            a = set(deep.perm[deep.leaf_start[b * per]:deep.leaf_start[(b + 1) * per]].tolist())
            s = set(shallow.perm[shallow.leaf_start[b]:shallow.leaf_start[b + 1]].tolist())
            assert a == s


def test_geometry_closed_form(orc):
    rects = np.array([[0.0, 1.0, 0.0, 1.0], [0.25, 0.75, -1.0, 0.5], [2.0, 2.0, 3.0, 3.0]])
    g = orc.geometry(rects)
    assert g[0].tolist() == [0.5, 0.5, 0.5 * np.sqrt(2.0)]
    assert g[1].tolist() == [0.5, -0.25, 0.5 * np.sqrt(0.25 + 2.25)]
    assert g[2].tolist() == [2.0, 3.0, 0.0]


def test_negative_zero_is_zero(orc):
    # -0 and +0 are the same number: trees of the two inputs are identical
    # bit for bit (rectangles included).
    ps = W.uniform(500, seed=31)
    x, y = ps.x.copy(), ps.y.copy()
    x[:60] = 0.0
    y[:40] = 0.0
    xn, yn = x.copy(), y.copy()
    xn[:30] = -0.0
    yn[10:25] = -0.0
    a = orc.tree(x, y, 3)
    b = orc.tree(xn, yn, 3)
    assert np.array_equal(a.perm, b.perm)
    assert np.array_equal(a.rects.view(np.int64), b.rects.view(np.int64))
