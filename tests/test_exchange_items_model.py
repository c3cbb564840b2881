"""A CPU replay of the work-item schedule of the exchanged-roles P2L pass,
checked for bounds and coverage on parity inputs.

The host picks the first level of whole-entry (lane-per-item) items, sizes
the item array from the X list sizes, and the device enumerates items per
target box: chunks of one entry's source points on the coarser levels, whole
entries from that level on.  The replay rebuilds that enumeration from the
oracle's optimised lists and checks that every index the kernels form lies
in its buffer, that the wavefront-per-item range precedes the lane-per-item
range, and that each P2L entry's source points are covered exactly once.

This is test infrastructure: it models the kernels' indexing only and holds
none of the method's arithmetic.
"""
import numpy as np
import pytest

from tests.gpu_cases import TREE_CASES

PCH = 512


def level_offset(l):
    return (4 ** l - 1) // 3


def level_of(g):
    l = 0
    while level_offset(l + 1) <= g:
        l += 1
    return l


def level_box_max(n, l):
    return -(-n // 4 ** l)


def level_chunk(n, l):
    m = level_box_max(n, l)
    k = min(32, max(1, -(-m // PCH)))
    return -(-m // k)


def lane_level_of(n, L, nx, lane_pts, lane_pts_many, lane_entries):
    ll = L + 1
    for l in range(L, 0, -1):
        m = level_box_max(n, l)
        if m <= lane_pts or (m <= lane_pts_many and nx[l] // 2 >= lane_entries):
            ll = l
        else:
            break
    return ll


@pytest.mark.parametrize("case", ["clustered_scaled_20k_L6", "mixed_scaled_20k_L6", "ring_scaled_20k_L6",
                                  "duplicates_4k_L4", "uniform_2000_L2", "single_box_L0"])
@pytest.mark.parametrize("thresholds", [(256, 4096, 32768), (16, 4096, 200), (0, 0, 1 << 40), (1 << 30, 0, 0)])
def test_p2l_items_cover_and_bound(orc, case, thresholds):
    maker, L = TREE_CASES[case]
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists_opt(t, 0.5, parent=True, swap_levels=range(1, L + 1))
    n = ps.n
    nx = [int(ls.xptr[l][-1]) for l in range(L + 1)]
    ll = lane_level_of(n, L, nx, *thresholds)
    bw = sum(nx[l] * -(-level_box_max(n, l) // level_chunk(n, l)) for l in range(1, min(ll, L + 1)))
    bl = sum(nx[l] for l in range(max(ll, 1), L + 1))
    bound = max(bw + bl, 1)
    starts = t.leaf_start
    items, itemoff, box = [], [0], {}
    for l in range(L + 1):
        r = t.geom[level_offset(l):level_offset(l + 1), 2]
        for b in range(4 ** l):
            if l >= 1:
                for pos in range(ls.xptr[l][b], ls.xptr[l][b + 1]):
                    c = int(ls.xidx[l][pos])
                    if not r[b] < r[c]:
                        continue  # M2P entry
                    a, e = starts[c << 2 * (L - l)], starts[(c + 1) << 2 * (L - l)]
                    assert 0 <= a < e <= n
                    box[(level_offset(l) + b, pos)] = (a, e)
                    if l >= ll:
                        items.append((level_offset(l) + b, pos, -1, a, e))
                    else:
                        ch = level_chunk(n, l)
                        for j in range(a, e, ch):
                            items.append((level_offset(l) + b, pos, j, j, min(e, j + ch)))
            itemoff.append(len(items))
    nitem = len(items)
    assert nitem <= bound
    wave_end = itemoff[level_offset(min(ll, L + 1))]
    assert all(it[2] >= 0 for it in items[:wave_end]) and all(it[2] == -1 for it in items[wave_end:])
    assert wave_end <= max(bw, 0) or bw == 0 and wave_end == 0
    assert nitem - wave_end <= bl
    # every P2L entry covered once, its chunks disjoint and inside the box
    cover = {}
    for g, pos, j, a, e in items:
        cover.setdefault((g, pos), []).append((a, e))
    for key, segs in cover.items():
        segs.sort()
        assert segs[0][0] == box[key][0] and segs[-1][1] == box[key][1]
        for (a0, e0), (a1, e1) in zip(segs, segs[1:]):
            assert e0 == a1
    assert set(cover) == set(box)
    # the items of a box are consecutive and the boxes in order
    gs = [it[0] for it in items]
    assert gs == sorted(gs)


M2P_WIDE_PTS = 256


def m2p_groups(w):
    return min(64 // w, 8)


def m2p_width(n, l):
    """Pass width: 64 on levels of M2P_WIDE_PTS points or more, else the
    width of the pass count (ceil(m / 64) up to three more) with the most
    groups per pass."""
    m = level_box_max(n, l)
    if m >= M2P_WIDE_PTS:
        return 64
    best_w, best_g, best_np = 64, 0, 1
    np0 = -(-m // 64)
    for np_ in range(np0, np0 + 4):
        w = -(-m // np_)
        ng = m2p_groups(w)
        if ng * best_np > best_g * np_:
            best_w, best_g, best_np = w, ng, np_
    return best_w


def test_m2p_width_fills_lanes():
    """Worked cases: 38-point boxes in two passes of 19 over three groups (57
    of 64 lanes), 152-point boxes in five passes of 31 over two groups, ten
    points in one pass over six groups, 64-point passes from 256 points."""
    assert m2p_width(38 * 4 ** 9, 9) == 19 and m2p_groups(19) == 3
    assert m2p_width(152 * 4 ** 8, 8) == 31 and m2p_groups(31) == 2
    assert m2p_width(10 * 4 ** 5, 5) == 10 and m2p_groups(10) == 6
    assert m2p_width(256 * 4 ** 3, 3) == 64
    for m in range(1, 256):
        w = m2p_width(m * 4, 1)
        assert 1 <= w <= 64 and -(-m // w) <= -(-m // 64) + 3
        assert m2p_groups(w) * w <= 64


MSPAN = 64


@pytest.mark.parametrize("case", ["clustered_scaled_20k_L6", "mixed_scaled_20k_L6", "ring_scaled_20k_L6",
                                  "duplicates_4k_L4", "uniform_2000_L2", "uniform_10k_L5"])
def test_m2p_items_cover_and_bound(orc, case):
    """M2P items: per box with an M2P entry, its point passes (of
    m2p_width(n, l) points) times balanced spans of its X row of at most MSPAN positions, point pass
    major.  Checks: the item count within the schedule's bound, every
    (point, row position) pair of such a box in exactly one item, and the
    per-point sum's indexing (pass and span from the box's item range) naming
    exactly the items that hold the point, at a lane below 64."""
    maker, L = TREE_CASES[case]
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    ls = orc.lists_opt(t, 0.5, parent=True, swap_levels=range(1, L + 1))
    n, starts = ps.n, t.leaf_start
    wl = next((l for l in range(1, L + 1) if level_box_max(n, l) < M2P_WIDE_PTS), L + 1)
    bound_w = bound_n = 0
    items, itemoff = [], {}
    for l in range(1, L + 1):
        nx = int(ls.xptr[l][-1])
        mp = m2p_width(n, l)
        npc_max = -(-level_box_max(n, l) // mp)
        bnd = npc_max * (min(nx, 4 ** l) + nx // MSPAN)
        if l < wl:
            bound_w += bnd
        else:
            bound_n += bnd
        r = t.geom[level_offset(l):level_offset(l + 1), 2]
        for b in range(4 ** l):
            t0, t1 = int(ls.xptr[l][b]), int(ls.xptr[l][b + 1])
            row = ls.xidx[l][t0:t1]
            g = level_offset(l) + b
            i0 = len(items)
            if any(r[b] > r[c] for c in row):
                a, e = int(starts[b << 2 * (L - l)]), int(starts[(b + 1) << 2 * (L - l)])
                step = mp
                npc = -(-(e - a) // step)
                assert npc <= npc_max
                nsp = -(-(t1 - t0) // MSPAN)
                span = -(-(t1 - t0) // nsp)
                for q in range(npc * nsp):
                    pc, sp = divmod(q, nsp)
                    s0 = t0 + sp * span
                    items.append((g, a + pc * step, s0, min(t1, s0 + span)))
            itemoff[g] = (i0, len(items))
    nw = sum(1 for it in items if level_of(it[0]) < wl)
    assert nw <= bound_w and len(items) - nw <= bound_n
    # items of a box consecutive, boxes in order (wide levels first)
    gs = [it[0] for it in items]
    assert gs == sorted(gs)
    for g, (i0, i1) in itemoff.items():
        if i0 == i1:
            continue
        l = level_of(g)
        b = g - level_offset(l)
        a, e = int(starts[b << 2 * (L - l)]), int(starts[(b + 1) << 2 * (L - l)])
        t0, t1 = int(ls.xptr[l][b]), int(ls.xptr[l][b + 1])
        step = m2p_width(n, l)
        npc = -(-(e - a) // step)
        assert (i1 - i0) % npc == 0
        nsp = (i1 - i0) // npc
        cover = np.zeros((e - a, t1 - t0), dtype=np.int64)
        for k in range(i0, i1):
            _, f, s0, s1 = items[k]
            assert s1 - s0 <= MSPAN and t0 <= s0 < s1 <= t1
            pts = np.arange(f, min(f + step, e))
            cover[np.ix_(pts - a, np.arange(s0, s1) - t0)] += 1
        assert (cover == 1).all()
        # the per-point sum: pass pc, items i0 + pc * nsp + [0, nsp), lane o
        for i in range(a, e):
            pc = (i - a) // step
            o = i - a - pc * step
            assert 0 <= o < 64 and o < step
            for s in range(nsp):
                _, f, s0, s1 = items[i0 + pc * nsp + s]
                assert f <= i < f + step and i - f == o
