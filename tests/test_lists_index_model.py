"""A CPU replay of the index arithmetic of the GPU list build, checked for
bounds on every parity input.

The GPU builds the interaction lists (Section 4's connectivity rule under
Criterion 2.1) in flat passes over each level's candidate space, with pool
sizes chosen on the host and grown on retry.  This module re-derives, in
NumPy, every index those kernels form -- the decoding of a candidate number
into (box, candidate box) through the owner table, the row pointers and
source-list reads, the word counts and tile sums of the scan, the pool
positions, owners, near-field records and self positions that the fill pass
writes -- for the list sizes the oracle's lists give, including the host's
retry loop and the device-side guards (pool space, entry limit).  Every index
is checked against the size of the buffer it addresses, and the lists the
replay assembles must equal the oracle's.  The decisions themselves are taken
from the oracle's lists; what is modelled is where each decision goes.

This is test infrastructure: it models the kernels' indexing only and holds
none of the method's arithmetic.
"""
import numpy as np
import pytest

from tests.gpu_cases import TREE_CASES

WS_TILE = 256 * 16        # words per scan tile
SMALL_BOXES = 64          # levels of at most this many boxes run in one workgroup
SMALL_GEOM = 85           # geometry of levels 0..3 staged in LDS
POOL_MAX = 1 << 34
INT32_MAX = (1 << 31) - 1


def level_offset(l):
    return (4 ** l - 1) // 3


class Bounds:
    """Largest index used per buffer, against its size."""

    def __init__(self):
        self.used = {}

    def touch(self, name, idx, size):
        idx = np.asarray(idx)
        if idx.size == 0:
            return
        lo, hi = int(idx.min()), int(idx.max())
        assert lo >= 0, "%s: index %d < 0" % (name, lo)
        assert hi < size, "%s: index %d >= size %d" % (name, hi, size)
        prev = self.used.get(name, (-1, size))
        self.used[name] = (max(prev[0], hi), size)


VFLAG = 1 << 30
GROW_S, GROW_W, GROW_X, GROW_CAND = 4, 8, 16, 32


def _attempt(ls, L, cap_s, cap_w, limit, bd, cap_x=0, all_flat=False):
    """One build_lists_device call; returns (overflow flag, pool offsets,
    replayed S and W lists per level).  With optimised lists (``ls.vptr``
    present) the W output holds V entries (flagged) and an X pool is used.
    ``all_flat``: every level in the flat passes (the relaxed criterion's
    build, which needs each level's threshold before its count pass)."""
    opt = getattr(ls, "vptr", None) is not None
    nS = [int(ls.sptr[l][-1]) for l in range(L + 1)]
    nW = [int(ls.wptr[l][-1]) + (int(ls.vptr[l][-1]) if opt else 0) for l in range(L + 1)]
    nX = [int(ls.xptr[l][-1]) if opt else 0 for l in range(L + 1)]
    s_off = [0] * (L + 2)
    w_off = [0] * (L + 2)
    x_off = [0] * (L + 2)
    s_off[1] = 1
    flag = 0
    got_s, got_w = {0: np.array([0])}, {0: np.zeros(0, np.int64)}
    got_x = {0: np.zeros(0, np.int64)}
    n_leaf = 4 ** L
    leaf_rows = n_leaf + 1
    # buffers as sized by the host
    if L >= 1 and 16 > limit:
        return 2, s_off, got_s, got_w, got_x, (s_off, w_off, x_off)
    words_cap = (cap_s + cap_w + 63) // 64 + 1
    ntile = (words_cap + WS_TILE - 1) // WS_TILE
    K = 0
    while not all_flat and K < L and 4 ** (K + 1) <= SMALL_BOXES:
        K += 1

    def advance(l):
        nonlocal flag
        if flag:
            return
        so = s_off[l] + nS[l]
        wo = w_off[l] + nW[l]
        xo = x_off[l] + nX[l]
        s_off[l + 1] = so
        w_off[l + 1] = wo
        x_off[l + 1] = xo
        grow = (GROW_S if so > cap_s else 0) | (GROW_W if wo > cap_w else 0) | (GROW_X if xo > cap_x else 0)
        if grow:
            flag = grow
            return
        if l < L:
            cand = 16 * nS[l]
            if cand > limit:
                flag = 2
            elif cand > (cap_s - so) + (cap_w - wo):
                flag = GROW_CAND

    for l in range(1, L + 1):
        if flag:
            break
        nb, nb_prev = 4 ** l, 4 ** (l - 1)
        sp_prev = np.asarray(ls.sptr[l - 1], np.int64)
        si_prev = np.asarray(ls.sidx[l - 1], np.int64)
        # candidates of level l in the order both passes number them
        P_of_entry = np.repeat(np.arange(nb_prev), np.diff(sp_prev))   # owner table of S_{l-1}
        NC = 16 * nS[l - 1]
        q = np.arange(NC, dtype=np.int64)
        if l > K:
            nwords = (NC + 63) // 64
            bd.touch("bits/cnt (words)", np.arange(nwords), words_cap)
            if opt:  # exchanged and group-head masks at wcap and 2 wcap
                bd.touch("bits (three masks)", 2 * words_cap + np.arange(nwords), 3 * words_cap)
            bd.touch("scan tiles", np.arange((nwords + WS_TILE - 1) // WS_TILE), ntile)
            bd.touch("owner_prev", q >> 4, cap_s)
            bd.touch("owner_prev written", q >> 4, nS[l - 1])
        P = P_of_entry[q >> 4]
        bd.touch("sptr_prev", P + 1, nb_prev + 1)
        s0, s1 = sp_prev[P], sp_prev[P + 1]
        r = q - 16 * s0
        m4 = 4 * (s1 - s0)
        c = (r >= m4).astype(np.int64) + (r >= 2 * m4) + (r >= 3 * m4)
        j = r - c * m4
        assert np.all((j >= 0) & (j < m4)), "candidate decodes outside its box"
        b = 4 * P + c
        ent_pos = s0 + (j >> 2)
        assert np.all(ent_pos < s1)
        bd.touch("sidx (previous level)", s_off[l - 1] + ent_pos, cap_s)
        cbox = 4 * si_prev[ent_pos] + (j & 3)
        bd.touch("geom b", b, nb)
        bd.touch("geom cbox", cbox, nb)
        if l <= K:
            bd.touch("geometry in LDS", level_offset(l) + np.concatenate([b, cbox]), SMALL_GEOM)
        # decisions from the oracle's lists: candidate weak iff in W_l(b)
        # (a member of a parent group iff its parent is in V_l(b), the
        # group's first child then writes the V entry), exchanged iff in X_l(b)
        wp, wi = np.asarray(ls.wptr[l], np.int64), np.asarray(ls.widx[l], np.int64)
        wkeys = np.repeat(np.arange(nb, dtype=np.int64), np.diff(wp)) * nb + wi
        weak = np.isin(b * nb + cbox, wkeys)
        head = np.zeros(NC, bool)
        exch = np.zeros(NC, bool)
        member = np.zeros(NC, bool)
        if opt:
            vp, vi = np.asarray(ls.vptr[l], np.int64), np.asarray(ls.vidx[l], np.int64)
            vkeys = np.repeat(np.arange(nb, dtype=np.int64), np.diff(vp)) * nb + vi
            member = np.isin(b * nb + (cbox >> 2), vkeys)
            head = member & ((cbox & 3) == 0)
            xp, xi = np.asarray(ls.xptr[l], np.int64), np.asarray(ls.xidx[l], np.int64)
            xkeys = np.repeat(np.arange(nb, dtype=np.int64), np.diff(xp)) * nb + xi
            exch = np.isin(b * nb + cbox, xkeys)
            assert not np.any(weak & (member | exch)) and not np.any(member & exch)
        wout = weak | head
        strong = ~(weak | member | exch)
        # scans: pool positions and row pointers
        posS = np.cumsum(strong) - strong
        posW = np.cumsum(wout) - wout
        posX = np.cumsum(exch) - exch
        advance(l)
        if flag:
            break
        bd.touch("sidx pool (level %d)" % l, s_off[l] + posS[strong], cap_s)
        bd.touch("widx pool (level %d)" % l, w_off[l] + posW[wout], cap_w)
        if opt:
            bd.touch("xidx pool (level %d)" % l, x_off[l] + posX[exch], max(cap_x, 1))
            if l > 1:
                bd.touch("parent geometry", (cbox >> 2)[head], 4 ** (l - 1))
        bd.touch("owner_cur", posS[strong], cap_s)
        first = np.zeros(NC, bool)
        first[np.flatnonzero(j == 0)] = True
        bd.touch("sptr_cur", b[first], nb + 1)
        if l == L:
            bd.touch("near records", posS[strong], cap_s)
            bd.touch("leaf starts", cbox[strong] + 1, leaf_rows)
            selfb = b[strong & (cbox == b)]
            bd.touch("selfpos", selfb, n_leaf)
            assert np.array_equal(np.sort(selfb), np.arange(nb)), "a leaf without its own entry"
        # the lists the fill pass writes
        S = np.empty(nS[l], np.int64)
        S[posS[strong]] = cbox[strong]
        W = np.empty(nW[l], np.int64)
        W[posW[weak]] = cbox[weak]
        W[posW[head]] = (cbox[head] >> 2) | VFLAG
        X = np.empty(nX[l], np.int64)
        X[posX[exch]] = cbox[exch]
        got_s[l], got_w[l], got_x[l] = S, W, X
    return flag, s_off, got_s, got_w, got_x, (s_off, w_off, x_off)


def split_w(W):
    """A W output list with parent entries flagged -> (W entries, V entries)."""
    W = np.asarray(W, np.int64)
    flagged = (W & VFLAG) != 0
    return W[~flagged], W[flagged] & (VFLAG - 1)


def replay_connectivity(ls, L, hint_s=0, hint_w=0, limit=INT32_MAX, swaps=False, hint_x=0, all_flat=False):
    """fmm2d_connectivity's retry loop around the replayed build.  Returns
    (status, attempts, bounds, caps)."""
    nbox = level_offset(L + 1)
    cap_s = max(32 * nbox + 64, hint_s)
    cap_w = max(96 * nbox + 64, hint_w)
    cap_x = max(16 * nbox + 64, hint_x) if swaps else 0
    bd = Bounds()
    opt = getattr(ls, "vptr", None) is not None
    for attempt in range(16):
        flag, s_off, got_s, got_w, got_x, offs = _attempt(ls, L, cap_s, cap_w, limit, bd, cap_x, all_flat)
        if flag == 0:
            for l in range(L + 1):
                assert np.array_equal(got_s[l], ls.sidx[l]), "replayed S list of level %d differs" % l
                w, v = split_w(got_w[l])
                assert np.array_equal(w, ls.widx[l]), "replayed W list of level %d differs" % l
                if opt:
                    assert np.array_equal(v, ls.vidx[l]), "replayed V list of level %d differs" % l
                    assert np.array_equal(got_x[l], ls.xidx[l]), "replayed X list of level %d differs" % l
            return "ok", attempt + 1, bd, (cap_s, cap_w, cap_x)
        if flag == 2:
            return "capacity", attempt + 1, bd, (cap_s, cap_w, cap_x)
        # only the flagged pools grow, to at least twice the entries so far
        need_s, need_w, need_x = (max(o) for o in offs)
        grown = lambda cap, need: min(POOL_MAX, max(4 * cap, 2 * need))
        old = (cap_s, cap_w, cap_x)
        if flag & GROW_S:
            cap_s = grown(cap_s, need_s)
        if flag & (GROW_W | GROW_CAND):
            cap_w = grown(cap_w, need_w)
        if flag & GROW_X:
            cap_x = grown(cap_x, need_x)
        if (cap_s, cap_w, cap_x) == old:
            break
    return "nomem", 16, bd, (cap_s, cap_w, cap_x)


@pytest.mark.parametrize("case", sorted(TREE_CASES))
@pytest.mark.parametrize("theta", [0.5, 0.3, 0.75])
def test_list_indices_in_bounds(orc, case, theta):
    maker, L = TREE_CASES[case]
    ps = maker()
    ls = orc.lists(orc.tree(ps.x, ps.y, L), theta)
    # a fresh context, and one whose pools were left large by earlier inputs
    for hint in (0, 1 << 22):
        status, attempts, bd, caps = replay_connectivity(ls, L, hint, 3 * hint)
        assert status == "ok"


def test_clustered_case_grows_pools_in_bounds(orc):
    """The clustered 20k-point input at theta = 1/2 needs larger pools than
    the first attempt's: the replay takes the retry and stays in bounds."""
    maker, L = TREE_CASES["clustered_scaled_20k_L6"]
    ps = maker()
    ls = orc.lists(orc.tree(ps.x, ps.y, L), 0.5)
    status, attempts, bd, caps = replay_connectivity(ls, L)
    assert status == "ok" and attempts >= 2
    for name, (hi, size) in sorted(bd.used.items()):
        assert hi < size


def test_entry_limit_reported_before_any_level_overflows(orc):
    maker, L = TREE_CASES["clustered_scaled_20k_L6"]
    ps = maker()
    ls = orc.lists(orc.tree(ps.x, ps.y, L), 0.5)
    status, _, _, _ = replay_connectivity(ls, L, limit=50000)
    assert status == "capacity"


@pytest.mark.parametrize("case", ["clustered_scaled_20k_L6", "mixed_scaled_20k_L6", "uniform_20k_L5",
                                  "duplicates_4k_L4", "scales_3k_L4", "single_box_L0", "uniform_1k_L3"])
@pytest.mark.parametrize("parent,swap", [(True, "finest"), (True, "all"), (False, "all"), (True, "none")])
def test_opt_list_indices_in_bounds(orc, case, parent, swap):
    maker, L = TREE_CASES[case]
    ps = maker()
    t = orc.tree(ps.x, ps.y, L)
    levels = {"finest": (L,), "all": tuple(range(1, L + 1)), "none": ()}[swap]
    ls = orc.lists_opt(t, 0.5, parent=parent, swap_levels=levels)
    for hint in (0, 1 << 22):
        status, attempts, bd, caps = replay_connectivity(ls, L, hint, 3 * hint, swaps=swap != "none",
                                                         hint_x=hint)
        assert status == "ok"


@pytest.mark.parametrize("case", ["clustered_scaled_20k_L6", "mixed_scaled_20k_L6", "ring_scaled_20k_L6",
                                  "uniform_20k_L5", "duplicates_4k_L4", "scales_3k_L4", "single_box_L0",
                                  "uniform_1k_L3"])
@pytest.mark.parametrize("theta,theta_max,p", [(0.5, 0.9, 12), (0.35, 0.8, 6), (0.7, 0.7, 12)])
def test_relaxed_list_indices_in_bounds(orc, case, theta, theta_max, p):
    """The relaxed criterion's build: every level (the coarse ones too) in the
    flat passes, with the lists the relaxed rule gives; the bin counters of
    a level are (L + 1) (k0 + k1) words, indexed l (k0 + k1) + bin."""
    maker, L = TREE_CASES[case]
    ps = maker()
    ls = orc.lists_relaxed(orc.tree(ps.x, ps.y, L), theta, theta_max, p)
    nbin = ls.k0 + ls.k1
    for l in range(L + 1):
        assert len(ls.count[l]) == nbin and 0 <= ls.kmax[l] < nbin
        assert l * nbin + nbin - 1 < (L + 1) * nbin
    for hint in (0, 1 << 22):
        status, attempts, bd, caps = replay_connectivity(ls, L, hint, 3 * hint, all_flat=True)
        assert status == "ok"
