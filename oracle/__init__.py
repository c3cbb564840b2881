"""CPU oracle for the asymmetric adaptive 2D FMM -- TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import it; the product path never
does.  It shares no code with the GPU library (its C part, ``fmm2d_oracle.c``,
is compiled on its own with gcc) and the two only meet through the seeded
input generators in ``paper_1006_2269_amd.workloads``.

What each function follows in Engblom, "On well-separated sets and fast
multipole methods":

* ``direct``     -- the interaction sum (1.1) with charges and G = log|x - y|.
* ``tree``       -- the balanced median-split pyramid (Section 4, Fig. 1.1).
* ``tree_midpoint`` -- the uniform quadtree (midpoint splits, all leaves at
                    one depth) that Section 5's second experiment compares
                    the adaptive tree with.
* ``shrink``     -- the same boxes with the balls of Criterion 2.1 drawn
                    around each box's points (their bounding box) instead of
                    the tiling rectangle.
* ``geometry``   -- centre / enclosing-ball radius of each box, the balls of
                    Criterion 2.1.
* ``lists``      -- the recursive strong/weak connectivity rule (Section 4)
                    with the theta-criterion (Criterion 2.1).
* ``lists_opt``  -- the same with the structural optimisations of Section 4:
                    interaction via the parent box, and exchanged roles
                    (P2L / M2P) for boxes of very different radii.
* ``lists_relaxed`` -- the plain rule with a locally relaxed theta (Section 4,
                    last paragraph): pairs with their own theta_i above theta
                    admitted as weak while the level's mean of theta_i^(p+1)
                    stays at most theta^(p+1).
* ``fmm``        -- upward pass, M2L along weak lists, downward pass, direct
                    sum along the finest strong lists (Section 4) in the
                    complex multipole representation (Section 5).
* ``rel_errors`` -- normwise relative error, as measured in Section 5.
* ``a_priori``   -- p from the estimate const * theta^(p+1) / (1-theta)^2
                    (Section 3) and the practical defaults of Section 4.

Every function here is pinned by tests under ``tests/`` that do not re-use its
own formulas (closed forms, brute force, invariants, the paper's bound).
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fmm2d_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liborc_fmm2d.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc into ``oracle/liborc_fmm2d.so``."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    d = ctypes.c_double
    lib.orc_direct.argtypes = [i64, P, P, P, i64, P, P]
    lib.orc_direct.restype = None
    lib.orc_tree.argtypes = [i64, P, P, i32, P, P, P]
    lib.orc_tree.restype = i32
    lib.orc_tree_midpoint.argtypes = [i64, P, P, i32, P, P, P]
    lib.orc_tree_midpoint.restype = i32
    lib.orc_geometry.argtypes = [i64, P, P]
    lib.orc_geometry.restype = None
    lib.orc_theta_test.argtypes = [d, P, P]
    lib.orc_theta_test.restype = i32
    lib.orc_lists_level.argtypes = [i32, d, P, P, P, P, P, P, P, i64]
    lib.orc_lists_level.restype = i32
    lib.orc_swap_test.argtypes = [d, P, P]
    lib.orc_swap_test.restype = i32
    lib.orc_lists_level_opt.argtypes = [i32, d, i32, i32, P, P, P, P, P, P, P, P, P, P, P, P, i64]
    lib.orc_lists_level_opt.restype = i32
    lib.orc_lists_level_relaxed.argtypes = [i32, d, d, i32, i32, i32, P, P, P, P, P, P, P, i64, P, P]
    lib.orc_lists_level_relaxed.restype = i32
    lib.orc_p2l.argtypes = [i64, P, P, P, d, d, d, i32, P]
    lib.orc_p2l.restype = None
    lib.orc_fmm_eval_opt.argtypes = [i64, P, P, P, i32, i32] + [P] * 17
    lib.orc_fmm_eval_opt.restype = i32
    lib.orc_p2m.argtypes = [i64, P, P, P, d, d, d, i32, P]
    lib.orc_p2m.restype = None
    lib.orc_m2m.argtypes = [P, d, d, d, d, d, d, i32, P]
    lib.orc_m2m.restype = None
    lib.orc_m2l.argtypes = [P, d, d, d, d, d, d, i32, P]
    lib.orc_m2l.restype = None
    lib.orc_l2l.argtypes = [P, d, d, d, d, d, d, i32, P]
    lib.orc_l2l.restype = None
    lib.orc_l2p.argtypes = [P, d, d, d, i32, i64, P, P, P]
    lib.orc_l2p.restype = None
    lib.orc_m2p.argtypes = [P, d, d, d, i32, i64, P, P, P]
    lib.orc_m2p.restype = None
    lib.orc_fmm_eval.argtypes = [i64, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P]
    lib.orc_fmm_eval.restype = i32
    lib.orc_fmm_eval_field.argtypes = [i64, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_fmm_eval_field.restype = i32
    lib.orc_direct_field.argtypes = [i64, P, P, P, i64, P, P, P]
    lib.orc_direct_field.restype = None
    lib.orc_l2p_grad.argtypes = [P, d, d, d, i32, i64, P, P, P, P]
    lib.orc_l2p_grad.restype = None
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def level_offset(l: int) -> int:
    """First global box id of level l: (4^l - 1) / 3."""
    return (4 ** l - 1) // 3


# --------------------------------------------------------------------------
# O1: direct sum (1.1)
# --------------------------------------------------------------------------
def direct(x, y, q, targets=None) -> np.ndarray:
    """Phi_i = sum over j with (x_j, y_j) != (x_i, y_i) of q_j log|z_i - z_j|,
    in binary64 with compensated summation, at the given target indices
    (all points when ``targets`` is None)."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    n = x.shape[0]
    t = _i64(np.arange(n) if targets is None else targets)
    out = np.empty(t.shape[0], dtype=np.float64)
    lib.orc_direct(n, _p(x), _p(y), _p(q), t.shape[0], _p(t), _p(out))
    return out


def direct_field(x, y, q, targets=None):
    """(d Phi/dx, d Phi/dy) at the given target indices: the gradient of the
    sum (1.1), sum over j with (x_j, y_j) != (x_i, y_i) of q_j (z_i - z_j) /
    |z_i - z_j|^2 componentwise, binary64 with compensated summation."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    n = x.shape[0]
    t = _i64(np.arange(n) if targets is None else targets)
    gx = np.empty(t.shape[0], dtype=np.float64)
    gy = np.empty(t.shape[0], dtype=np.float64)
    lib.orc_direct_field(n, _p(x), _p(y), _p(q), t.shape[0], _p(t), _p(gx), _p(gy))
    return gx, gy


# --------------------------------------------------------------------------
# O2: tree and box geometry
# --------------------------------------------------------------------------
@dataclass
class Tree:
    n: int
    levels: int
    perm: np.ndarray        # int64 [n]: original index of each point, leaf order
    leaf_start: np.ndarray  # int64 [4^L + 1]
    rects: np.ndarray       # float64 [nbox, 4]: xlo, xhi, ylo, yhi (all levels)
    geom: np.ndarray        # float64 [nbox, 3]: cx, cy, r (all levels)

    def level_rects(self, l: int) -> np.ndarray:
        return self.rects[level_offset(l):level_offset(l + 1)]

    def level_geom(self, l: int) -> np.ndarray:
        return self.geom[level_offset(l):level_offset(l + 1)]


def tree(x, y, levels: int) -> Tree:
    """Median-split pyramid with `levels` levels (Section 4, Fig. 1.1)."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    if levels < 0 or levels > 13 or n < 4 ** levels:
        raise ValueError("need 0 <= levels <= 13 and n >= 4^levels")
    nbox = level_offset(levels + 1)
    perm = np.empty(n, dtype=np.int64)
    start = np.empty(4 ** levels + 1, dtype=np.int64)
    rects = np.empty((nbox, 4), dtype=np.float64)
    rc = lib.orc_tree(n, _p(x), _p(y), levels, _p(perm), _p(start), _p(rects))
    if rc != 0:
        raise RuntimeError("orc_tree failed: %d" % rc)
    geom = geometry(rects)
    return Tree(n, levels, perm, start, rects, geom)


def tree_midpoint(x, y, levels: int) -> Tree:
    """The uniform quadtree of the comparison in Section 5's second
    experiment: every box split at its rectangle's midpoint in both
    coordinates, all leaves at depth ``levels`` (congruent boxes per level,
    any number of points per box, empty boxes included)."""
    lib = _load()
    x, y = _f64(x), _f64(y)
    n = x.shape[0]
    if levels < 0 or levels > 13 or n < 1:
        raise ValueError("need 0 <= levels <= 13 and n >= 1")
    nbox = level_offset(levels + 1)
    perm = np.empty(n, dtype=np.int64)
    start = np.empty(4 ** levels + 1, dtype=np.int64)
    rects = np.empty((nbox, 4), dtype=np.float64)
    rc = lib.orc_tree_midpoint(n, _p(x), _p(y), levels, _p(perm), _p(start), _p(rects))
    if rc != 0:
        raise RuntimeError("orc_tree_midpoint failed: %d" % rc)
    return Tree(n, levels, perm, start, rects, geometry(rects))


def point_rects(t: Tree, x, y) -> np.ndarray:
    """(xmin, xmax, ymin, ymax) of the points of every box of every level
    (a box's points are the leaves b 4^(L-l) .. (b+1) 4^(L-l) - 1)."""
    x, y = _f64(x)[t.perm], _f64(y)[t.perm]
    out = np.empty((level_offset(t.levels + 1), 4), dtype=np.float64)
    for l in range(t.levels + 1):
        nb, span = 4 ** l, 4 ** (t.levels - l)
        st = t.leaf_start[::span]
        for b in range(nb):
            a, e = st[b], st[b + 1]
            out[level_offset(l) + b] = (x[a:e].min(), x[a:e].max(), y[a:e].min(), y[a:e].max())
    return out


def shrink(t: Tree, x, y) -> Tree:
    """The tree with each box's ball drawn around its points: centre and half
    diagonal of the points' bounding box (the rectangles stay the tiling
    ones).  Criterion 2.1 holds for any balls enclosing the two point sets;
    the tiling rectangle's ball is one choice, this one is the smallest
    axis-aligned one."""
    pr = point_rects(t, x, y)
    return Tree(t.n, t.levels, t.perm, t.leaf_start, t.rects, geometry(pr))


def geometry(rects) -> np.ndarray:
    """(cx, cy, r): rectangle centre and half diagonal, each operation a single
    rounded binary64 operation."""
    lib = _load()
    rects = _f64(rects).reshape(-1, 4)
    geom = np.empty((rects.shape[0], 3), dtype=np.float64)
    lib.orc_geometry(rects.shape[0], _p(rects), _p(geom))
    return geom


def theta_test(theta: float, gb, gc) -> bool:
    """Criterion 2.1 on two balls (cx, cy, r)."""
    lib = _load()
    gb, gc = _f64(gb), _f64(gc)
    return bool(lib.orc_theta_test(theta, _p(gb), _p(gc)))


# --------------------------------------------------------------------------
# O3: connectivity
# --------------------------------------------------------------------------
@dataclass
class Lists:
    theta: float
    sptr: list   # per level l = 0..L: int64 [4^l + 1]
    sidx: list   # per level: int64 [nnz]
    wptr: list
    widx: list


def lists(t: Tree, theta: float) -> Lists:
    """Strong and weak lists of every level by the recursive rule of Section 4."""
    if not (0.0 < theta < 1.0):
        raise ValueError("theta must lie in (0, 1)")
    lib = _load()
    sptr = [np.array([0, 1], dtype=np.int64)]
    sidx = [np.array([0], dtype=np.int64)]
    wptr = [np.array([0, 0], dtype=np.int64)]
    widx = [np.zeros(0, dtype=np.int64)]
    for l in range(1, t.levels + 1):
        nb = 4 ** l
        cap = 16 * int(sidx[-1].shape[0])
        sp = np.empty(nb + 1, dtype=np.int64)
        wp = np.empty(nb + 1, dtype=np.int64)
        si = np.empty(cap, dtype=np.int64)
        wi = np.empty(cap, dtype=np.int64)
        g = np.ascontiguousarray(t.level_geom(l))
        rc = lib.orc_lists_level(l, theta, _p(g), _p(sptr[-1]), _p(sidx[-1]),
                                 _p(sp), _p(si), _p(wp), _p(wi), cap)
        if rc != 0:
            raise RuntimeError("orc_lists_level overflow")
        sptr.append(sp)
        sidx.append(si[:sp[-1]].copy())
        wptr.append(wp)
        widx.append(wi[:wp[-1]].copy())
    return Lists(theta, sptr, sidx, wptr, widx)


def swap_test(theta: float, gb, gc) -> bool:
    """The criterion with the roles of the radii exchanged (Section 4's
    structural optimisation): r + theta R <= theta d, balls disjoint."""
    lib = _load()
    gb, gc = _f64(gb), _f64(gc)
    return bool(lib.orc_swap_test(theta, _p(gb), _p(gc)))


@dataclass
class ListsOpt(Lists):
    vptr: list = None   # per level: int64 [4^l + 1]; V entries are boxes of level l - 1
    vidx: list = None
    xptr: list = None   # per level: exchanged-roles entries (boxes of level l)
    xidx: list = None
    parent: bool = False
    swap_levels: tuple = ()


def lists_opt(t: Tree, theta: float, parent: bool = True, swap_levels=None) -> ListsOpt:
    """Lists with the structural optimisations of Section 4: interaction via
    the parent box (``parent``) and exchanged roles at the levels in
    ``swap_levels`` (default: the finest level only, as in the paper).  An
    exchanged pair is not refined further."""
    if not (0.0 < theta < 1.0):
        raise ValueError("theta must lie in (0, 1)")
    if swap_levels is None:
        swap_levels = (t.levels,)
    swap_levels = tuple(sorted(set(int(l) for l in swap_levels)))
    lib = _load()
    z = lambda: np.zeros(0, dtype=np.int64)
    sptr, sidx = [np.array([0, 1], dtype=np.int64)], [np.array([0], dtype=np.int64)]
    wptr, widx = [np.array([0, 0], dtype=np.int64)], [z()]
    vptr, vidx = [np.array([0, 0], dtype=np.int64)], [z()]
    xptr, xidx = [np.array([0, 0], dtype=np.int64)], [z()]
    for l in range(1, t.levels + 1):
        nb = 4 ** l
        cap = 16 * int(sidx[-1].shape[0])
        arrs = [np.empty(nb + 1, dtype=np.int64) if k % 2 == 0 else np.empty(max(cap, 1), dtype=np.int64)
                for k in range(8)]
        g = np.ascontiguousarray(t.level_geom(l))
        gp = np.ascontiguousarray(t.level_geom(l - 1))
        rc = lib.orc_lists_level_opt(l, theta, int(parent), int(l in swap_levels), _p(g), _p(gp),
                                     _p(sptr[-1]), _p(sidx[-1]), *[_p(a) for a in arrs], cap)
        if rc != 0:
            raise RuntimeError("orc_lists_level_opt overflow")
        sp, si, wp, wi, vp, vi, xp, xi = arrs
        sptr.append(sp); sidx.append(si[:sp[-1]].copy())
        wptr.append(wp); widx.append(wi[:wp[-1]].copy())
        vptr.append(vp); vidx.append(vi[:vp[-1]].copy())
        xptr.append(xp); xidx.append(xi[:xp[-1]].copy())
    return ListsOpt(theta, sptr, sidx, wptr, widx, vptr, vidx, xptr, xidx, bool(parent), swap_levels)


@dataclass
class ListsRelaxed(Lists):
    theta_max: float = 0.0
    p: int = 0
    k0: int = 0
    k1: int = 0
    count: list = None   # per level: int64 [k0 + k1], candidates of each threshold bin
    kmax: list = None    # per level: last bin admitted as weak (k0 - 1 = the plain rule)


def relax_thresholds(theta: float, theta_max: float, k0: int, k1: int) -> np.ndarray:
    """The grid of thresholds on which the relaxed lists read theta_i:
    k0 steps up to theta (the last one theta itself), then k1 steps to
    theta_max, each a binary64 expression evaluated as written."""
    t = [theta * float(k + 1) / float(k0) for k in range(k0)]
    t += [theta + (theta_max - theta) * float(k + 1) / float(k1) for k in range(k1)]
    return np.array(t, dtype=np.float64)


def lists_relaxed(t: Tree, theta: float, theta_max: float, p: int, k0: int = 16,
                  k1: int = 16) -> ListsRelaxed:
    """Lists under a locally relaxed theta-criterion (Section 4, last
    paragraph): on every level the candidates whose least grid threshold
    passing Criterion 2.1 lies above theta are admitted as weak, lowest
    thresholds first, while the mean of t^(p+1) over the level's weak pairs
    stays at most theta^(p+1).  theta_max = theta gives the plain lists."""
    if not (0.0 < theta <= theta_max < 1.0):
        raise ValueError("need 0 < theta <= theta_max < 1")
    if p < 0 or k0 < 1 or k1 < 1 or k0 + k1 > 256:
        raise ValueError("need p >= 0, k0, k1 >= 1 and k0 + k1 <= 256")
    lib = _load()
    sptr = [np.array([0, 1], dtype=np.int64)]
    sidx = [np.array([0], dtype=np.int64)]
    wptr = [np.array([0, 0], dtype=np.int64)]
    widx = [np.zeros(0, dtype=np.int64)]
    count = [np.zeros(k0 + k1, dtype=np.int64)]
    kmax = [k0 - 1]
    for l in range(1, t.levels + 1):
        nb = 4 ** l
        cap = 16 * int(sidx[-1].shape[0])
        sp = np.empty(nb + 1, dtype=np.int64)
        wp = np.empty(nb + 1, dtype=np.int64)
        si = np.empty(max(cap, 1), dtype=np.int64)
        wi = np.empty(max(cap, 1), dtype=np.int64)
        cnt = np.zeros(k0 + k1, dtype=np.int64)
        km = ctypes.c_int(0)
        g = np.ascontiguousarray(t.level_geom(l))
        rc = lib.orc_lists_level_relaxed(l, theta, theta_max, p, k0, k1, _p(g), _p(sptr[-1]),
                                         _p(sidx[-1]), _p(sp), _p(si), _p(wp), _p(wi), cap,
                                         _p(cnt), ctypes.byref(km))
        if rc != 0:
            raise RuntimeError("orc_lists_level_relaxed failed: %d" % rc)
        sptr.append(sp)
        sidx.append(si[:sp[-1]].copy())
        wptr.append(wp)
        widx.append(wi[:wp[-1]].copy())
        count.append(cnt)
        kmax.append(int(km.value))
    return ListsRelaxed(theta, sptr, sidx, wptr, widx, theta_max, p, k0, k1, count, kmax)


# --------------------------------------------------------------------------
# O4: expansion operators and the whole FMM
# --------------------------------------------------------------------------
def _cplx_out(p):
    return np.zeros(2 * (p + 1), dtype=np.float64)


def _as_cplx(a):
    a = _f64(a)
    return a[0::2] + 1j * a[1::2]


def _from_cplx(c):
    c = np.asarray(c, dtype=np.complex128)
    out = np.empty(2 * c.shape[0], dtype=np.float64)
    out[0::2] = c.real
    out[1::2] = c.imag
    return out


def p2m(x, y, q, center, scale, p) -> np.ndarray:
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    A = _cplx_out(p)
    lib.orc_p2m(x.shape[0], _p(x), _p(y), _p(q), center[0], center[1], scale, p, _p(A))
    return _as_cplx(A)


def m2m(A, c_child, s_child, c_parent, s_parent) -> np.ndarray:
    lib = _load()
    p = len(A) - 1
    Ain = _from_cplx(A)
    out = _cplx_out(p)
    lib.orc_m2m(_p(Ain), c_child[0], c_child[1], s_child, c_parent[0], c_parent[1], s_parent, p, _p(out))
    return _as_cplx(out)


def m2l(A, c_src, s_src, c_tgt, s_tgt) -> np.ndarray:
    lib = _load()
    p = len(A) - 1
    Ain = _from_cplx(A)
    out = _cplx_out(p)
    lib.orc_m2l(_p(Ain), c_src[0], c_src[1], s_src, c_tgt[0], c_tgt[1], s_tgt, p, _p(out))
    return _as_cplx(out)


def l2l(B, c_parent, s_parent, c_child, s_child) -> np.ndarray:
    lib = _load()
    p = len(B) - 1
    Bin = _from_cplx(B)
    out = _cplx_out(p)
    lib.orc_l2l(_p(Bin), c_parent[0], c_parent[1], s_parent, c_child[0], c_child[1], s_child, p, _p(out))
    return _as_cplx(out)


def l2p(B, center, scale, x, y) -> np.ndarray:
    lib = _load()
    p = len(B) - 1
    Bin = _from_cplx(B)
    x, y = _f64(x), _f64(y)
    out = np.zeros(x.shape[0], dtype=np.float64)
    lib.orc_l2p(_p(Bin), center[0], center[1], scale, p, x.shape[0], _p(x), _p(y), _p(out))
    return out


def p2l(x, y, q, center, scale, p) -> np.ndarray:
    """Local expansion about (center, scale) of sources outside its ball."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    B = _cplx_out(p)
    lib.orc_p2l(x.shape[0], _p(x), _p(y), _p(q), center[0], center[1], scale, p, _p(B))
    return _as_cplx(B)


def m2p(A, center, scale, x, y) -> np.ndarray:
    lib = _load()
    p = len(A) - 1
    Ain = _from_cplx(A)
    x, y = _f64(x), _f64(y)
    out = np.zeros(x.shape[0], dtype=np.float64)
    lib.orc_m2p(_p(Ain), center[0], center[1], scale, p, x.shape[0], _p(x), _p(y), _p(out))
    return out


def fmm_eval(x, y, q, t: Tree, ls: Lists, p: int) -> np.ndarray:
    """The FMM potentials on an oracle tree and oracle lists, original order."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    L = t.levels
    wptr_off = np.zeros(L + 1, dtype=np.int64)
    widx_off = np.zeros(L + 1, dtype=np.int64)
    for l in range(1, L + 1):
        wptr_off[l] = wptr_off[l - 1] + ls.wptr[l - 1].shape[0]
        widx_off[l] = widx_off[l - 1] + ls.widx[l - 1].shape[0]
    wptr = _i64(np.concatenate(ls.wptr))
    widx = _i64(np.concatenate(ls.widx)) if sum(w.shape[0] for w in ls.widx) else np.zeros(1, np.int64)
    geom = _f64(t.geom)
    phi = np.empty(x.shape[0], dtype=np.float64)
    rc = lib.orc_fmm_eval(x.shape[0], _p(x), _p(y), _p(q), L, p, _p(_i64(t.perm)),
                          _p(_i64(t.leaf_start)), _p(geom), _p(wptr), _p(widx),
                          _p(wptr_off), _p(widx_off), _p(_i64(ls.sptr[L])),
                          _p(_i64(ls.sidx[L]) if ls.sidx[L].shape[0] else np.zeros(1, np.int64)),
                          _p(phi))
    if rc != 0:
        raise RuntimeError("orc_fmm_eval failed: %d" % rc)
    return phi


def _concat(per_level):
    L = len(per_level) - 1
    off = np.zeros(L + 1, dtype=np.int64)
    for l in range(1, L + 1):
        off[l] = off[l - 1] + per_level[l - 1].shape[0]
    cat = np.concatenate(per_level) if sum(a.shape[0] for a in per_level) else np.zeros(1, np.int64)
    return _i64(cat), off


def fmm_eval_opt(x, y, q, t: Tree, ls: ListsOpt, p: int) -> np.ndarray:
    """The FMM potentials with the optimised lists (V via the parent, X with
    exchanged roles), original order."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    L = t.levels
    wptr, wptr_off = _concat(ls.wptr)
    widx, widx_off = _concat(ls.widx)
    vptr, vptr_off = _concat(ls.vptr)
    vidx, vidx_off = _concat(ls.vidx)
    xptr, xptr_off = _concat(ls.xptr)
    xidx, xidx_off = _concat(ls.xidx)
    geom = _f64(t.geom)
    phi = np.empty(x.shape[0], dtype=np.float64)
    rc = lib.orc_fmm_eval_opt(x.shape[0], _p(x), _p(y), _p(q), L, p, _p(_i64(t.perm)),
                              _p(_i64(t.leaf_start)), _p(geom), _p(wptr), _p(widx),
                              _p(wptr_off), _p(widx_off), _p(_i64(ls.sptr[L])),
                              _p(_i64(ls.sidx[L]) if ls.sidx[L].shape[0] else np.zeros(1, np.int64)),
                              _p(vptr), _p(vidx), _p(vptr_off), _p(vidx_off),
                              _p(xptr), _p(xidx), _p(xptr_off), _p(xidx_off), _p(phi))
    if rc != 0:
        raise RuntimeError("orc_fmm_eval_opt failed: %d" % rc)
    return phi


def fmm(x, y, q, levels: int, p: int, theta: float) -> np.ndarray:
    """Tree, lists and evaluation in one call."""
    t = tree(x, y, levels)
    return fmm_eval(x, y, q, t, lists(t, theta), p)


def fmm_field(x, y, q, levels: int, p: int, theta: float):
    """(phi, d phi/dx, d phi/dy) by the FMM: as fmm(), and at the leaves the
    derivative of the local expansion plus the direct gradient over the
    strong list.  Original order."""
    lib = _load()
    x, y, q = _f64(x), _f64(y), _f64(q)
    t = tree(x, y, levels)
    ls = lists(t, theta)
    L = t.levels
    wptr_off = np.zeros(L + 1, dtype=np.int64)
    widx_off = np.zeros(L + 1, dtype=np.int64)
    for l in range(1, L + 1):
        wptr_off[l] = wptr_off[l - 1] + ls.wptr[l - 1].shape[0]
        widx_off[l] = widx_off[l - 1] + ls.widx[l - 1].shape[0]
    wptr = _i64(np.concatenate(ls.wptr))
    widx = _i64(np.concatenate(ls.widx)) if sum(w.shape[0] for w in ls.widx) else np.zeros(1, np.int64)
    geom = _f64(t.geom)
    n = x.shape[0]
    phi, gx, gy = (np.empty(n, dtype=np.float64) for _ in range(3))
    rc = lib.orc_fmm_eval_field(n, _p(x), _p(y), _p(q), L, p, _p(_i64(t.perm)),
                                _p(_i64(t.leaf_start)), _p(geom), _p(wptr), _p(widx),
                                _p(wptr_off), _p(widx_off), _p(_i64(ls.sptr[L])),
                                _p(_i64(ls.sidx[L]) if ls.sidx[L].shape[0] else np.zeros(1, np.int64)),
                                _p(phi), _p(gx), _p(gy))
    if rc != 0:
        raise RuntimeError("orc_fmm_eval_field failed: %d" % rc)
    return phi, gx, gy


# --------------------------------------------------------------------------
# O5: error metric (normwise, as the relative errors of Section 5)
# --------------------------------------------------------------------------
def rel_errors(approx, exact):
    """(e_inf, e_2): max|a - e| / max|e| and ||a - e||_2 / ||e||_2."""
    a = np.asarray(approx, dtype=np.float64)
    e = np.asarray(exact, dtype=np.float64)
    d = np.abs(a - e)
    einf = float(d.max() / np.abs(e).max()) if e.size else 0.0
    e2 = float(np.linalg.norm(a - e) / np.linalg.norm(e)) if e.size else 0.0
    return einf, e2


# --------------------------------------------------------------------------
# O6: a-priori parameter choice (Section 3 estimate, Section 4 defaults)
# --------------------------------------------------------------------------
def a_priori(n: int, tol: float, k_const: float, theta: float = 0.5,
             per_leaf: float = 20.0):
    """(levels, p, theta): theta = 1/2, about `per_leaf` sources per leaf, and
    the least p with k_const * theta^(p+1) / (1-theta)^2 <= tol."""
    lmax = int(math.floor(math.log(n, 4) + 1e-12))
    # round half up (Python's round() would round half to even)
    levels = int(math.floor(math.log(max(n / per_leaf, 1.0)) / math.log(4.0) + 0.5))
    levels = max(1, min(levels, lmax, 13))
    p = 1
    while k_const * theta ** (p + 1) / (1.0 - theta) ** 2 > tol and p < 63:
        p += 1
    return levels, p, theta
