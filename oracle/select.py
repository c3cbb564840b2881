"""Selector features and decision rules -- TEST INFRASTRUCTURE ONLY.

Plain numpy reference of what the GPU library's parameter selection computes
(only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package).

* ``features``      -- density features of a point set: log10 N, log10 TOL,
                       and for each level l = 1..10 of a uniform 2^l x 2^l
                       grid over the tight bounding box the occupied-cell
                       fraction and an 8-bin histogram of the points by the
                       relative density count 4^l / N of their cell, the
                       cells counted over every ceil(N / 2^18)-th point (all
                       points when N <= 2^18; N then means the sample size
                       in the densities and fractions).  The
                       paper fixes no features; these describe the spread of
                       box sizes of the median-split pyramid (Section 4),
                       whose boxes shrink where points crowd.  Parity
                       unpinned against the paper; pinned by brute force and
                       closed forms.
* ``rule``          -- the a-priori choice of (levels, p, theta): theta = 1/2
                       and about 20 points per leaf (the practical choice at
                       the end of Section 4), p the least order meeting the
                       truncation bound of Section 3 with constant 0.1.
* ``decide``        -- the mapping from the network's three raw outputs to
                       (levels, p, theta).  The network's targets are an
                       encoding chosen here: levels - round(log4(N/16)),
                       log10 C of the error model C theta^(p+1) (the form of
                       the truncation bound of Section 3), and theta; p is
                       the least order the model says meets TOL / 2.
                       The paper has no learned selector, so this is parity
                       unpinned against the paper.
"""
from __future__ import annotations

import math

import numpy as np

FL = 10
NFEAT = 2 + 9 * FL
HEADER = 194
THETAS = (0.35, 0.45, 0.55, 0.65, 0.75)
MAX_LEVELS = 13
MAX_P = 63
SAFETY_LOG10 = 0.30102999566398120  # log10(2)


def round_half_up(v: float) -> int:
    return int(math.floor(v + 0.5))


def finest_cells(x, y):
    """Level-10 cell of every point: floor((v - min) 2^10 / extent), clamped."""
    x = np.asarray(x, dtype=np.float64) + 0.0
    y = np.asarray(y, dtype=np.float64) + 0.0
    out = []
    for v in (x, y):
        lo, hi = float(v.min()), float(v.max())
        ext = hi - lo
        s = (1 << FL) / ext if ext > 0.0 else 0.0
        t = (v - lo) * s
        t = np.where(t >= 0.0, t, 0.0)
        t = np.where(t < float(1 << FL), t, float((1 << FL) - 1))
        out.append(t.astype(np.int64))
    return out[0], out[1]


def density_class(count: np.ndarray, n: int, level: int) -> np.ndarray:
    """Number of edges 2^-3 .. 2^3 that are <= count 4^level / n (exact)."""
    lhs = count.astype(np.int64) << (2 * level + 4)
    k = np.zeros(count.shape, dtype=np.int64)
    for j in range(1, 8):
        k += lhs >= (np.int64(n) << j)
    return k


SAMPLE_MAX = 1 << 18


def sample_stride(n: int) -> int:
    """Cells are counted over every stride-th point (at most 2^18 points)."""
    return -(-n // SAMPLE_MAX) if n > SAMPLE_MAX else 1


def features(x, y, tol: float) -> np.ndarray:
    n = len(x)
    ix, iy = finest_cells(x, y)          # bounding box of all points
    stride = sample_stride(n)
    ix, iy = ix[::stride], iy[::stride]
    ns = len(ix)
    f = np.zeros(NFEAT, dtype=np.float64)
    f[0] = math.log10(n)
    f[1] = math.log10(tol)
    for l in range(1, FL + 1):
        sh = FL - l
        cell = (iy >> sh) * (1 << l) + (ix >> sh)
        counts = np.bincount(cell, minlength=1 << (2 * l))
        occ = counts[counts > 0]
        base = 2 + 9 * (l - 1)
        f[base] = occ.size / float(4 ** l)
        cls = density_class(occ, ns, l)
        for k in range(8):
            f[base + 1 + k] = float(occ[cls == k].sum()) / float(ns)
    return f.astype(np.float32)


def levels_max(n: int) -> int:
    lmax = 0
    while lmax < MAX_LEVELS and 4 ** (lmax + 1) <= n:
        lmax += 1
    return lmax


def rule(n: int, tol: float, k_const: float = 0.1):
    theta = 0.5
    L = round_half_up(math.log(max(n / 20.0, 1.0)) / math.log(4.0))
    L = max(1, min(L, levels_max(n)))
    p = 1
    while k_const * theta ** (p + 1) / (1.0 - theta) ** 2 > tol and p < MAX_P:
        p += 1
    return L, p, theta


def decide(out3, blob, n: int, tol: float):
    """(levels, p, theta, from_network) from raw network outputs out3."""
    blob = np.asarray(blob, dtype=np.float32)
    ln, lt = math.log10(n), math.log10(tol)
    r = blob[2 * NFEAT + 6: 2 * NFEAT + 10].astype(np.float64)
    inside = r[0] <= ln <= r[1] and r[2] <= lt <= r[3]
    mean = blob[2 * NFEAT: 2 * NFEAT + 3].astype(np.float64)
    std = blob[2 * NFEAT + 3: 2 * NFEAT + 6].astype(np.float64)
    dl, lc, th = (float(np.float64(out3[i]) * std[i] + mean[i]) for i in range(3))
    ok = inside and all(math.isfinite(v) for v in (dl, lc, th)) and abs(dl) < 64.0 and abs(lc) < 1e4
    if not ok:
        L, p, theta = rule(n, tol)
        return L, p, theta, False
    # dl is the level count's offset from log4(N / 16)
    L = max(1, min(round_half_up(math.log(max(n / 16.0, 1.0)) / math.log(4.0) + dl), levels_max(n)))
    g = max(0, min(round_half_up((th - 0.35) / 0.1), 4))
    theta = THETAS[g]
    # error model e(p) = C theta^(p+1) with a safety factor of 2 on the
    # error: the least p with C theta^(p+1) <= tol / 2
    q = math.ceil((lt - SAFETY_LOG10 - lc) / math.log10(theta)) - 1
    p = max(1, min(q, MAX_P))
    return L, p, theta, True
