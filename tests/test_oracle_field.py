"""Pins of the oracle's field (the gradient of the potential): against
central differences of the potential, a symmetry that makes it vanish, the
derivative of the local expansion against differences of the expansion itself,
and the FMM field converging to the direct one as the order grows."""
import math

import numpy as np

import oracle
from paper_1006_2269_amd import workloads as W


def _with_probes(x, y, q, i, h):
    # point i's charge removed (the gradient at i excludes i itself) and four
    # charge-free probes at z_i +- h, z_i +- ih: the potential there is the
    # sum over the other points
    px = np.concatenate([x, [x[i] + h, x[i] - h, x[i], x[i]]])
    py = np.concatenate([y, [y[i], y[i], y[i] + h, y[i] - h]])
    pq = np.concatenate([q, np.zeros(4)])
    pq[i] = 0.0
    n = x.shape[0]
    return px, py, pq, np.arange(n, n + 4)


def test_direct_field_is_the_gradient_of_the_potential():
    ps = W.uniform(500, 31)
    rng = np.random.default_rng(5)
    idx = rng.choice(ps.n, 12, replace=False)
    gx, gy = oracle.direct_field(ps.x, ps.y, ps.q, idx)
    h = 1e-5
    for t, i in enumerate(idx):
        px, py, pq, probes = _with_probes(ps.x, ps.y, ps.q, i, h)
        f = oracle.direct(px, py, pq, probes)
        dx = (f[0] - f[1]) / (2 * h)
        dy = (f[2] - f[3]) / (2 * h)
        scale = max(abs(gx[t]), abs(gy[t]), 1.0)
        assert abs(dx - gx[t]) <= 1e-5 * scale, (i, dx, gx[t])
        assert abs(dy - gy[t]) <= 1e-5 * scale, (i, dy, gy[t])


def test_field_of_a_ring_of_charges():
    # m equal charges evenly on a circle of radius R about c: the sum of
    # log|z - z_k| is log|(z - c)^m - R^m| (the z_k are the m-th roots), so
    # inside the gradient is O((r/R)^(m-1)) and outside it is the field of
    # the total charge at c up to O((R/r)^(m+1))
    m, R, c = 64, 0.2, (0.3, 0.4)
    ang = 2 * math.pi * np.arange(m) / m
    probes_x = np.array([0.3, 0.33, 0.27, 0.62])   # three inside (r <= 0.03), one outside (r = 0.32)
    probes_y = np.array([0.4, 0.4, 0.42, 0.4])
    x = np.concatenate([c[0] + R * np.cos(ang), probes_x])
    y = np.concatenate([c[1] + R * np.sin(ang), probes_y])
    q = np.concatenate([np.ones(m), np.zeros(4)])
    gx, gy = oracle.direct_field(x, y, q, np.arange(m, m + 4))
    bound = 1e-12 * m / R
    assert np.all(np.abs(gx[:3]) <= bound) and np.all(np.abs(gy[:3]) <= bound), (gx, gy)
    dx, dy = probes_x[3] - c[0], probes_y[3] - c[1]
    r2 = dx * dx + dy * dy
    assert abs(gx[3] - m * dx / r2) <= 1e-12 * m / math.sqrt(r2)
    assert abs(gy[3] - m * dy / r2) <= 1e-12 * m / math.sqrt(r2)


def test_local_expansion_gradient_against_differences():
    rng = np.random.default_rng(11)
    p = 12
    B = rng.normal(size=2 * (p + 1)) * (0.6 ** np.repeat(np.arange(p + 1), 2))
    c, s = (0.5, 0.25), 0.3
    lib = oracle._load()
    x = 0.5 + 0.1 * rng.uniform(-1, 1, 6)
    y = 0.25 + 0.1 * rng.uniform(-1, 1, 6)
    gx, gy = np.zeros(6), np.zeros(6)
    lib.orc_l2p_grad(oracle._p(oracle._f64(B)), c[0], c[1], s, p, 6, oracle._p(oracle._f64(x)),
                     oracle._p(oracle._f64(y)), oracle._p(gx), oracle._p(gy))

    def pot(xx, yy):
        out = np.zeros(xx.shape[0])
        lib.orc_l2p(oracle._p(oracle._f64(B)), c[0], c[1], s, p, xx.shape[0], oracle._p(oracle._f64(xx)),
                    oracle._p(oracle._f64(yy)), oracle._p(out))
        return out

    h = 1e-6
    dx = (pot(x + h, y) - pot(x - h, y)) / (2 * h)
    dy = (pot(x, y + h) - pot(x, y - h)) / (2 * h)
    np.testing.assert_allclose(gx, dx, rtol=0, atol=1e-7 * np.abs(dx).max())
    np.testing.assert_allclose(gy, dy, rtol=0, atol=1e-7 * np.abs(dy).max())


def test_fmm_field_converges_to_the_direct_field():
    ps = W.clustered_10m(scale=0.0003)  # 3000 clustered points
    ex, ey = oracle.direct_field(ps.x, ps.y, ps.q)
    scale = max(np.abs(ex).max(), np.abs(ey).max())
    errs = []
    for p in (6, 12, 24):
        phi, gx, gy = oracle.fmm_field(ps.x, ps.y, ps.q, 3, p, 0.5)
        errs.append(max(np.abs(gx - ex).max(), np.abs(gy - ey).max()) / scale)
        # the potential is the one the potential-only FMM gives
        np.testing.assert_array_equal(phi, oracle.fmm(ps.x, ps.y, ps.q, 3, p, 0.5))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] <= 1e-8, errs
