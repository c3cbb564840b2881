"""Pins of the oracle's direct sum, the interaction sum (1.1) with charges and
G = log|x - y|.  Each check uses a fact that does not come from the oracle's
own formula: a closed form, a 40-digit brute force, or an exact identity."""
import math

import mpmath
import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W


@pytest.mark.parametrize("n,rho,c", [(3, 1.0, (0.0, 0.0)), (17, 0.7, (0.3, -0.2)),
                                     (64, 2.5, (-4.0, 1e3)), (101, 1e-3, (0.5, 0.5))])
def test_regular_polygon_closed_form(orc, n, rho, c):
    # prod_{k=1}^{n-1} |1 - w^k| = n for w = exp(2 pi i / n), so with unit
    # charges every vertex has Phi = log n + (n - 1) log rho.
    ang = 2.0 * np.pi * np.arange(n) / n
    x = c[0] + rho * np.cos(ang)
    y = c[1] + rho * np.sin(ang)
    phi = orc.direct(x, y, np.ones(n))
    exact = math.log(n) + (n - 1) * math.log(rho)
    assert np.abs(phi - exact).max() <= 1e-12 * max(1.0, abs(exact)) * n


def test_two_points(orc):
    x = np.array([0.25, -1.5])
    y = np.array([3.0, 0.5])
    q = np.array([0.7, -2.0])
    phi = orc.direct(x, y, q)
    d = math.hypot(0.25 + 1.5, 3.0 - 0.5)
    assert phi[0] == pytest.approx(-2.0 * math.log(d), rel=1e-15)
    assert phi[1] == pytest.approx(0.7 * math.log(d), rel=1e-15)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_brute_force_40_digits(orc, seed):
    g = np.random.Generator(np.random.PCG64(seed))
    n = 48
    x = g.normal(size=n) * 10.0 ** g.uniform(-3, 2, n)
    y = g.normal(size=n) * 10.0 ** g.uniform(-3, 2, n)
    q = g.uniform(-1, 1, n)
    phi = orc.direct(x, y, q)
    mpmath.mp.dps = 40
    for i in range(n):
        s = mpmath.mpf(0)
        for j in range(n):
            if j == i:
                continue
            dx = mpmath.mpf(x[i]) - mpmath.mpf(x[j])
            dy = mpmath.mpf(y[i]) - mpmath.mpf(y[j])
            s += mpmath.mpf(q[j]) * mpmath.log(mpmath.sqrt(dx * dx + dy * dy))
        assert abs(phi[i] - float(s)) <= 4e-16 * max(1.0, sum(abs(q) * 8))


def test_coincident_points_contribute_nothing(orc):
    # Reading of (1.1) for distinct points at one location: those pairs are
    # left out, like j == i itself.
    x = np.array([0.0, 0.0, 1.0])
    y = np.array([0.0, 0.0, 0.0])
    q = np.array([1.0, 5.0, 2.0])
    phi = orc.direct(x, y, q)
    assert phi[0] == 0.0 and phi[1] == 0.0
    assert phi[2] == 0.0  # log 1 = 0 from both
    x[2] = 2.0
    phi = orc.direct(x, y, q)
    assert phi[0] == pytest.approx(2.0 * math.log(2.0))
    assert phi[2] == pytest.approx(6.0 * math.log(2.0))


def test_scaling_translation_rotation(orc):
    ps = W.uniform(500, seed=11)
    base = orc.direct(ps.x, ps.y, ps.q)
    s = 3.7
    scaled = orc.direct(s * ps.x, s * ps.y, ps.q)
    qsum_others = ps.q.sum() - ps.q
    assert np.abs(scaled - (base + math.log(s) * qsum_others)).max() <= 1e-12 * np.abs(base).max()
    a = 0.6
    xr = math.cos(a) * ps.x - math.sin(a) * ps.y + 0.37
    yr = math.sin(a) * ps.x + math.cos(a) * ps.y - 1.2
    rot = orc.direct(xr, yr, ps.q)
    assert np.abs(rot - base).max() <= 1e-12 * np.abs(base).max()


def test_linear_in_charges(orc):
    ps = W.uniform(300, seed=5)
    q2 = np.random.Generator(np.random.PCG64(9)).uniform(-1, 1, ps.n)
    a = orc.direct(ps.x, ps.y, ps.q)
    b = orc.direct(ps.x, ps.y, q2)
    c = orc.direct(ps.x, ps.y, 2.0 * ps.q - 3.0 * q2)
    assert np.abs(c - (2.0 * a - 3.0 * b)).max() <= 1e-12 * np.abs(c).max()


def test_target_subset_matches_full(orc):
    ps = W.uniform(400, seed=8)
    full = orc.direct(ps.x, ps.y, ps.q)
    t = W.sample_targets(ps.n, 37, seed=3)
    part = orc.direct(ps.x, ps.y, ps.q, t)
    assert np.array_equal(part, full[t])
