"""Pins of the error metric and of the calibrated constant of the a-priori
error model.

* ``rel_errors`` is the normwise relative error of Section 5 (maximum norm and
  2-norm), checked against values worked out by hand on fixed vectors, with
  cases that tell apart the plausible mistakes: e_inf and e_2 swapped, a
  division by max|approx| instead of max|exact|, a pointwise instead of a
  normwise ratio, a missing absolute value.
* ``k_calibration.json`` (written by ``golden/make_k_calibration.py`` from
  the oracle alone) records the constant of K theta^(p+1) / (1-theta)^2
  (Section 3): the shipped constant must not be below it, and a slice of
  the table must come out the same when recomputed.
"""
import json
import math
import os
import sys

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_rel_errors_hand_values(orc):
    # d = (0, 0.5, 0.5): e_inf = 0.5 / 3, e_2 = sqrt(0.5) / sqrt(1 + 6.25 + 9)
    e_inf, e_2 = orc.rel_errors([1.0, 2.0, 3.5], [1.0, 2.5, 3.0])
    assert e_inf == pytest.approx(1.0 / 6.0, rel=1e-15)
    assert e_2 == pytest.approx(math.sqrt(0.5) / math.sqrt(16.25), rel=1e-15)


def test_rel_errors_normwise_not_pointwise(orc):
    # the largest pointwise ratio is 1 (at the 1e-3 entry); normwise it is 1e-3 / 4
    e_inf, e_2 = orc.rel_errors([-4.0, 2e-3, 1.0], [-4.0, 1e-3, 1.0])
    assert e_inf == pytest.approx(1e-3 / 4.0, rel=1e-13)
    assert e_2 == pytest.approx(1e-3 / math.sqrt(16.0 + 1e-6 + 1.0), rel=1e-13)


def test_rel_errors_divides_by_exact(orc):
    # max|approx| = 10, max|exact| = 5: the error is relative to the exact values
    e_inf, _ = orc.rel_errors([10.0, -1.0], [5.0, -1.0])
    assert e_inf == pytest.approx(1.0, rel=1e-15)
    e_inf, _ = orc.rel_errors([-3.0, 1.0], [-4.0, 1.0])  # signs: |a - e| and |e|
    assert e_inf == pytest.approx(0.25, rel=1e-15)


def test_rel_errors_inf_below_two_norm_bound(orc):
    g = np.random.Generator(np.random.PCG64(3))
    e = g.normal(size=1000)
    a = e + 1e-6 * g.normal(size=1000)
    e_inf, e_2 = orc.rel_errors(a, e)
    assert e_inf == pytest.approx(np.abs(a - e).max() / np.abs(e).max(), rel=1e-14)
    assert e_2 == pytest.approx(math.sqrt(np.sum((a - e) ** 2) / np.sum(e ** 2)), rel=1e-12)
    assert orc.rel_errors(e, e) == (0.0, 0.0)


def _table():
    with open(os.path.join(GOLDEN, "k_calibration.json")) as f:
        return json.load(f)


def test_k_calibration_recorded_and_below_shipped_constant():
    tab = _table()
    consts = [r["const"] for rows in tab["layouts"].values() for r in rows if r["const"] is not None]
    assert len(consts) > 100
    assert tab["max_observed"] == max(consts)
    assert tab["K"] == 2.0 * tab["max_observed"]
    # the constant the rule ships with (oracle, GPU selector) is at least the calibrated one
    assert 0.1 >= tab["K"]


def test_k_calibration_reproducible(orc):
    sys.path.insert(0, GOLDEN)
    try:
        import make_k_calibration as mk
    finally:
        sys.path.remove(GOLDEN)
    tab = _table()
    rows = mk.observed_constants("mixture_10k", orders=(6, 12), thetas=(0.5,))
    stored = {(r["theta"], r["p"]): r for r in tab["layouts"]["mixture_10k"]}
    for r in rows:
        s = stored[(r["theta"], r["p"])]
        assert r["e_inf"] == pytest.approx(s["e_inf"], rel=1e-12)
