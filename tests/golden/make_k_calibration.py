"""Writes ``k_calibration.json``: the constant K of the a-priori error model
K * theta^(p+1) / (1 - theta)^2 (the truncation estimate of Section 3, used as
a model with a calibrated constant), computed with the CPU oracle only.

For each calibration layout (10,000 points, 5 levels of median splits, the
size of the smallest benchmark configuration), each theta in
{0.25, 0.5, sqrt(1/2)} (the values of Section 5's error-vs-p experiment) and
each p = 4..30, the oracle FMM is compared with the oracle direct sum, and
the observed constant e_inf * (1 - theta)^2 / theta^(p+1) is recorded.
Errors below 1e-13 sit on the binary64 rounding floor and say nothing about
truncation; they are left out.  K is twice the largest observed constant.

Run:  python tests/golden/make_k_calibration.py
"""
import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1006_2269_amd import workloads as W  # noqa: E402

FLOOR = 1e-13
THETAS = (0.25, 0.5, math.sqrt(0.5))
ORDERS = tuple(range(4, 31))
LEVELS = 5
LAYOUTS = {
    "uniform_10k": lambda: W.uniform_10k(),
    "disc_uniform_10k": lambda: W.unit_disc(10000, 5, radial_inverse=False),
    "disc_1r_10k": lambda: W.unit_disc(10000, 6, radial_inverse=True),
    "mixture_10k": lambda: W.random_mixture(10000, 8),
}


def observed_constants(name, orders=ORDERS, thetas=THETAS):
    ps = LAYOUTS[name]()
    ex = oracle.direct(ps.x, ps.y, ps.q)
    t = oracle.tree(ps.x, ps.y, LEVELS)
    rows = []
    for theta in thetas:
        ls = oracle.lists(t, theta)
        for p in orders:
            e, _ = oracle.rel_errors(oracle.fmm_eval(ps.x, ps.y, ps.q, t, ls, p), ex)
            const = e * (1.0 - theta) ** 2 / theta ** (p + 1)
            rows.append({"theta": theta, "p": p, "e_inf": e, "const": const if e >= FLOOR else None})
    return rows


def main():
    out = {"what": "K = 2 x max over the table of e_inf (1-theta)^2 / theta^(p+1), e_inf >= %g" % FLOOR,
           "levels": LEVELS, "floor": FLOOR, "layouts": {}}
    worst = 0.0
    for name in LAYOUTS:
        rows = observed_constants(name)
        out["layouts"][name] = rows
        worst = max([worst] + [r["const"] for r in rows if r["const"] is not None])
        print(name, "max const %.4g" % max(r["const"] for r in rows if r["const"] is not None), flush=True)
    out["max_observed"] = worst
    out["K"] = 2.0 * worst
    with open(os.path.join(HERE, "k_calibration.json"), "w") as f:
        json.dump(out, f, indent=1)
    print("K = %.4g (max observed %.4g)" % (2.0 * worst, worst))


if __name__ == "__main__":
    main()
