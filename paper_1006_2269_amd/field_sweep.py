"""Relative error of the FMM field (the gradient of the potential) against
the direct field, versus the expansion order, for several theta (needs the
GPU): the shape of Section 5's first experiment, here for the logarithmic
kernel's gradient q_j (z_i - z_j)/|z_i - z_j|^2 (the complex conjugate of the
force kernel q_j/(z_i - z_j) of that experiment, so the same magnitudes).

10^6 points of total mass 1 in the unit disc, uniform density and radial
density proportional to 1/r (``workloads.unit_disc``); theta in {0.25, 0.5,
sqrt(1/2)}; about 20 points per leaf (8 levels); error measured at M = 1000
sampled targets as max_i |g_i - g~_i| / max_i |g~_i| with g = (gx, gy) and the
binary64 direct sum g~ (fmm2d_direct_field).  Also the time of one
fmm2d_evaluate_field (HIP events on the library stream).

    python -m paper_1006_2269_amd.field_sweep --out gpurun_out/field_sweep.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

THETAS = (0.25, 0.5, math.sqrt(0.5))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--pmax", type=int, default=30)
    ap.add_argument("--samples", type=int, default=1000)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import torch

    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2D

    f = FMM2D(0)
    dev = f.device
    rows = []
    for radial in (False, True):
        ps = W.unit_disc(args.n, 501 + int(radial), radial_inverse=radial)
        x, y, q = (torch.from_numpy(a).to(dev) for a in (ps.x, ps.y, ps.q))
        tg = torch.from_numpy(W.sample_targets(ps.n, args.samples, seed=4242)).to(dev)
        ex, ey = (a.cpu().numpy() for a in f.direct_field(x, y, q, tg))
        emag = np.hypot(ex, ey).max()
        f.build_tree(x, y, args.levels)
        for th in THETAS:
            f.connectivity(th)
            for p in range(2, args.pmax + 1, 2):
                f.evaluate_field(q, p)  # warm (allocations)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(f.stream)
                phi, gx, gy = f.evaluate_field(q, p)
                b.record(f.stream)
                b.synchronize()
                ms = a.elapsed_time(b)
                gxs, gys = gx[tg].cpu().numpy(), gy[tg].cpu().numpy()
                err = float(np.hypot(gxs - ex, gys - ey).max() / emag)
                rows.append({"layout": ps.name, "theta": th, "p": p, "e_inf": err, "ms": ms})
                print("[field] %s theta=%.3f p=%2d  e_inf=%.3e  %.2f ms" % (ps.name, th, p, err, ms), flush=True)
    with open(args.out, "w") as fh:
        json.dump({"n": args.n, "levels": args.levels, "samples": args.samples, "rows": rows}, fh, indent=1)
    f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
