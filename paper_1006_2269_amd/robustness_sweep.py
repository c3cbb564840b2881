"""Time of the whole path versus N for three layouts at TOL = 1e-6 (needs the
GPU): the shape of Section 5's third experiment (uniform in the unit square,
and the 'normal' and 'layer' layouts of the second, sigma = 0.1).

Per layout and N: (1) the library's reduced form: fmm2d_select_build_tree
(the learned selector; outside its trained range of N the a-priori rule) +
connectivity + evaluate in FP32_ACC64; (2) plain binary64 at the rule's
(levels, p, theta).  Time = median of 3 runs after a warm-up (HIP events on
the library stream), error e_inf against the binary64 direct sum at 1000
sampled targets.

    python -m paper_1006_2269_amd.robustness_sweep --out gpurun_out/robust.json
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

SIZES = (10_000, 30_000, 100_000, 300_000, 1_000_000, 2_000_000, 5_000_000)
TOL = 1e-6


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--sizes", default=",".join(str(s) for s in SIZES))
    args = ap.parse_args()
    import torch

    from paper_1006_2269_amd import selector
    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2D

    f = FMM2D(0)
    dev = f.device
    wts = selector.weights_tensor(dev)
    makers = {"uniform": lambda n, s: W.uniform(n, s), "normal": W.normal_corner, "layer": W.layer}
    rows = []

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(f.stream)
            r = fn()
            b.record(f.stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
        return r, float(np.median(ts))

    for name, mk in makers.items():
        for n in (int(s) for s in args.sizes.split(",")):
            ps = mk(n, 7000 + n % 997)
            x, y, q = (torch.from_numpy(a).to(dev) for a in (ps.x, ps.y, ps.q))
            tg = torch.from_numpy(W.sample_targets(ps.n, 1000, seed=4242)).to(dev)
            exact = f.direct(x, y, q, tg)
            scale = float(exact.abs().max())
            out = torch.empty_like(q)

            def reduced():
                L, p, th, net = f.select_build_tree(x, y, TOL, wts)
                f.connectivity(th)
                f.evaluate(q, p, "fp32_acc64", out=out)
                return L, p, th, net

            (L, p, th, net), ms = timed(reduced)
            e = float((out[tg] - exact).abs().max()) / scale
            rec = {"layout": name, "n": n, "reduced": {"levels": L, "p": p, "theta": th, "network": net, "ms": ms,
                                                       "e_inf": e}}
            Lr, pr, thr, _ = f.select(x, y, TOL)  # the rule (no weights)

            def plain():
                f.build_tree(x, y, Lr)
                f.connectivity(thr)
                f.evaluate(q, pr, "fp64", out=out)

            _, ms64 = timed(plain)
            e64 = float((out[tg] - exact).abs().max()) / scale
            rec["fp64_rule"] = {"levels": Lr, "p": pr, "theta": thr, "ms": ms64, "e_inf": e64}
            rows.append(rec)
            print("[robust] %-7s n=%8d  reduced (L=%d p=%d th=%.2f net=%d) %.2f ms e=%.1e | fp64 rule (L=%d p=%d) "
                  "%.2f ms e=%.1e" % (name, n, L, p, th, net, ms, e, Lr, pr, ms64, e64), flush=True)
    with open(args.out, "w") as fh:
        json.dump({"tol": TOL, "rows": rows}, fh, indent=1)
    f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
