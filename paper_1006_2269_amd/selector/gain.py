"""Held-out comparison of the learned selector with the a-priori rule (needs
the GPU).

For each held-out layout (``workloads.selector_layout`` with seeds disjoint
from training, N = 10^U[lo, hi]) and TOL (default 1e-6): both forms run the
whole path -- select, build_tree, connectivity (the lists with
``selector.LIST_OPTIONS``), evaluate (``selector.reduced_mode(TOL)``) --
timed with HIP events on the library's stream after one warm-up, and their
normwise error is measured against the binary64 judge at 1000 sampled
targets.  A form counts on a layout only where it meets TOL: the summary
gives each form's fraction meeting TOL and the speed-up over the layouts
where both do.

    python -m paper_1006_2269_amd.selector.gain --first 90000 --count 40 --out gpurun_out/gain.json
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

def timed_path(f, torch, x, y, q, tol, weights, out, reps=3):
    from paper_1006_2269_amd.selector import LIST_OPTIONS, reduced_mode

    mode = reduced_mode(tol)

    def once():
        L, p, th, net = f.select(x, y, tol, weights)
        f.build_tree(x, y, L)
        f.connectivity(th, **LIST_OPTIONS)
        f.evaluate(q, p, mode, out=out)
        return L, p, th, net

    once()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(f.stream)
        cfg = once()
        b.record(f.stream)
        b.synchronize()
        ts.append(a.elapsed_time(b))
    return cfg, float(np.median(ts))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--first", type=int, default=90000)
    ap.add_argument("--count", type=int, default=40)
    ap.add_argument("--lo", type=float, default=4.0)
    ap.add_argument("--hi", type=float, default=7.0)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--out", required=True)
    args = ap.parse_args()
    import torch

    from paper_1006_2269_amd import selector
    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2D

    f = FMM2D(0)
    dev = f.device
    wts = selector.weights_tensor(dev)
    if wts is None:
        print("no trained weights at %s" % selector.WEIGHTS_PATH, file=sys.stderr)
        return 2
    rows = []
    for i in range(args.count):
        ps = W.selector_layout(args.first + i, args.lo, args.hi)
        x = torch.from_numpy(ps.x).to(dev)
        y = torch.from_numpy(ps.y).to(dev)
        q = torch.from_numpy(ps.q).to(dev)
        tg = torch.from_numpy(W.sample_targets(ps.n, 1000, seed=4242)).to(dev)
        exact = f.direct(x, y, q, tg)
        scale = float(exact.abs().max())
        out = torch.empty_like(q)
        rec = {"seed": args.first + i, "n": ps.n}
        for form, w in (("learned", wts), ("rule", None)):
            (L, p, th, net), ms = timed_path(f, torch, x, y, q, args.tol, w, out)
            e = float((out[tg] - exact).abs().max()) / scale
            rec[form] = {"levels": L, "p": p, "theta": th, "network": net, "ms": ms, "e_inf": e,
                         "ok": e <= args.tol}
        rows.append(rec)
        print("[gain] %d n=%d learned (L=%d p=%d th=%.2f) %.2f ms e=%.1e | rule (L=%d p=%d) %.2f ms e=%.1e"
              % (i, ps.n, rec["learned"]["levels"], rec["learned"]["p"], rec["learned"]["theta"],
                 rec["learned"]["ms"], rec["learned"]["e_inf"], rec["rule"]["levels"], rec["rule"]["p"],
                 rec["rule"]["ms"], rec["rule"]["e_inf"]), flush=True)
    summ = {}
    for form in ("learned", "rule"):
        ok = [r[form]["ok"] for r in rows]
        tot_ms = sum(r[form]["ms"] for r in rows)
        summ[form] = {"fraction_meeting_tol": float(np.mean(ok)),
                      "points_per_s_total": float(sum(r["n"] for r in rows) / (tot_ms * 1e-3)),
                      "median_points_per_s": float(np.median([r["n"] / (r[form]["ms"] * 1e-3) for r in rows]))}
    both = [r for r in rows if r["learned"]["ok"] and r["rule"]["ok"]]
    speed = [r["rule"]["ms"] / r["learned"]["ms"] for r in both]
    summ["layouts_both_meet_tol"] = len(both)
    summ["geomean_speedup_learned_over_rule"] = float(math.exp(np.mean(np.log(speed)))) if speed else None
    summ["tol"] = args.tol
    summ["layouts"] = len(rows)
    with open(args.out, "w") as fh:
        json.dump({"summary": summ, "rows": rows}, fh, indent=1)
    print("[gain] summary", json.dumps(summ), flush=True)
    f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
