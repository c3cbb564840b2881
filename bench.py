#!/usr/bin/env python
"""Throughput benchmark: target points per second at relative error 1e-6.

Workload (default): the 1M-point mixed set -- 500,000 uniform points in
[0,1]^2 plus 4 x 125,000 Gaussian points (sigma 0.1, 0.03, 0.01, 0.003),
charges U[-1,1] -- at tolerance 1e-6; the plain form uses 8 levels and
theta = 1/2.

A step is one pass of the whole hot path with inputs already in device
memory.  Two forms are timed:

* learned (``value``): parameter selection by the trained selector (its
  density features and network run on the GPU inside the step), then tree,
  lists and evaluation in mode ``fp32_acc64`` (FP32 near field and FP32 M2L
  products, binary64 power scaling and accumulation);
* plain FP64 (``config.fp64_points_per_s``): 8 levels, theta = 1/2, and the
  least p whose error passes the judge.

The judge is the binary64 direct sum (compensated) at 1000 seeded targets; a
form counts only when its normwise relative error there is <= the tolerance.
If the learned choice misses the judge, the reduced-precision form falls
back to the judge-verified order at 8 levels (and says so in ``config``).
One JSON line goes to stdout; phase timings and list statistics to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

MI355X = {"hbm_GBps": 8000.0, "fp32_TFLOPs": 157.3, "fp64_TFLOPs": 78.6, "fp32_mfma_TFLOPs": 157.3}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_mixed_1m.json")


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what the counter reads
    for a plain copy of known size), or None when there is none or the
    kernel's source file has changed since the counters were taken."""
    import hashlib

    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as fh:
        entry = json.load(fh).get(kernel)
    if not entry:
        return None
    with open(os.path.join(ROOT, entry["source"]), "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != entry["source_sha256"]:
            return None
    return entry["bytes_per_launch"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="mixed_1m")
    ap.add_argument("--scale", type=float, default=1.0, help="workload size factor (1.0 = full size)")
    ap.add_argument("--levels", type=int, default=8)
    ap.add_argument("--theta", type=float, default=0.5)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--samples", type=int, default=1000)
    ap.add_argument("--cpu-baseline", type=int, default=1)
    ap.add_argument("--cpu-scale", type=float, default=1.0,
                    help="size factor of the CPU-baseline sample of the same workload")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="repeat the CPU baseline until this much time has passed")
    ap.add_argument("--fp64", type=int, default=1, help="also time the plain FP64 form")
    ap.add_argument("--sweep", choices=["field", "robustness"],
                    help="run a measurement sweep instead of the benchmark (JSON table to --out)")
    ap.add_argument("--out", help="output file of a sweep")
    ap.add_argument("--sizes", help="robustness sweep: comma-separated N")
    ap.add_argument("--sweep-n", type=int, default=0, help="field sweep: points (default 10^6)")
    ap.add_argument("--sweep-levels", type=int, default=8, help="field sweep: levels")
    return ap.parse_args()


def sweep_field(args):
    """Relative error of the FMM field (the gradient of the potential) against
    the direct field versus the expansion order, for theta in {0.25, 0.5,
    sqrt(1/2)}: the shape of Section 5's first experiment, for the gradient
    q_j (z_i - z_j)/|z_i - z_j|^2 of the logarithmic kernel (the complex
    conjugate of that experiment's force kernel q_j/(z_i - z_j)).  10^6 points
    of total mass 1 in the unit disc, uniform and 1/r radial density, 8 levels,
    error at 1000 sampled targets against fmm2d_direct_field; the time of one
    fmm2d_evaluate_field by HIP events on the library stream."""
    args.n = args.sweep_n or 1_000_000
    args.pmax = 30
    THETAS = (0.25, 0.5, math.sqrt(0.5))
    import numpy as np
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
        f.build_tree(x, y, args.sweep_levels)
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
        json.dump({"n": args.n, "levels": args.sweep_levels, "samples": args.samples, "rows": rows}, fh, indent=1)
    f.close()
    return 0


def sweep_robustness(args):
    """Time of the whole path versus N on three layouts at TOL = 1e-6: the shape
    of Section 5's third experiment (uniform in the unit square, and the
    'normal' and 'layer' layouts of the second, sigma = 0.1).  Per layout and
    N: the reduced form (fmm2d_select_build_tree, connectivity, evaluate in
    FP32_ACC64) and plain binary64 at the a-priori rule's parameters; time =
    median of 3 after a warm-up (HIP events on the library stream), e_inf
    against the binary64 direct sum at 1000 sampled targets."""
    SIZES = (10_000, 30_000, 100_000, 300_000, 1_000_000, 2_000_000, 5_000_000)
    TOL = 1e-6
    sizes = args.sizes or ",".join(str(s) for s in SIZES)
    import numpy as np
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
        for n in (int(s) for s in sizes.split(",")):
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



def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: this library has no multi-GPU path (the design notes describe how the "
              "tree would shard); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.sweep:
        if not args.out:
            print("--sweep needs --out", file=sys.stderr)
            sys.exit(2)
        sys.exit({"field": sweep_field, "robustness": sweep_robustness}[args.sweep](args))
    import numpy as np
    import torch

    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2D

    ps = W.WORKLOADS[args.workload](scale=args.scale)
    n, L, theta, tol = ps.n, args.levels, args.theta, args.tol
    while L > 0 and n < 4 ** L:
        L -= 1
    log("[bench] workload %s n=%d levels=%d theta=%.3f tol=%.1e" % (ps.name, n, L, theta, tol))
    dev = torch.device("cuda", 0)
    x = torch.from_numpy(ps.x).to(dev)
    y = torch.from_numpy(ps.y).to(dev)
    q = torch.from_numpy(ps.q).to(dev)
    tg = torch.from_numpy(W.sample_targets(n, args.samples, seed=4242)).to(dev)
    f = FMM2D(0)
    exact = f.direct(x, y, q, tg)
    torch.cuda.synchronize()
    scale_ref = float(exact.abs().max())

    def rel_err(phi):
        return float((phi[tg] - exact).abs().max()) / scale_ref

    def one_step(p, mode, out):
        f.build_tree(x, y, L)
        f.connectivity(theta)
        f.evaluate(q, p, mode, out=out)

    out = torch.empty_like(q)
    f.build_tree(x, y, L)
    f.connectivity(theta)
    sizes = [f.list_sizes(l) for l in range(L + 1)]
    log("[bench] list entries per level (strong, weak):", sizes)

    def search_p(mode, lo=2, hi=40):
        # least p passing the judge (error decreases with p)
        best = None
        while lo <= hi:
            mid = (lo + hi) // 2
            f.evaluate(q, mid, mode, out=out)
            e = rel_err(out)
            log("[bench] %s p=%d e_inf=%.3e" % (mode, mid, e))
            if e <= tol:
                best, hi = (mid, e), mid - 1
            else:
                lo = mid + 1
        return best

    def timed(p, mode):
        for _ in range(args.warmup):
            one_step(p, mode, out)
        torch.cuda.synchronize()
        f.timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one_step(p, mode, out)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        tm = f.timings()
        f.timing(False)
        return dt, tm, rel_err(out)

    results = {}

    # -- learned form: select + tree + lists + evaluate per step ------------
    from paper_1006_2269_amd import selector

    weights = selector.weights_tensor(dev)
    learned = None
    if weights is not None:
        def step_learned():
            # select + build_tree in one call (the sort overlaps the selector)
            Ls, ps_, th, net = f.select_build_tree(x, y, tol, weights)
            f.connectivity(th)
            f.evaluate(q, ps_, "fp32_acc64", out=out)
            return Ls, ps_, th, net

        for _ in range(args.warmup):
            cfg = step_learned()
        torch.cuda.synchronize()
        f.timing(True)
        t0 = time.perf_counter()
        for _ in range(args.steps):
            cfg = step_learned()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / args.steps
        tm = f.timings()
        f.timing(False)
        e = rel_err(out)
        Ls, ps_, th, net = cfg
        log("[bench] learned: levels=%d p=%d theta=%.2f (network=%s)  %.2f ms/step  %.3e pts/s  e_inf=%.2e"
            % (Ls, ps_, th, net, dt * 1e3, n / dt, e))
        for ph, (ms, cnt) in tm.items():
            if cnt:
                log("   %-7s %9.3f ms/step  (%d intervals)" % (ph, ms / args.steps, cnt))
        learned = {"levels": Ls, "p": ps_, "theta": th, "network": net, "s_per_step": dt, "points_per_s": n / dt,
                   "e_inf": e, "phases": tm}
        if e <= tol:
            results["fp32_acc64"] = dict(learned, selector="learned")
        else:
            log("[bench] the learned choice misses the judge (%.2e > %.1e)" % (e, tol))
    else:
        log("[bench] no trained selector weights at %s" % selector.WEIGHTS_PATH)

    forms = ([] if "fp32_acc64" in results else [("fp32_acc64", "reduced")]) + \
        ([("fp64", "plain")] if args.fp64 else [])
    for mode, label in forms:
        f.build_tree(x, y, L)
        f.connectivity(theta)
        found = search_p(mode)
        if found is None:
            log("[bench] %s: no p <= 40 passes the judge" % mode)
            continue
        p, _ = found
        dt, tm, e = timed(p, mode)
        results[mode] = {"levels": L, "theta": theta, "p": p, "s_per_step": dt, "points_per_s": n / dt, "e_inf": e,
                         "phases": tm, "selector": "judge-verified order"}
        log("[bench] %s p=%d  %.2f ms/step  %.3e pts/s  e_inf=%.2e" % (mode, p, dt * 1e3, n / dt, e))
        for ph, (ms, cnt) in tm.items():
            if cnt:
                log("   %-7s %9.3f ms/step  (%d intervals)" % (ph, ms / args.steps, cnt))

    main_form = results.get("fp32_acc64")
    # roofline of the dominant single kernel launch of the reduced form: the
    # near-field kernel, or the M2L kernel (all levels; both timed alone with
    # HIP events on the library's stream during the timed steps)
    roof = None
    if main_form:
        p = main_form["p"]
        Lm = main_form["levels"]
        f.build_tree(x, y, Lm)
        f.connectivity(main_form["theta"])
        ph = main_form["phases"]
        near_ms = ph["near_kernel"][0] / max(ph["near_kernel"][1], 1)
        m2l_ms = ph["m2l_kernel"][0] / max(ph["m2l_kernel"][1], 1)
        sptr, sidx, _, _ = f.lists(Lm)
        st = f.leaf_start().cpu().numpy().astype(np.int64)
        cnt = np.diff(st)
        sp = sptr.cpu().numpy().astype(np.int64)
        si = sidx.cpu().numpy().astype(np.int64)
        src_per_leaf = np.add.reduceat(cnt[si], sp[:-1]) if si.size else np.zeros_like(cnt)
        src_per_leaf[np.diff(sp) == 0] = 0
        pairs = float((cnt * src_per_leaf).sum())    # ordered (target, source) point pairs
        rows = np.repeat(np.arange(cnt.size), np.diff(sp))
        diag = float((cnt[rows[si == rows]].astype(np.float64) ** 2).sum())  # pairs within one leaf
        weak_all = float(sum(f.list_sizes(l)[1] for l in range(Lm + 1)))
        # The library's leaf pass takes each pair of distinct leaves once when
        # the largest leaf, ceil(N / 4^L) points, holds 17 to 64 (FP32 modes):
        # one log serves both directions, 2 sub, mul, fma (2), log2, fma (2),
        # fma (2) = 10 flops per pair of points; pairs within a leaf, and every
        # pair in the one-sided kernels, need 8 (one fma less).
        maxleaf = -(-n // 4 ** Lm)
        if 16 < maxleaf <= 64:
            near_name = "k_near32s (pair-once near field, one launch)"
            near_flops = (pairs - diag) / 2.0 * 10.0 + diag * 8.0
            near_work = "%d point pairs of distinct leaves, each taken once x 10 flops + %d within leaves x 8" % (
                (pairs - diag) / 2, diag)
        else:
            near_name = "%s (near field, one launch)" % ("k_near32_big" if maxleaf > 64 else "k_near32")
            near_flops = pairs * 8.0
            near_work = "%d point pairs x 8 flops" % pairs
        m2l_flops = weak_all * 4.0 * (p + 1) ** 2               # useful product flops per weak pair
        if m2l_ms >= near_ms:
            ach = m2l_flops / (m2l_ms * 1e-3) / 1e12
            roof = {"kernel": "k_m2l_lp (M2L, all levels, one launch)", "bound": "mfma", "achieved": round(ach, 3),
                    "peak": MI355X["fp32_mfma_TFLOPs"], "unit": "TFLOP/s",
                    "frac": round(ach / MI355X["fp32_mfma_TFLOPs"], 5), "traffic": None,
                    "work": "%d weak pairs x 4(p+1)^2 flops" % weak_all, "launch_ms": round(m2l_ms, 4)}
        else:
            ach = near_flops / (near_ms * 1e-3) / 1e12
            roof = {"kernel": near_name, "bound": "alu", "achieved": round(ach, 3),
                    "peak": MI355X["fp32_TFLOPs"], "unit": "TFLOP/s", "frac": round(ach / MI355X["fp32_TFLOPs"], 5),
                    "traffic": None, "work": near_work, "launch_ms": round(near_ms, 4)}
        log("[bench] near kernel %.4f ms (%.3e pairs/s), M2L kernel %.4f ms (%.3e weak pairs/s)"
            % (near_ms, pairs / (near_ms * 1e-3), m2l_ms, weak_all / (m2l_ms * 1e-3)))

    if roof is not None:
        roof["traffic"] = measured_traffic(roof["kernel"])

    cpu = None
    if args.cpu_baseline:
        import oracle

        cps = W.WORKLOADS[args.workload](scale=args.cpu_scale)
        Lc = main_form["levels"] if main_form else L
        thc = main_form["theta"] if main_form else theta
        cl = max(1, int(round(math.log(cps.n / (n / 4 ** Lc), 4))))   # same points per leaf
        p = main_form["p"] if main_form else 12
        # repeat the whole oracle path until about 10 s of CPU work have run
        reps, t0 = 0, time.perf_counter()
        while True:
            tr = oracle.tree(cps.x, cps.y, cl)
            ls = oracle.lists(tr, thc)
            oracle.fmm_eval(cps.x, cps.y, cps.q, tr, ls, p)
            reps += 1
            dt = time.perf_counter() - t0
            if dt >= args.cpu_seconds or reps >= 20:
                break
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        cpu = {"value": round(reps * cps.n / dt, 1), "unit": "target points/s", "cores": threads, "kind": "oracle",
               "sample": "%s at size factor %g (%d points, %d levels, p=%d, theta=%.2f): tree + lists + FP64 FMM, "
                         "%d repetitions in %.1f s" % (args.workload, args.cpu_scale, cps.n, cl, p, thc, reps, dt)}
        log("[bench] cpu oracle: %.1f s for %d x %d points" % (dt, reps, cps.n))

    if main_form is None:
        log("[bench] no form passed the judge")
        sys.exit(1)
    line = {
        "metric": "target points/sec at rel. error 1e-6 (FP32+learned vs plain FP64 FMM)",
        "value": round(main_form["points_per_s"], 1),
        "unit": "target points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_form["s_per_step"] * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s (n=%d)" % (args.workload, n), "levels": main_form["levels"],
                   "theta": main_form["theta"], "tol": tol, "p": main_form["p"], "mode": "fp32_acc64",
                   "selector": main_form["selector"],
                   "learned_choice": None if learned is None else
                   {k: learned[k] for k in ("levels", "p", "theta", "network", "e_inf")},
                   "e_inf": main_form["e_inf"], "judge_samples": args.samples,
                   "fp64_points_per_s": round(results["fp64"]["points_per_s"], 1) if "fp64" in results else None,
                   "fp64_p": results["fp64"]["p"] if "fp64" in results else None},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    f.close()


if __name__ == "__main__":
    main()
