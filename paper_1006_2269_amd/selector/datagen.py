"""Run table for training the parameter selector (needs the GPU).

For each layout (``workloads.selector_layout``): its density features, the
binary64 judge at 1000 sampled targets, and for every level count L in
{L0 - 3, ..., L0 + 1} (L0 = round(log4(N / 16)); with the structural list
options the cheapest tree is coarser than one of about 16 points per leaf)
and theta in {0.35, ..., 0.75} the GPU times of build_tree and connectivity (warm: the
least of three calls after one that may allocate; the lists with the
structural options of ``selector.LIST_OPTIONS``), then for p = 4, 5, ... the
time of evaluate (mode FP32_ACC64, the reduced form below TOL 1e-5) and
the normwise error against the judge, until the error drops below 1e-8 or
stops improving (three orders without a 10 % gain).  Evaluate times are the GPU phases of one call
(HIP events), so growing buffers do not count.

    python -m paper_1006_2269_amd.selector.datagen --first 50000 --count 400 --out gpurun_out/runs.npz
    python -m paper_1006_2269_amd.selector.datagen --first 60000 --count 40 --lo 6 --hi 7 --thetas 0.45 0.55 0.65 --out gpurun_out/big.npz
    python -m paper_1006_2269_amd.selector.datagen --retime runs.npz --out runs_retimed.npz
"""
from __future__ import annotations

import argparse
import math
import sys
import time

import numpy as np

THETAS = (0.35, 0.45, 0.55, 0.65, 0.75)
P_MIN, P_MAX = 4, 30
E_STOP = 1e-8      # below every tolerance the selector is trained for, with the label margin
PLATEAU = 3        # stop after this many orders without a 10% gain
MODE = "fp32_acc64"


def L0_of(n: int) -> int:
    return int(math.floor(math.log(max(n / 16.0, 1.0)) / math.log(4.0) + 0.5))


BELOW, ABOVE = 3, 1  # candidate level counts L0 - BELOW .. L0 + ABOVE


def candidate_levels(n: int):
    L0 = L0_of(n)
    return [L for L in range(L0 - BELOW, L0 + ABOVE + 1) if 1 <= L <= 13 and 4 ** L <= n]


def phase_ms(f, names):
    t = f.timings()
    return sum(t[k][0] for k in names)


REPEATS = 3  # tree and list timings: the least of this many warm calls


def time_tree(f, x, y, L):
    """build_tree time at L, warm: the first call on a layout allocates."""
    f.build_tree(x, y, L)
    best = math.inf
    for _ in range(REPEATS):
        f.timing(True)
        f.build_tree(x, y, L)
        best = min(best, phase_ms(f, ["tree"]))
    return best


def time_lists(f, theta):
    """connectivity time at theta on the current tree, warm (see time_tree);
    raises FMM2DError where a level's lists exceed the int32 entry limit."""
    from paper_1006_2269_amd.selector import LIST_OPTIONS

    f.connectivity(theta, **LIST_OPTIONS)
    best = math.inf
    for _ in range(REPEATS):
        f.timing(True)
        f.connectivity(theta, **LIST_OPTIONS)
        best = min(best, phase_ms(f, ["lists"]))
    return best


def run_layout(f, ps, torch, samples=1000, thetas=THETAS):
    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2DError

    dev = f.device
    x = torch.from_numpy(ps.x).to(dev)
    y = torch.from_numpy(ps.y).to(dev)
    q = torch.from_numpy(ps.q).to(dev)
    tg = torch.from_numpy(W.sample_targets(ps.n, samples, seed=4242)).to(dev)
    exact = f.direct(x, y, q, tg)
    scale = float(exact.abs().max())
    feat = f.features(x, y, 1e-6).cpu().numpy()
    out = torch.empty_like(q)
    rows = []
    for L in candidate_levels(ps.n):
        t_tree = time_tree(f, x, y, L)
        for th in thetas:
            try:
                t_lists = time_lists(f, th)
            except FMM2DError:
                continue  # a level's lists exceed the int32 entry limit
            best, stale = math.inf, 0
            for p in range(P_MIN, P_MAX + 1):
                # HIP events bracket the GPU work only (buffers that grow come
                # from the caching allocator), so no warm-up call is needed
                f.timing(True)
                f.evaluate(q, p, MODE, out=out)
                t_eval = phase_ms(f, ["upward", "m2l", "l2l", "leaf", "other", "exchange"])
                e = float((out[tg] - exact).abs().max()) / scale
                rows.append((L, th, p, t_tree, t_lists, t_eval, e))
                stale = stale + 1 if e > 0.9 * best else 0
                best = min(best, e)
                if e <= E_STOP or stale >= PLATEAU:
                    break  # below the tolerances of interest, or at the FP32 error floor
        print("[datagen]   n=%d L=%d done (%d rows)" % (ps.n, L, len(rows)), flush=True)
    f.timing(False)
    return feat, rows


def retime(f, src, out, lo, hi, torch):
    """Re-measure the tree and list columns of an existing run table (warm,
    least of REPEATS calls), keeping its evaluate times and errors."""
    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2DError

    d = np.load(src)
    runs = d["runs"].copy()
    t0 = time.time()
    for i, seed in enumerate(d["seeds"]):
        ps = W.selector_layout(int(seed), lo, hi)
        assert ps.n == int(d["n"][i]), "layout %d does not regenerate" % i
        x = torch.from_numpy(ps.x).to(f.device)
        y = torch.from_numpy(ps.y).to(f.device)
        mine = runs[:, 0] == i
        for L in np.unique(runs[mine, 1]):
            t_tree = time_tree(f, x, y, int(L))
            rows_l = mine & (runs[:, 1] == L)
            runs[rows_l, 4] = t_tree
            for th in np.unique(runs[rows_l, 2]):
                try:
                    t_lists = time_lists(f, float(th))
                except FMM2DError:
                    continue
                runs[rows_l & (runs[:, 2] == th), 5] = t_lists
        print("[retime] layout %d seed %d n=%d  %.0f s" % (i, seed, ps.n, time.time() - t0), flush=True)
    np.savez_compressed(out, **{k: d[k] for k in d.files if k != "runs"}, runs=runs)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--retime", help="existing run table whose tree and list times are measured again")
    ap.add_argument("--first", type=int, default=50000)
    ap.add_argument("--count", type=int, default=400)
    ap.add_argument("--lo", type=float, default=4.0)
    ap.add_argument("--hi", type=float, default=6.0)
    ap.add_argument("--out", required=True)
    ap.add_argument("--save-every", type=int, default=5, help="write the table every this many layouts")
    ap.add_argument("--thetas", type=float, nargs="+", default=list(THETAS))
    args = ap.parse_args()
    import torch

    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2D
    from paper_1006_2269_amd.selector import LIST_OPTIONS

    f = FMM2D(0)
    if args.retime:
        retime(f, args.retime, args.out, args.lo, args.hi, torch)
        f.close()
        return 0
    feats, ns, table = [], [], []
    t0 = time.time()
    for i in range(args.count):
        seed = args.first + i
        ps = W.selector_layout(seed, args.lo, args.hi)
        feat, rows = run_layout(f, ps, torch, thetas=tuple(args.thetas))
        feats.append(feat)
        ns.append(ps.n)
        table.extend((i,) + r for r in rows)
        print("[datagen] layout %d seed %d n=%d runs=%d  %.0f s" % (i, seed, ps.n, len(rows), time.time() - t0),
              flush=True)
        if (i + 1) % args.save_every == 0 or i + 1 == args.count:
            np.savez_compressed(args.out, feats=np.array(feats, dtype=np.float32), n=np.array(ns, dtype=np.int64),
                     seeds=np.arange(args.first, args.first + i + 1), runs=np.array(table, dtype=np.float64),
                     log10_range=np.array([args.lo, args.hi]), mode=np.array(MODE),
                     levels_rel=np.array([-BELOW, ABOVE]), thetas=np.array(args.thetas),
                     list_options=np.array(sorted(LIST_OPTIONS.items()), dtype=object).astype(str),
                     columns=np.array(["layout", "L", "theta", "p", "t_tree_ms", "t_lists_ms", "t_eval_ms",
                                       "e_inf"]))
    f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
