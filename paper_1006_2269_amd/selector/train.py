"""Training of the parameter selector on a run table (needs the GPU: the
network's forward pass, gradient and Adam steps are the library's kernels).

Samples.  For a layout of the run table and a tolerance TOL = 10^U[-7, -3]
(several per layout, seeded), the label is the cheapest measured
(L, theta, p) whose error meets TOL / M (the label margin M, default 4: a
configuration at the reduced-precision error floor of its level, where a
larger p gains nothing, is not taken for TOL itself), the cost being the
measured GPU time of build_tree + connectivity + evaluate.  The input is the layout's feature
vector with its second entry set to log10 TOL.  Pairs for which no measured
configuration meets TOL (below the FP32 error floor) are left out.

Targets (L - log4(N / 16), log10 C, theta), C the constant of the error
model C theta^(p+1), placed in the middle of the label's order
(log10 TOL = log10 C + (p + 1/2) log10 theta); decoding adds a safety factor
of 2 on the error.  The level target is the offset from log4(N / 16) itself:
the best level count follows the leaf size, which is smooth in N, while an
offset from round(log4(N / 16)) jumps by one wherever that rounding does and
is a sawtooth in N that the network fits poorly.  Targets and inputs are
standardised; mean and scale go into the weight blob's header together with
the trained range of log10 N (widened by 0.1 decade below and 0.15 above)
and log10 TOL.  Regularisation: an L2 penalty on the parameters (in the Adam
kernel) and Gaussian noise on the standardised inputs of each batch; the run
table has only a few hundred distinct layouts.  The parameters kept are
those of the lowest validation loss (layouts held out from training),
checked every 50 steps.

    python -m paper_1006_2269_amd.selector.train --runs a.npz b.npz --out weights.f32
"""
from __future__ import annotations

import argparse
import json
import math
import sys

import numpy as np

NFEAT = 92
HEADER = 194
TOL_LO, TOL_HI = -7.0, -3.0


def L0_of(n: int) -> int:
    return int(math.floor(log4_16(n) + 0.5))


def log4_16(n) -> float:
    """log4(N / 16), 0 below 16 points."""
    return math.log(max(n / 16.0, 1.0)) / math.log(4.0)


def load_runs(paths):
    feats, ns, runs, off = [], [], [], 0
    for p in paths:
        d = np.load(p)
        r = d["runs"].copy()
        r[:, 0] += off
        feats.append(d["feats"])
        ns.append(d["n"])
        runs.append(r)
        off += d["n"].shape[0]
    return np.concatenate(feats), np.concatenate(ns), np.concatenate(runs)


TIE = 1.10  # configurations within 10% of the cheapest count as ties


def best_config(R, tol):
    """Cheapest (cost_ms, L, theta, p) of one layout's runs meeting tol.
    Near-ties (within 10%: the cost is flat across theta for most layouts,
    and timing noise would flip the label) go to theta nearest 0.55, then
    more levels (smaller leaves: a lower reduced-precision error floor)."""
    cands = []
    keys = np.unique(R[:, 1:3], axis=0)
    for L, th in keys:
        S = R[(R[:, 1] == L) & (R[:, 2] == th)]
        S = S[np.argsort(S[:, 3])]
        ok = np.nonzero(S[:, 7] <= tol)[0]
        if ok.size == 0:
            continue
        row = S[ok[0]]
        cands.append((float(row[4] + row[5] + row[6]), int(L), float(th), int(row[3])))
    if not cands:
        return None
    cmin = min(c[0] for c in cands)
    near = [c for c in cands if c[0] <= TIE * cmin]
    return min(near, key=lambda c: (abs(c[2] - 0.55), -c[1], c[0]))


def make_samples(feats, ns, runs, layouts, per_layout, seed, margin=4.0):
    """Inputs and targets (L - log4(N / 16), log10 C, theta), where log10 C puts the
    label's order in the middle of the error model's interval:
    log10 TOL = log10 C + (p + 1/2) log10 theta."""
    rng = np.random.default_rng(seed)
    X, Y = [], []
    for i in layouts:
        R = runs[runs[:, 0] == i]
        if R.shape[0] == 0:
            continue
        for lt in rng.uniform(TOL_LO, TOL_HI, per_layout):
            b = best_config(R, 10.0 ** lt / margin)
            if b is None:
                continue
            x = feats[i].astype(np.float64).copy()
            x[1] = lt
            X.append(x)
            lc = lt - (b[3] + 0.5) * math.log10(b[2])
            Y.append((b[1] - log4_16(int(ns[i])), lc, b[2]))
    return np.array(X), np.array(Y, dtype=np.float64)


def init_params(d_in, seed):
    rng = np.random.default_rng(seed)
    dims = [d_in, 64, 64, 64, 3]
    parts = []
    for i in range(4):
        fan_in, fan_out = dims[i], dims[i + 1]
        parts.append(rng.normal(0.0, 1.0 / math.sqrt(fan_in), fan_out * fan_in))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", nargs="+", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--per-layout", type=int, default=32)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--weight-decay", type=float, default=1e-2)
    ap.add_argument("--input-noise", type=float, default=0.5)
    ap.add_argument("--val-frac", type=float, default=0.1)
    ap.add_argument("--seed", type=int, default=7)
    ap.add_argument("--label-margin", type=float, default=4.0)
    args = ap.parse_args()
    import torch

    from paper_1006_2269_amd.fmm import FMM2D

    feats, ns, runs = load_runs(args.runs)
    nl = ns.shape[0]
    order = np.random.default_rng(args.seed).permutation(nl)
    nval = max(1, int(round(args.val_frac * nl)))
    val_l, tr_l = order[:nval], order[nval:]
    Xtr, Ytr = make_samples(feats, ns, runs, tr_l, args.per_layout, args.seed, args.label_margin)
    Xva, Yva = make_samples(feats, ns, runs, val_l, args.per_layout, args.seed + 1, args.label_margin)
    print("[train] layouts %d (val %d), samples %d (val %d)" % (nl, nval, Xtr.shape[0], Xva.shape[0]), flush=True)

    xm = Xtr.mean(axis=0)
    xs = Xtr.std(axis=0)
    xscale = np.where(xs > 1e-6, 1.0 / np.maximum(xs, 1e-12), 1.0)
    ym, ysd = Ytr.mean(axis=0), Ytr.std(axis=0)
    ysd = np.where(ysd > 1e-6, ysd, 1.0)
    norm_x = lambda X: ((X - xm) * xscale).astype(np.float32)
    norm_y = lambda Y: ((Y - ym) / ysd).astype(np.float32)

    dev = torch.device("cuda", 0)
    f = FMM2D(0)
    params = torch.from_numpy(init_params(NFEAT, args.seed)).to(dev)
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    Xt, Yt = torch.from_numpy(norm_x(Xtr)).to(dev), torch.from_numpy(norm_y(Ytr)).to(dev)
    Xv, Yv = torch.from_numpy(norm_x(Xva)).to(dev), torch.from_numpy(norm_y(Yva)).to(dev)
    grad = torch.empty_like(params)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    gen = torch.Generator(device="cpu").manual_seed(args.seed)
    ntr = Xt.shape[0]
    best = (math.inf, 0, params.clone())
    for step in range(1, args.steps + 1):
        idx = torch.randint(0, ntr, (min(args.batch, ntr),), generator=gen).to(dev)
        xb, yb = Xt[idx].contiguous(), Yt[idx].contiguous()
        if args.input_noise > 0.0:
            xb += (args.input_noise * torch.randn(xb.shape, generator=gen)).to(dev)
        lr = args.lr * 0.5 * (1.0 + math.cos(math.pi * step / args.steps))  # cosine decay
        f.mlp_grad(params, xb, yb, grad, loss)
        f.mlp_adam(params, m, v, grad, step=step, lr=max(lr, 1e-5), weight_decay=args.weight_decay)
        if step % 50 == 0 or step == args.steps:
            _, lv = f.mlp_grad(params, Xv, Yv)
            lv = float(lv.cpu())
            if lv < best[0]:
                best = (lv, step, params.clone())
            if step % 500 == 0 or step == args.steps:
                print("[train] step %d  batch loss %.4f  val loss %.4f  (best %.4f at %d)"
                      % (step, float(loss.cpu()), lv, best[0], best[1]), flush=True)
    params = best[2]

    # decision quality on the validation layouts: decoded (levels, theta, p)
    # against the labels
    pred = f.mlp_forward(params, Xv).cpu().numpy().astype(np.float64) * ysd + ym
    thetas = np.array([0.35, 0.45, 0.55, 0.65, 0.75])
    th_p = thetas[np.clip(np.floor((pred[:, 2] - 0.35) / 0.1 + 0.5), 0, 4).astype(int)]
    p_dec = np.ceil((Xva[:, 1] - math.log10(2.0) - pred[:, 1]) / np.log10(th_p)) - 1
    p_lab = np.round((Xva[:, 1] - Yva[:, 1]) / np.log10(Yva[:, 2]) - 0.5)
    l4 = np.log(np.maximum(10.0 ** Xva[:, 0] / 16.0, 1.0)) / math.log(4.0)
    dl_ok = np.mean(np.floor(pred[:, 0] + l4 + 0.5) == np.floor(Yva[:, 0] + l4 + 0.5))
    th_ok = np.mean(np.isclose(th_p, Yva[:, 2]))
    p_ok = np.mean(p_dec >= p_lab)
    print("[train] val: levels exact %.3f, theta exact %.3f, decoded p >= label p %.3f" % (dl_ok, th_ok, p_ok),
          flush=True)

    blob = np.zeros(HEADER + params.numel(), dtype=np.float32)
    blob[:NFEAT] = xm
    blob[NFEAT:2 * NFEAT] = xscale
    blob[2 * NFEAT:2 * NFEAT + 3] = ym
    blob[2 * NFEAT + 3:2 * NFEAT + 6] = ysd
    lnn = np.log10(ns.astype(np.float64))
    blob[2 * NFEAT + 6:2 * NFEAT + 10] = (lnn.min() - 0.1, lnn.max() + 0.15, TOL_LO, TOL_HI)
    blob[HEADER:] = params.cpu().numpy()
    blob.astype("<f4").tofile(args.out)
    meta = {"layouts": int(nl), "val_layouts": int(nval), "samples": int(Xtr.shape[0]),
            "val_samples": int(Xva.shape[0]), "steps": args.steps, "batch": args.batch, "lr": args.lr,
            "weight_decay": args.weight_decay, "input_noise": args.input_noise, "label_margin": args.label_margin,
            "val_levels_exact": float(dl_ok), "val_theta_exact": float(th_ok), "val_p_covers_label": float(p_ok),
            "best_step": int(best[1]), "best_val_loss": float(best[0]),
            "log10_n_range": [float(lnn.min()) - 0.1, float(lnn.max()) + 0.15], "log10_tol_range": [TOL_LO, TOL_HI]}
    with open(args.out + ".json", "w") as fh:
        json.dump(meta, fh, indent=1)
    print("[train] wrote %s (%d floats)" % (args.out, blob.size), flush=True)
    f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
