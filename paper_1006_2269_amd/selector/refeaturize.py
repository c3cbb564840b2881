"""Recompute the feature vectors of a run table with the library (needs the
GPU), e.g. after the feature definition changed: each layout is regenerated
from its seed (``workloads.selector_layout``) and its features replace the
stored ones; the runs themselves are kept.

    python -m paper_1006_2269_amd.selector.refeaturize --runs a.npz --out a2.npz
"""
from __future__ import annotations

import argparse
import sys

import numpy as np


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--runs", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--lo", type=float, default=4.0)
    ap.add_argument("--hi", type=float, default=6.0)
    args = ap.parse_args()
    import torch

    from paper_1006_2269_amd import workloads as W
    from paper_1006_2269_amd.fmm import FMM2D

    d = np.load(args.runs)
    data = {k: d[k] for k in d.files}
    f = FMM2D(0)
    feats = np.empty_like(data["feats"])
    for i, seed in enumerate(data["seeds"]):
        ps = W.selector_layout(int(seed), args.lo, args.hi)
        if ps.n != int(data["n"][i]):
            raise RuntimeError("layout %d (seed %d) regenerates with n=%d, table has %d"
                               % (i, seed, ps.n, int(data["n"][i])))
        x = torch.from_numpy(ps.x).to(f.device)
        y = torch.from_numpy(ps.y).to(f.device)
        feats[i] = f.features(x, y, 1e-6).cpu().numpy()
    data["feats"] = feats
    np.savez_compressed(args.out, **data)
    print("[refeaturize] %s: %d layouts -> %s" % (args.runs, feats.shape[0], args.out), flush=True)
    f.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
