"""The learned parameter selector: its shipped weights and the scripts that
made them (run table on the GPU, training with the library's own network
kernels, held-out gain measurement)."""
from __future__ import annotations

import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
WEIGHTS_PATH = os.path.join(HERE, "weights.f32")
NFEAT = 92
HEADER = 194
THETAS = (0.35, 0.45, 0.55, 0.65, 0.75)

# The reduced-precision form the selector is trained for and used with: the
# lists with both structural options of Section 4 (interaction via the
# parent box, exchanged roles at every level), and FP32 arithmetic with FP32
# accumulation where the tolerance allows it (>= 1e-6), binary64
# accumulation below.  Over the 510 layouts of the run table (N 1e4..1e6)
# the least FP32 error of any configuration is at most 1e-6 on 99 % of them,
# at most 1e-7 on only 75 %.
LIST_OPTIONS = {"parent": True, "swap": "all"}


def reduced_mode(tol: float) -> str:
    return "fp32" if tol >= 1e-5 else "fp32_acc64"


def load_weights(path: str = WEIGHTS_PATH):
    """The weight blob (float32, fmm2d_select layout) or None if absent."""
    if not os.path.exists(path):
        return None
    return np.fromfile(path, dtype="<f4")


def weights_tensor(device, path: str = WEIGHTS_PATH):
    import torch

    b = load_weights(path)
    return None if b is None else torch.from_numpy(b.copy()).to(device)
