"""FP64 reference of the parameter-selector network -- TEST INFRASTRUCTURE ONLY.

A multilayer perceptron with three hidden layers of width H and tanh
activations, a linear output layer, the mean-squared-error loss over all
outputs of a batch, its analytic gradient by back-propagation, and one Adam
update (Kingma & Ba, 2015: bias-corrected first and second moments).

The flat parameter vector is laid out layer by layer, each layer as its weight
matrix (row-major, [fan_out][fan_in]) followed by its bias vector.
"""
from __future__ import annotations

import numpy as np


def layer_shapes(d_in: int, hidden: int = 64, d_out: int = 3, depth: int = 3):
    dims = [d_in] + [hidden] * depth + [d_out]
    return [(dims[i + 1], dims[i]) for i in range(len(dims) - 1)]


def n_params(d_in: int, hidden: int = 64, d_out: int = 3, depth: int = 3) -> int:
    return sum(o * i + o for o, i in layer_shapes(d_in, hidden, d_out, depth))


def unpack(theta, shapes):
    theta = np.asarray(theta, dtype=np.float64)
    out, k = [], 0
    for o, i in shapes:
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    assert k == theta.shape[0]
    return out


def forward(theta, X, shapes):
    """Returns the outputs [B, d_out] and the hidden activations."""
    h = np.asarray(X, dtype=np.float64)
    acts = [h]
    layers = unpack(theta, shapes)
    for li, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.tanh(z) if li < len(layers) - 1 else z
        acts.append(h)
    return h, acts


def loss(theta, X, Y, shapes) -> float:
    out, _ = forward(theta, X, shapes)
    d = out - np.asarray(Y, dtype=np.float64)
    return float(np.mean(d * d))


def grad(theta, X, Y, shapes):
    """Loss and its gradient with respect to the flat parameter vector."""
    out, acts = forward(theta, X, shapes)
    Y = np.asarray(Y, dtype=np.float64)
    d = out - Y
    L = float(np.mean(d * d))
    delta = 2.0 * d / d.size                    # dL/d(out)
    layers = unpack(theta, shapes)
    grads = [None] * len(layers)
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in = acts[li]
        gW = delta.T @ a_in
        gb = delta.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            delta = (delta @ W) * (1.0 - acts[li] ** 2)   # tanh' = 1 - tanh^2
    flat = np.concatenate([np.concatenate([gW.ravel(), gb]) for gW, gb in grads])
    return L, flat


def adam_step(theta, m, v, g, step: int, lr: float, b1=0.9, b2=0.999, eps=1e-8, wd=0.0):
    """One Adam update; `step` counts from 1.  wd adds the gradient of the L2
    penalty (wd / 2) |theta|^2 to g first.  Returns new (theta, m, v)."""
    g = np.asarray(g, dtype=np.float64) + wd * np.asarray(theta, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    theta = np.asarray(theta, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v
