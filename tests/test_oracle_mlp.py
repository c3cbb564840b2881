"""Pins of the FP64 selector-network reference: a forward pass with hand-set
weights against its closed form, gradients against central finite
differences, the first Adam step against its closed form, and Adam with the
L2 term against the ridge minimiser it must reach."""
import numpy as np

from oracle import mlp


def test_forward_closed_form():
    shapes = mlp.layer_shapes(2, hidden=4, d_out=1, depth=3)
    layers = []
    for o, i in shapes:
        layers.append([np.zeros((o, i)), np.zeros(o)])
    layers[0][0][0, 0] = 1.0      # h1[0] = tanh(x0)
    layers[1][0][0, 0] = 2.0      # h2[0] = tanh(2 h1[0])
    layers[2][1][1] = 0.3         # h3[1] = tanh(0.3)
    layers[2][0][0, 0] = 1.0      # h3[0] = tanh(h2[0])
    layers[3][0][0, :2] = [1.5, -1.0]
    layers[3][1][0] = 0.25
    theta = np.concatenate([np.concatenate([W.ravel(), b]) for W, b in layers])
    X = np.array([[0.7, -3.0], [-0.2, 9.0]])
    out, _ = mlp.forward(theta, X, shapes)
    want = 1.5 * np.tanh(np.tanh(2 * np.tanh(X[:, 0]))) - np.tanh(0.3) + 0.25
    assert np.allclose(out[:, 0], want, rtol=0, atol=1e-15)


def test_gradient_central_differences():
    g = np.random.Generator(np.random.PCG64(3))
    shapes = mlp.layer_shapes(7, hidden=6, d_out=3, depth=3)
    theta = g.normal(size=mlp.n_params(7, 6, 3, 3)) * 0.5
    X = g.normal(size=(5, 7))
    Y = g.normal(size=(5, 3))
    L, gr = mlp.grad(theta, X, Y, shapes)
    assert abs(L - mlp.loss(theta, X, Y, shapes)) < 1e-15
    h = 1e-6
    for k in range(theta.shape[0]):
        e = np.zeros_like(theta)
        e[k] = h
        fd = (mlp.loss(theta + e, X, Y, shapes) - mlp.loss(theta - e, X, Y, shapes)) / (2 * h)
        assert abs(fd - gr[k]) <= 1e-7 * max(1.0, abs(fd))


def test_first_adam_step_closed_form():
    # After one step from zero moments: mhat = g, vhat = g^2, so every
    # parameter moves by -lr * g / (|g| + eps).
    g = np.array([0.5, -2.0, 1e-3, 0.0])
    theta = np.array([1.0, 1.0, 1.0, 1.0])
    lr = 0.01
    t1, m, v = mlp.adam_step(theta, np.zeros(4), np.zeros(4), g, 1, lr)
    assert np.allclose(t1, theta - lr * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_weight_decay_reaches_ridge_minimiser():
    # Adam with the L2 term on f(t) = sum (t - a)^2 settles at the minimiser
    # of f + (wd / 2) |t|^2, which is t* = 2a / (2 + wd) (ridge shrinkage);
    # without the term it settles at a.
    a = np.array([1.5, -0.75, 0.25])
    for wd, want in ((0.5, 2 * a / 2.5), (0.0, a)):
        t, m, v = np.zeros(3), np.zeros(3), np.zeros(3)
        for step in range(1, 6001):
            lr = 0.05 * 0.5 * (1 + np.cos(np.pi * step / 6000)) + 1e-6
            t, m, v = mlp.adam_step(t, m, v, 2 * (t - a), step, lr, wd=wd)
        assert np.allclose(t, want, atol=1e-4), (wd, t, want)
