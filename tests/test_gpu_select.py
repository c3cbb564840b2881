"""GPU parity of the parameter selector through the C ABI.

Features must equal the oracle's exactly (integer cell counts; the two
logarithms to one float ulp); the decision with no weights must equal the
a-priori rule; with a weight blob, the decision must equal the oracle's
decoding of the network's own outputs; the network kernels (forward,
gradient, Adam) must match the binary64 reference of oracle/mlp.py.
"""
import math
import sys

import numpy as np
import pytest

from oracle import mlp as M
from oracle import select as S
from paper_1006_2269_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_2269_amd.fmm import FMM2D

    ctx = FMM2D(0)
    yield ctx
    ctx.close()


def _layouts():
    g = (np.arange(64) + 0.5) / 64
    X, Y = np.meshgrid(g, g)
    return {
        "uniform_10k": W.uniform_10k(),
        "mixed_1m_scaled_50k": W.mixed_1m(scale=0.05),
        "mixed_1m_scaled_400k": W.mixed_1m(scale=0.4),  # above 2^18: sampled cell counts
        "clustered_scaled_30k": W.clustered_10m(scale=0.003),
        "grid_64x64": W.PointSet("grid", X.ravel().copy(), Y.ravel().copy(), np.ones(4096)),
        "coincident_100": W.PointSet("coincident", np.full(100, 0.25), np.full(100, -3.0), np.ones(100)),
    }


LAYOUTS = _layouts()


@pytest.mark.parametrize("name", sorted(LAYOUTS))
@pytest.mark.parametrize("tol", [1e-3, 1e-6, 1e-9])
def test_features_parity(fmm, name, tol):
    ps = LAYOUTS[name]
    _announce("features", name, ps.n, tol)
    got = fmm.features(_dev(ps.x), _dev(ps.y), tol).cpu().numpy()
    exp = S.features(ps.x, ps.y, tol)
    np.testing.assert_array_equal(got[2:], exp[2:])
    np.testing.assert_array_max_ulp(got[:2], exp[:2], maxulp=1)


@pytest.mark.parametrize("n,tol", [(10_000, 1e-3), (200_000, 1e-6), (1_000_000, 1e-6), (50_000, 1e-9),
                                   (40, 1e-4), (5, 0.9)])
def test_select_rule_without_weights(fmm, n, tol):
    ps = W.uniform(n, 99)
    _announce("select rule", n, tol)
    L, p, th, net = fmm.select(_dev(ps.x), _dev(ps.y), tol)
    assert (L, p, th) == S.rule(n, tol) and net is False


def _random_blob(fmm, seed):
    rng = np.random.default_rng(seed)
    npar = fmm.mlp_nparams(S.NFEAT)
    b = np.zeros(S.HEADER + npar, dtype=np.float32)
    b[:S.NFEAT] = rng.normal(0, 0.1, S.NFEAT)
    b[S.NFEAT:2 * S.NFEAT] = rng.uniform(0.5, 2.0, S.NFEAT)
    b[2 * S.NFEAT: 2 * S.NFEAT + 3] = (0.0, 12.0, 0.5)
    b[2 * S.NFEAT + 3: 2 * S.NFEAT + 6] = (1.0, 4.0, 0.15)
    b[2 * S.NFEAT + 6: 2 * S.NFEAT + 10] = (3.5, 6.5, -8.0, -3.0)
    b[S.HEADER:] = rng.normal(0, 0.3, npar)
    return b


@pytest.mark.parametrize("seed", [11, 12, 13])
@pytest.mark.parametrize("name", ["uniform_10k", "mixed_1m_scaled_50k", "clustered_scaled_30k"])
def test_select_network_decision(fmm, name, seed):
    ps = LAYOUTS[name]
    tol = 1e-6
    blob = _random_blob(fmm, seed)
    _announce("select network", name, seed)
    x, y = _dev(ps.x), _dev(ps.y)
    L, p, th, net = fmm.select(x, y, tol, _dev(blob))
    # the network's outputs on the GPU features, standardised in FP32
    feat = fmm.features(x, y, tol).cpu().numpy()
    xin = (feat - blob[:S.NFEAT]) * blob[S.NFEAT:2 * S.NFEAT]
    out = fmm.mlp_forward(_dev(blob[S.HEADER:]), _dev(xin[None, :])).cpu().numpy()[0]
    assert (L, p, th, net) == S.decide(out, blob, ps.n, tol)
    assert net is True
    # the outputs themselves against the binary64 reference
    ref, _ = M.forward(blob[S.HEADER:].astype(np.float64), xin[None, :].astype(np.float64),
                       M.layer_shapes(S.NFEAT))
    np.testing.assert_allclose(out, ref[0], rtol=1e-4, atol=1e-5)


def test_select_outside_range_uses_rule(fmm):
    ps = LAYOUTS["uniform_10k"]
    blob = _random_blob(fmm, 5)
    for tol in (1e-9, 0.5):  # log10 tol outside [-8, -3]
        L, p, th, net = fmm.select(_dev(ps.x), _dev(ps.y), tol, _dev(blob))
        assert (L, p, th) == S.rule(ps.n, tol) and net is False


def test_select_rejects_bad_coordinates(fmm):
    from paper_1006_2269_amd.fmm import FMM2DError

    x = np.random.default_rng(0).random(1000)
    y = x.copy()
    x[17] = np.nan
    with pytest.raises(FMM2DError):
        fmm.select(_dev(x), _dev(y), 1e-6)
    y[3] = 2.0 ** 501
    x[17] = 0.5
    with pytest.raises(FMM2DError):
        fmm.select(_dev(x), _dev(y), 1e-6)


@pytest.mark.parametrize("d_in,batch", [(92, 1), (92, 37), (92, 256), (5, 70), (128, 33)])
def test_mlp_forward(fmm, d_in, batch):
    rng = np.random.default_rng(d_in * 1000 + batch)
    shapes = M.layer_shapes(d_in)
    theta = rng.normal(0, 1.0 / math.sqrt(d_in), M.n_params(d_in)).astype(np.float32)
    X = rng.normal(0, 1, (batch, d_in)).astype(np.float32)
    got = fmm.mlp_forward(_dev(theta), _dev(X)).cpu().numpy()
    ref, _ = M.forward(theta.astype(np.float64), X.astype(np.float64), shapes)
    np.testing.assert_allclose(got, ref, rtol=1e-5, atol=1e-5 * np.abs(ref).max())


@pytest.mark.parametrize("d_in,batch", [(92, 64), (92, 256), (7, 45)])
def test_mlp_gradient(fmm, d_in, batch):
    rng = np.random.default_rng(7 + batch)
    shapes = M.layer_shapes(d_in)
    theta = rng.normal(0, 0.5 / math.sqrt(d_in), M.n_params(d_in)).astype(np.float32)
    X = rng.normal(0, 1, (batch, d_in)).astype(np.float32)
    Y = rng.normal(0, 1, (batch, 3)).astype(np.float32)
    g, loss = fmm.mlp_grad(_dev(theta), _dev(X), _dev(Y))
    g = g.cpu().numpy().astype(np.float64)
    lref, gref = M.grad(theta.astype(np.float64), X.astype(np.float64), Y.astype(np.float64), shapes)
    assert abs(float(loss.cpu()) - lref) <= 1e-5 * abs(lref)
    assert np.abs(g - gref).max() <= 1e-4 * np.abs(gref).max()


@pytest.mark.parametrize("wd", [0.0, 0.01])
def test_mlp_adam_step(fmm, wd):
    rng = np.random.default_rng(3)
    npar = M.n_params(92)
    theta = rng.normal(0, 0.1, npar).astype(np.float32)
    m = rng.normal(0, 0.01, npar).astype(np.float32)
    v = rng.uniform(0, 1e-3, npar).astype(np.float32)
    g = rng.normal(0, 0.05, npar).astype(np.float32)
    tp, tm, tv = _dev(theta), _dev(m), _dev(v)
    fmm.mlp_adam(tp, tm, tv, _dev(g), step=5, lr=1e-3, weight_decay=wd)
    # the reference with the kernel's FP32 constants (0.9f, 0.999f, 1e-8f are
    # not the decimal values), so only the rounding of the update remains
    f32 = lambda v_: float(np.float32(v_))
    rt, rm, rv = M.adam_step(theta.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                             g.astype(np.float64), 5, 1e-3, b1=f32(0.9), b2=f32(0.999), eps=f32(1e-8),
                             wd=f32(wd))
    # FP32 rounding of each update, measured against the size of its terms
    eps = 2.0 ** -24
    gm, gv, gp = (t.cpu().numpy().astype(np.float64) for t in (tm, tv, tp))
    ge = np.abs(g.astype(np.float64)) + f32(wd) * np.abs(theta.astype(np.float64))  # |g + wd theta| bound
    assert np.all(np.abs(gm - rm) <= 4 * eps * (0.9 * np.abs(m) + 0.1 * ge))
    assert np.all(np.abs(gv - rv) <= 4 * eps * (0.999 * v + 0.001 * ge ** 2))
    step_size = np.abs(theta.astype(np.float64) - rt)
    assert np.all(np.abs(gp - rt) <= 4 * eps * np.abs(theta) + 1e-4 * step_size)


def test_mlp_training_reduces_loss(fmm):
    # a few hundred Adam steps on a smooth target must cut the loss
    rng = np.random.default_rng(21)
    d_in, batch = 92, 256
    X = rng.normal(0, 1, (batch, d_in)).astype(np.float32)
    w = rng.normal(0, 0.2, (d_in, 3))
    Y = np.tanh(X @ w).astype(np.float32)
    npar = fmm.mlp_nparams(d_in)
    shapes = M.layer_shapes(d_in)
    theta = np.concatenate([np.concatenate([rng.normal(0, 1 / math.sqrt(i), o * i), np.zeros(o)])
                            for o, i in shapes]).astype(np.float32)
    assert theta.size == npar
    tp, tm, tv = _dev(theta), torch.zeros(npar, device="cuda"), torch.zeros(npar, device="cuda")
    Xd, Yd = _dev(X), _dev(Y)
    _, l0 = fmm.mlp_grad(tp, Xd, Yd)
    l0 = float(l0.cpu())
    for step in range(1, 301):
        g, _ = fmm.mlp_grad(tp, Xd, Yd)
        fmm.mlp_adam(tp, tm, tv, g, step=step, lr=3e-3)
    _, l1 = fmm.mlp_grad(tp, Xd, Yd)
    assert float(l1.cpu()) < 0.1 * l0


def test_shipped_weights_decode_like_the_oracle(fmm):
    # the trained blob that ships with the package: right size, the network
    # decides inside its range, and the decision equals the oracle's decoding
    # of the network's own outputs
    from paper_1006_2269_amd import selector

    blob = selector.load_weights()
    assert blob is not None and blob.size == S.HEADER + fmm.mlp_nparams(S.NFEAT)
    assert np.all(np.isfinite(blob))
    ps = LAYOUTS["mixed_1m_scaled_50k"]
    x, y = _dev(ps.x), _dev(ps.y)
    for tol in (1e-4, 1e-6):
        L, p, th, net = fmm.select(x, y, tol, _dev(blob))
        feat = fmm.features(x, y, tol).cpu().numpy()
        xin = (feat - blob[:S.NFEAT]) * blob[S.NFEAT:2 * S.NFEAT]
        out = fmm.mlp_forward(_dev(blob[S.HEADER:]), _dev(xin[None, :])).cpu().numpy()[0]
        assert net is True
        assert (L, p, th, net) == S.decide(out, blob, ps.n, tol)
        assert 1 <= L <= S.levels_max(ps.n) and 1 <= p <= 63 and th in S.THETAS


def _tree_arrays(fmm):
    torch.cuda.synchronize()
    return (fmm.perm().cpu().numpy().copy(), fmm.leaf_start().cpu().numpy().copy(),
            fmm.rects().cpu().numpy().view(np.int64).copy())


@pytest.mark.parametrize("name", sorted(LAYOUTS))
@pytest.mark.parametrize("with_net", [True, False])
def test_select_build_tree_equals_separate_calls(fmm, name, with_net):
    # one call = select, then build_tree at the selected level count: the same
    # decision and a bit-identical tree (grid_64x64 and coincident_100 have
    # digits on which all keys agree, which build_tree skips and the combined
    # call sorts anyway)
    from paper_1006_2269_amd import selector

    ps = LAYOUTS[name]
    tol = 1e-6
    w = selector.weights_tensor(torch.device("cuda", 0)) if with_net else None
    if with_net and w is None:
        pytest.skip("no shipped weights")
    _announce("select_build_tree", name, ps.n, with_net)
    x, y = _dev(ps.x), _dev(ps.y)
    dec = fmm.select(x, y, tol, w)
    fmm.build_tree(x, y, dec[0])
    ref = _tree_arrays(fmm)
    got_dec = fmm.select_build_tree(x, y, tol, w)
    assert got_dec == dec
    for a, b in zip(_tree_arrays(fmm), ref):
        np.testing.assert_array_equal(a, b)


def test_select_build_tree_then_evaluate(fmm):
    # the rest of the path runs on the combined call's tree exactly as on
    # build_tree's (binary64 potentials bit-identical)
    ps = LAYOUTS["mixed_1m_scaled_50k"]
    _announce("select_build_tree evaluate", ps.n)
    x, y, q = _dev(ps.x), _dev(ps.y), _dev(ps.q)
    L, p, th, _ = fmm.select(x, y, 1e-6)
    fmm.build_tree(x, y, L)
    fmm.connectivity(th)
    ref = fmm.evaluate(q, p, "fp64").cpu().numpy()
    assert fmm.select_build_tree(x, y, 1e-6) == (L, p, th, False)
    fmm.connectivity(th)
    np.testing.assert_array_equal(fmm.evaluate(q, p, "fp64").cpu().numpy(), ref)


def test_select_build_tree_rejects_bad_input(fmm):
    from paper_1006_2269_amd.fmm import FMM2DError

    ps = LAYOUTS["uniform_10k"]
    x, y = ps.x.copy(), ps.y.copy()
    fmm.build_tree(_dev(x), _dev(y), 4)
    fmm.connectivity(0.5)
    x[123] = np.nan
    _announce("select_build_tree nan")
    with pytest.raises(FMM2DError):
        fmm.select_build_tree(_dev(x), _dev(y), 1e-6)
    # the previous tree is given up: nothing to connect until a tree is built
    with pytest.raises(FMM2DError):
        fmm.connectivity(0.5)
    L, p, th, _ = fmm.select_build_tree(_dev(ps.x), _dev(ps.y), 1e-6)
    fmm.connectivity(th)
    phi = fmm.evaluate(_dev(ps.q), p, "fp64").cpu().numpy()
    assert np.all(np.isfinite(phi))
