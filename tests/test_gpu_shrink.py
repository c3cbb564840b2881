"""GPU parity of the shrink-to-points tree option (each box's ball drawn
around its points' bounding box) against the CPU oracle's `shrink`.

* Geometry bit-exact (the bounding boxes are exact min / max, the centre and
  half diagonal single rounded operations on both sides); the tiling
  rectangles stay as built.
* Lists bit-exact on the shrunk balls, plain and with the structural options.
* Binary64 potentials within 1e-12 of the oracle FMM on the same tree and
  lists; reduced modes within their tolerances of the direct sum.
* Switching the option off again restores the tiling balls.
"""
import numpy as np
import pytest

from tests.gpu_cases import TREE_CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

VFLAG = 1 << 30


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_2269_amd.fmm import FMM2D

    ctx = FMM2D(0)
    ctx.set_tree_options(shrink=True)
    yield ctx
    ctx.close()


def _announce(*a):
    print("[case]", *a, flush=True)


GEOM_CASES = ["uniform_1k_L3", "ties_3k_L4", "grid_L4", "ragged_4pow5_plus1", "duplicates_4k_L4",
              "vertical_2k_L3", "scales_3k_L4", "negzero_2k_L4", "single_box_L0", "clustered_scaled_20k_L6",
              "mixed_scaled_20k_L6", "ring_scaled_20k_L6"]
EVAL_CASES = ["clustered_scaled_20k_L6", "mixed_scaled_20k_L6", "ring_scaled_20k_L6", "duplicates_4k_L4",
              "uniform_10k_L5", "single_box_L0"]


def _oracle(orc, ps, L):
    t = orc.tree(ps.x, ps.y, L)
    return t, orc.shrink(t, ps.x, ps.y)


def _oracle_lists(orc, ts, theta, opt):
    if opt == "plain":
        return orc.lists(ts, theta)
    return orc.lists_opt(ts, theta, parent=True, swap_levels=range(1, ts.levels + 1))


@pytest.mark.parametrize("case", GEOM_CASES)
def test_shrink_geometry_bit_exact(fmm, orc, case):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("shrink geometry", case, ps.n, L)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    t, ts = _oracle(orc, ps, L)
    geom = fmm.geometry().cpu().numpy()
    rects = fmm.rects().cpu().numpy()
    assert np.array_equal(geom[:, :3], ts.geom)
    assert np.array_equal(geom[:, 3], np.where(ts.geom[:, 2] > 0, ts.geom[:, 2], 1.0))
    assert np.array_equal(rects, t.rects)


@pytest.mark.parametrize("case", GEOM_CASES)
@pytest.mark.parametrize("opt", ["plain", "all"])
@pytest.mark.parametrize("theta", [0.5, 0.35, 0.7])
def test_shrink_lists_bit_exact(fmm, orc, case, opt, theta):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("shrink lists", case, ps.n, L, opt, theta)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    if opt == "plain":
        fmm.connectivity(theta)
    else:
        fmm.connectivity(theta, parent=True, swap="all")
    ls = _oracle_lists(orc, _oracle(orc, ps, L)[1], theta, opt)
    torch.cuda.synchronize()
    for l in range(L + 1):
        sp, si, wp, wi = (a.cpu().numpy().astype(np.int64) for a in fmm.lists(l))
        assert np.array_equal(si, ls.sidx[l]) and np.array_equal(sp, ls.sptr[l])
        if opt == "plain":
            assert np.array_equal(wi, ls.widx[l]) and np.array_equal(wp, ls.wptr[l])
            continue
        xp, xi = (a.cpu().numpy().astype(np.int64) for a in fmm.xlists(l))
        flagged = (wi & VFLAG) != 0
        assert np.array_equal(wi[~flagged], ls.widx[l])
        assert np.array_equal(wi[flagged] & (VFLAG - 1), ls.vidx[l])
        assert np.array_equal(np.diff(wp), np.diff(ls.wptr[l]) + np.diff(ls.vptr[l]))
        assert np.array_equal(xi, ls.xidx[l]) and np.array_equal(xp, ls.xptr[l])


@pytest.mark.parametrize("case", EVAL_CASES)
@pytest.mark.parametrize("opt", ["plain", "all"])
@pytest.mark.parametrize("p", [6, 20])
def test_shrink_fp64_matches_oracle_fmm(fmm, orc, case, opt, p):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("shrink fp64", case, ps.n, L, opt, p)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    if opt == "plain":
        fmm.connectivity(0.5)
    else:
        fmm.connectivity(0.5, parent=True, swap="all")
    phi = fmm.evaluate(_dev(ps.q), p, "fp64")
    _, ts = _oracle(orc, ps, L)
    ls = _oracle_lists(orc, ts, 0.5, opt)
    if opt == "plain":
        ref = orc.fmm_eval(ps.x, ps.y, ps.q, ts, ls, p)
    else:
        ref = orc.fmm_eval_opt(ps.x, ps.y, ps.q, ts, ls, p)
    torch.cuda.synchronize()
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("case", ["clustered_scaled_20k_L6", "ring_scaled_20k_L6", "uniform_10k_L5"])
@pytest.mark.parametrize("mode,tol", [("fp32", 2e-5), ("fp32_acc64", 2e-5), ("bf16x3", 1e-3)])
def test_shrink_reduced_modes(fmm, orc, case, mode, tol):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("shrink reduced", case, ps.n, L, mode)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5, parent=True, swap="all")
    phi = fmm.evaluate(_dev(ps.q), 20, mode)
    ex = orc.direct(ps.x, ps.y, ps.q)
    torch.cuda.synchronize()
    e, _ = orc.rel_errors(phi.cpu().numpy(), ex)
    assert e <= tol


def test_shrink_off_restores_tiling_balls(orc):
    from paper_1006_2269_amd.fmm import FMM2D

    maker, L = TREE_CASES["clustered_scaled_20k_L6"]
    ps = maker()
    _announce("shrink toggle", ps.n, L)
    t, ts = _oracle(orc, ps, L)
    with FMM2D(0) as ctx:
        x, y, q = _dev(ps.x), _dev(ps.y), _dev(ps.q)
        ctx.set_tree_options(shrink=True)
        ctx.build_tree(x, y, L)
        assert np.array_equal(ctx.geometry().cpu().numpy()[:, :3], ts.geom)
        ctx.set_tree_options(shrink=False)
        ctx.build_tree(x, y, L)
        assert np.array_equal(ctx.geometry().cpu().numpy()[:, :3], t.geom)
        ctx.connectivity(0.5)
        phi = ctx.evaluate(q, 12, "fp64")
        ref = orc.fmm(ps.x, ps.y, ps.q, L, 12, 0.5)
        torch.cuda.synchronize()
        assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
        from paper_1006_2269_amd import _capi

        assert ctx._lib.fmm2d_set_tree_options(ctx._h, 8) == _capi.EINVAL
