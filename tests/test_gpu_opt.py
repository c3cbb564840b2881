"""GPU parity of Section 4's structural optimisations (interaction via the
parent box; exchanged roles with P2L / M2P) against the CPU oracle.

* Lists bit-exact: S, W (parent entries flagged), X against the oracle's
  optimised lists, for the finest-level exchange of the paper, the exchange
  at every level, and the parent option alone, at theta in {0.35, 0.5, 0.7}.
* Binary64 potentials within 1e-12 of the oracle FMM on the same lists,
  across both P2L/M2P orders of magnitude (coarse levels hold thousands of
  points per box) and both M2L kernels (p + 1 <= 16 and above).
* Reduced modes within their tolerances of the oracle's direct sum.
"""
import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W
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
    yield ctx
    ctx.close()


def _announce(*a):
    print("[case]", *a, flush=True)


OPTS = {"paper": (True, "finest"), "all": (True, "all"), "swap_all": (False, "all"), "parent": (True, None)}
CASES = ["clustered_scaled_20k_L6", "clustered_scaled_30k_L6", "mixed_scaled_20k_L6", "ring_scaled_20k_L6",
         "duplicates_4k_L4", "scales_3k_L4", "uniform_3200_L3", "single_box_L0", "uniform_10k_L5"]


def _oracle_lists(orc, t, theta, opt):
    parent, swap = OPTS[opt]
    L = t.levels
    levels = {"finest": (L,), "all": tuple(range(1, L + 1)), None: ()}[swap]
    return orc.lists_opt(t, theta, parent=parent, swap_levels=levels)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("opt", sorted(OPTS))
@pytest.mark.parametrize("theta", [0.5, 0.35, 0.7])
def test_opt_lists_bit_exact(fmm, orc, case, opt, theta):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("opt lists", case, ps.n, L, opt, theta)
    parent, swap = OPTS[opt]
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(theta, parent=parent, swap=swap)
    ls = _oracle_lists(orc, orc.tree(ps.x, ps.y, L), theta, opt)
    torch.cuda.synchronize()
    for l in range(L + 1):
        sp, si, wp, wi = (a.cpu().numpy().astype(np.int64) for a in fmm.lists(l))
        xp, xi = (a.cpu().numpy().astype(np.int64) for a in fmm.xlists(l))
        assert np.array_equal(si, ls.sidx[l]) and np.array_equal(sp, ls.sptr[l])
        flagged = (wi & VFLAG) != 0
        assert np.array_equal(wi[~flagged], ls.widx[l])
        assert np.array_equal(wi[flagged] & (VFLAG - 1), ls.vidx[l])
        assert np.array_equal(np.diff(wp), np.diff(ls.wptr[l]) + np.diff(ls.vptr[l]))
        assert np.array_equal(xi, ls.xidx[l]) and np.array_equal(xp, ls.xptr[l])


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("opt", sorted(OPTS))
@pytest.mark.parametrize("p", [6, 15, 20])
def test_opt_fp64_matches_oracle_fmm(fmm, orc, case, opt, p):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("opt fp64", case, ps.n, L, opt, p)
    parent, swap = OPTS[opt]
    theta = 0.5
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(theta, parent=parent, swap=swap)
    phi = fmm.evaluate(_dev(ps.q), p, "fp64")
    t = orc.tree(ps.x, ps.y, L)
    ref = orc.fmm_eval_opt(ps.x, ps.y, ps.q, t, _oracle_lists(orc, t, theta, opt), p)
    torch.cuda.synchronize()
    got = phi.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("case", ["clustered_scaled_20k_L6", "mixed_scaled_20k_L6", "uniform_10k_L5"])
@pytest.mark.parametrize("mode,tol", [("fp32", 2e-5), ("fp32_acc64", 2e-5), ("bf16x3", 1e-3)])
def test_opt_reduced_modes(fmm, orc, case, mode, tol):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("opt reduced", case, ps.n, L, mode)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5, parent=True, swap="all")
    phi = fmm.evaluate(_dev(ps.q), 20, mode)
    ex = orc.direct(ps.x, ps.y, ps.q)
    torch.cuda.synchronize()
    e, _ = orc.rel_errors(phi.cpu().numpy(), ex)
    assert e <= tol


def test_opt_then_plain_lists(fmm, orc):
    # a context that built optimised lists builds the plain ones afterwards
    maker, L = TREE_CASES["clustered_scaled_20k_L6"]
    ps = maker()
    x, y, q = _dev(ps.x), _dev(ps.y), _dev(ps.q)
    fmm.build_tree(x, y, L)
    fmm.connectivity(0.5, parent=True, swap="all")
    fmm.evaluate(q, 12, "fp64")
    fmm.connectivity(0.5)
    phi = fmm.evaluate(q, 12, "fp64")
    ref = orc.fmm(ps.x, ps.y, ps.q, L, 12, 0.5)
    torch.cuda.synchronize()
    assert np.abs(phi.cpu().numpy() - ref).max() <= 1e-12 * np.abs(ref).max()
    for l in range(L + 1):
        xp, xi = fmm.xlists(l)
        assert xi.numel() == 0 and int(xp.abs().max()) == 0
