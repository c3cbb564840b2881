"""GPU parity through the C ABI against the CPU oracle.

Tree (permutation, leaf offsets, rectangles) and interaction lists must match
bit for bit; binary64 potentials must match the oracle FMM to 1e-12 relative
(normwise, e_inf); the direct-sum judge must match the oracle's direct sum.
"""
import math
import sys

import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W
from tests.gpu_cases import TREE_CASES

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.fixture(scope="module")
def fmm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_2269_amd.fmm import FMM2D

    ctx = FMM2D(0)
    yield ctx
    ctx.close()


# Cases held off the GPU: none.  (The clustered 20k-point input at theta = 1/2
# was held off after an interim list build, never committed, faulted on it;
# the current build's indices on that input are replayed on the CPU in
# test_lists_index_model.py and stay in bounds through both pool regrowths.)
FAULTED = set()


def _skip_faulted(case, theta):
    if (case, theta) in FAULTED:
        pytest.skip("connectivity(theta=%.2f) on %s is held off the GPU" % (theta, case))


def _announce(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("case", sorted(TREE_CASES))
def test_tree_bit_exact(fmm, orc, case):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce(case, ps.n, L)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    t = orc.tree(ps.x, ps.y, L)
    torch.cuda.synchronize()
    assert np.array_equal(fmm.perm().cpu().numpy().astype(np.int64), t.perm)
    assert np.array_equal(fmm.leaf_start().cpu().numpy().astype(np.int64), t.leaf_start)
    got = fmm.rects().cpu().numpy()
    assert np.array_equal(got.view(np.int64), t.rects.view(np.int64))


@pytest.mark.parametrize("case", sorted(TREE_CASES))
@pytest.mark.parametrize("theta", [0.5, 0.3, 0.75])
def test_lists_bit_exact(fmm, orc, case, theta):
    _skip_faulted(case, theta)
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce(case, ps.n, L, theta)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(theta)
    ls = orc.lists(orc.tree(ps.x, ps.y, L), theta)
    for l in range(L + 1):
        sp, si, wp, wi = (a.cpu().numpy().astype(np.int64) for a in fmm.lists(l))
        assert np.array_equal(sp, ls.sptr[l]), l
        assert np.array_equal(si, ls.sidx[l]), l
        assert np.array_equal(wp, ls.wptr[l]), l
        assert np.array_equal(wi, ls.widx[l]), l


FP64_CASES = ["uniform_1k_L3", "clustered_scaled_30k_L6", "ties_3k_L4", "ragged_4pow5_plus1", "duplicates_4k_L4", "vertical_2k_L3",
              "scales_3k_L4", "single_box_L0", "uniform_10k_L5", "mixed_scaled_20k_L6",
              "clustered_scaled_20k_L6", "ring_scaled_20k_L6",
              # leaves of 20, 50, 63 and 125 points (multipoles by one wavefront per leaf for p + 1 <= 16)
              "uniform_20k_L5", "uniform_3200_L3", "duplicates_4k_L3", "uniform_2000_L2"]


@pytest.mark.parametrize("case", FP64_CASES)
@pytest.mark.parametrize("p", [3, 12, 15, 17, 40])
def test_fp64_potentials_match_oracle_fmm(fmm, orc, case, p):
    theta = 0.5
    _skip_faulted(case, theta)
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce(case, ps.n, L, p)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(theta)
    phi = fmm.evaluate(_dev(ps.q), p, "fp64").cpu().numpy()
    ref = orc.fmm(ps.x, ps.y, ps.q, L, p, theta)
    scale = np.abs(ref).max()
    assert np.all(np.isfinite(phi))
    assert np.abs(phi - ref).max() <= 1e-12 * scale


@pytest.mark.parametrize("case", ["uniform_10k_L5", "clustered_scaled_20k_L6", "duplicates_4k_L4", "scales_3k_L4"])
def test_direct_judge_matches_oracle(fmm, orc, case):
    maker, _ = TREE_CASES[case]
    ps = maker()
    _announce(case, ps.n)
    tg = W.sample_targets(ps.n, 300, seed=5)
    got = fmm.direct(_dev(ps.x), _dev(ps.y), _dev(ps.q), _dev(tg)).cpu().numpy()
    ref = orc.direct(ps.x, ps.y, ps.q, tg)
    assert np.abs(got - ref).max() <= 1e-14 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("mode,tol", [("fp32", 2e-5), ("fp32_acc64", 2e-5), ("bf16x3", 1e-3)])
@pytest.mark.parametrize("case", ["uniform_10k_L5", "clustered_scaled_20k_L6", "ring_scaled_20k_L6",
                                  "duplicates_4k_L4", "mixed_scaled_20k_L6", "uniform_20k_L5", "uniform_3200_L3",
                                  "uniform_2500_L3", "uniform_2900_L3", "duplicates_4k_L3"])
def test_reduced_modes_error(fmm, orc, case, mode, tol):
    _skip_faulted(case, 0.5)
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce(case, mode)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5)
    phi = fmm.evaluate(_dev(ps.q), 20, mode).cpu().numpy()
    ex = orc.direct(ps.x, ps.y, ps.q)
    e, _ = orc.rel_errors(phi, ex)
    assert e <= tol


@pytest.mark.parametrize("mode", ["fp32", "fp32_acc64"])
def test_reduced_modes_collinear(fmm, orc, mode):
    # Points on one vertical line: the FP32 modes keep about 6e-5 here (the
    # same before and after the near field took each leaf pair once); binary64
    # reaches 2e-10.  Tracked with its own bound.
    maker, L = TREE_CASES["vertical_2k_L3"]
    ps = maker()
    _announce("vertical_2k_L3", mode)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5)
    phi = fmm.evaluate(_dev(ps.q), 20, mode).cpu().numpy()
    e, _ = orc.rel_errors(phi, orc.direct(ps.x, ps.y, ps.q))
    assert e <= 1e-4


@pytest.mark.parametrize("p", [12, 20])
def test_bf16x3_product_differs_from_fp32(fmm, p):
    # the BF16X3 M2L keeps about 16 bits per product (the dropped lo x lo term
    # is ~2^-16 relative), FP32 about 24: against the binary64 result its
    # error must be larger than FP32's yet within 1e-3 (one and two 16-wide
    # coefficient tiles: p + 1 = 13 and 21)
    maker, L = TREE_CASES["uniform_10k_L5"]
    ps = maker()
    _announce("bf16x3 vs fp32", p)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5)
    q = _dev(ps.q)
    ref = fmm.evaluate(q, p, "fp64").cpu().numpy()
    e32 = np.abs(fmm.evaluate(q, p, "fp32").cpu().numpy() - ref).max() / np.abs(ref).max()
    eb = np.abs(fmm.evaluate(q, p, "bf16x3").cpu().numpy() - ref).max() / np.abs(ref).max()
    assert eb <= 1e-3
    assert eb > 1.5 * e32


def test_call_order_and_argument_errors(fmm):
    from paper_1006_2269_amd.fmm import FMM2D, FMM2DError

    ctx = FMM2D(0)
    q = torch.zeros(16, dtype=torch.float64, device="cuda")
    with pytest.raises(FMM2DError) as e:
        ctx.connectivity(0.5)
    assert e.value.code == -4
    with pytest.raises(FMM2DError) as e:
        ctx.evaluate(q, 5)
    assert e.value.code == -4
    x = torch.rand(16, dtype=torch.float64, device="cuda")
    with pytest.raises(FMM2DError) as e:
        ctx.build_tree(x, x, 3)   # 16 < 4^3
    assert e.value.code == -1
    bad = x.clone()
    bad[3] = float("nan")
    with pytest.raises(FMM2DError) as e:
        ctx.build_tree(bad, x, 1)
    assert e.value.code == -1
    ctx.build_tree(x, x.flip(0).contiguous(), 1)
    for th in (0.0, 1.0, -0.5, float("nan")):
        with pytest.raises(FMM2DError):
            ctx.connectivity(th)
    ctx.connectivity(0.5)
    for p in (0, 64):
        with pytest.raises(FMM2DError):
            ctx.evaluate(q, p)
    with pytest.raises(FMM2DError):
        ctx.evaluate(q, 5, "fp64") if False else ctx._check(ctx._lib.fmm2d_evaluate(ctx._h, q.data_ptr(), 5, 9, q.data_ptr()))
    tg = torch.tensor([0, 16], dtype=torch.int64, device="cuda")
    with pytest.raises(FMM2DError):
        ctx.direct(x, x, q, tg)
    ctx.close()


def test_list_limit_fails_cleanly(orc, monkeypatch):
    # A level whose strong or weak list would exceed the entry limit is
    # refused with ECAPACITY before anything is written; the limit is lowered
    # from the host so the path runs on a small input.
    from paper_1006_2269_amd.fmm import FMM2D, FMM2DError

    ps = W.uniform(3000, seed=3)
    monkeypatch.setenv("FMM2D_LIST_LIMIT", "500")
    ctx = FMM2D(0)
    ctx.build_tree(_dev(ps.x), _dev(ps.y), 4)
    with pytest.raises(FMM2DError) as e:
        ctx.connectivity(0.5)
    assert e.value.code == -5 and "exceeds 500 entries" in str(e.value)
    with pytest.raises(FMM2DError) as e:
        ctx.evaluate(_dev(ps.q), 5)
    assert e.value.code == -4
    ctx.close()
    monkeypatch.delenv("FMM2D_LIST_LIMIT")
    ctx = FMM2D(0)
    ctx.build_tree(_dev(ps.x), _dev(ps.y), 4)
    ctx.connectivity(0.5)
    ls = orc.lists(orc.tree(ps.x, ps.y, 4), 0.5)
    sp, si, wp, wi = (a.cpu().numpy().astype(np.int64) for a in ctx.lists(4))
    assert np.array_equal(wi, ls.widx[4]) and np.array_equal(si, ls.sidx[4])
    ctx.close()


def test_call_orders_with_second_stream(fmm, orc):
    # Work queued on the library's second stream (transposed positions after
    # connectivity, the near field during evaluate, the selector during the
    # combined call) must be ordered against every later call: trees and
    # lists rebuilt without an evaluate in between, evaluates back to back,
    # the combined call right after connectivity.  Each result against the
    # oracle FMM in binary64.
    cases = ["uniform_3200_L3", "uniform_20k_L5", "duplicates_4k_L3"]
    pts = {c: TREE_CASES[c][0]() for c in cases}
    ref = {}
    for c in cases:
        ps, L = pts[c], TREE_CASES[c][1]
        ref[c] = orc.fmm(ps.x, ps.y, ps.q, L, 12, 0.5)

    def check(c, phi):
        scale = np.abs(ref[c]).max()
        assert np.abs(phi - ref[c]).max() <= 1e-12 * scale, c

    a, b, d = cases
    _announce("call orders", *cases)
    # connectivity with no evaluate, then another tree and its lists
    fmm.build_tree(_dev(pts[a].x), _dev(pts[a].y), TREE_CASES[a][1])
    fmm.connectivity(0.5)
    fmm.build_tree(_dev(pts[b].x), _dev(pts[b].y), TREE_CASES[b][1])
    fmm.connectivity(0.5)
    # the reduced mode queues the pair-once near field (20-point leaves) on
    # the second stream; then binary64 on the same lists, twice
    fmm.evaluate(_dev(pts[b].q), 12, "fp32_acc64")
    check(b, fmm.evaluate(_dev(pts[b].q), 12, "fp64").cpu().numpy())
    check(b, fmm.evaluate(_dev(pts[b].q), 12, "fp64").cpu().numpy())
    # the combined call right after a connectivity, then the rule's tree
    # replaced by the case's own level count
    fmm.connectivity(0.5)
    fmm.select_build_tree(_dev(pts[d].x), _dev(pts[d].y), 1e-6)
    fmm.build_tree(_dev(pts[d].x), _dev(pts[d].y), TREE_CASES[d][1])
    fmm.connectivity(0.5)
    fmm.evaluate(_dev(pts[d].q), 12, "fp32")
    check(d, fmm.evaluate(_dev(pts[d].q), 12, "fp64").cpu().numpy())
    # and back to the first case
    fmm.build_tree(_dev(pts[a].x), _dev(pts[a].y), TREE_CASES[a][1])
    fmm.connectivity(0.5)
    check(a, fmm.evaluate(_dev(pts[a].q), 12, "fp64").cpu().numpy())


@pytest.mark.parametrize("mode,tol", [("fp32", 2e-5), ("fp32_acc64", 2e-5), ("bf16x3", 1e-3)])
@pytest.mark.parametrize("per_leaf", [12, 24, 48, 100])
def test_reduced_modes_close_pair_in_sparse_leaf(fmm, orc, mode, tol, per_leaf):
    # Two distinct points 2^-19.5 R apart in one leaf of half diagonal R
    # (leaf sizes 12, 24, 48, 100 take the one-sided, both pair-once and the
    # large-leaf FP32 kernels).  Within a leaf only exact duplicates may be
    # masked: the pair's log r is resolved to |dlog r| <= d / (r - d), with
    # d = 2 sqrt2 2^-24 R the rounding of the two FP32 offsets; masking it
    # would cost |log r| ~ 15 at both points.
    L = 1
    g = np.random.default_rng(4242 + per_leaf)
    n = 4 * per_leaf
    x, y = g.random(n), g.random(n)
    q = g.uniform(-1.0, 1.0, n)
    x[0], y[0] = 0.2, 0.3
    q[0] = q[1] = 1.0
    r_pair = 4e-7
    x[1], y[1] = 0.2 + r_pair * math.cos(0.7), 0.3 + r_pair * math.sin(0.7)
    r_pair = math.hypot(x[1] - x[0], y[1] - y[0])
    t = orc.tree(x, y, L)
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(t.perm)] = np.arange(n)
    leaf = np.searchsorted(np.asarray(t.leaf_start), pos[:2], side="right") - 1
    assert leaf[0] == leaf[1], "the pair must share a leaf"
    R = float(np.asarray(t.geom)[orc.level_offset(L) + leaf[0], 2])
    assert 2.0 ** -21 * R < r_pair < 2.0 ** -19 * R  # resolvable in FP32, below the old self threshold
    _announce("close_pair", per_leaf, mode)
    fmm.build_tree(_dev(x), _dev(y), L)
    fmm.connectivity(0.5)
    phi = fmm.evaluate(_dev(q), 20, mode).cpu().numpy()
    ex = orc.direct(x, y, q)
    scale = np.abs(ex).max()
    d = 2.0 * math.sqrt(2.0) * 2.0 ** -24 * R
    bound = abs(q[1]) * d / (r_pair - d) + tol * scale
    err = np.abs(phi - ex)
    assert err[0] <= bound and err[1] <= bound, (err[:2], bound)
    assert err[2:].max() <= tol * scale


@pytest.mark.parametrize("mode", ["fp32", "fp32_acc64", "bf16x3"])
@pytest.mark.parametrize("s", [1e15, 1e-15])
def test_reduced_modes_scaled_inputs(fmm, orc, mode, s):
    # A uniform set scaled by s (root half-diagonal s / sqrt(2)): inside the
    # FP32 modes' range [2^-60, 2^56], so they run; the potentials shift by
    # log(s) sum q, the leaf-local offsets scale with s, and the normwise
    # error stays at the FP32 level of the unscaled set (its log terms are
    # larger in magnitude by |log s|, so the bound is 5x the unscaled 2e-5;
    # BF16X3 keeps its 1e-3)
    ps = W.uniform(3000, seed=41)
    x, y = ps.x * s, ps.y * s
    _announce("scaled", s, mode)
    fmm.build_tree(_dev(x), _dev(y), 4)
    fmm.connectivity(0.5)
    phi = fmm.evaluate(_dev(ps.q), 20, mode).cpu().numpy()
    e, _ = orc.rel_errors(phi, orc.direct(x, y, ps.q))
    assert e <= (1e-3 if mode == "bf16x3" else 1e-4)


@pytest.mark.parametrize("mode", ["fp32", "fp32_acc64", "bf16x3"])
def test_reduced_modes_refuse_out_of_range(fmm, orc, mode):
    # coordinates spanning 1e+-18 (beyond 2^56 for the root half-diagonal):
    # the FP32 modes refuse, binary64 evaluates
    from paper_1006_2269_amd.fmm import FMM2DError

    g = W.rng(43)
    n = 2000
    x = np.sign(g.uniform(-1, 1, n)) * 10.0 ** g.uniform(-18, 18, n)
    y = np.sign(g.uniform(-1, 1, n)) * 10.0 ** g.uniform(-18, 18, n)
    q = g.uniform(-1, 1, n)
    _announce("out of range", mode)
    fmm.build_tree(_dev(x), _dev(y), 3)
    fmm.connectivity(0.5)
    with pytest.raises(FMM2DError) as e:
        fmm.evaluate(_dev(q), 12, mode)
    assert e.value.code == -1 and "2^56" in str(e.value)
    phi = fmm.evaluate(_dev(q), 12, "fp64").cpu().numpy()
    ref = orc.fmm(x, y, q, 3, 12, 0.5)
    assert np.abs(phi - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("per_leaf", [12, 24, 48, 100])
@pytest.mark.parametrize("across", [False, True])
def test_acc64_two_part_differences_resolve_close_pairs(fmm, orc, per_leaf, across):
    # A pair 2^-30 R apart (R the leaf's half diagonal), in one leaf or in two
    # leaves across the x-median split line: far below what FP32 offsets
    # resolve (about 2^-24 R), so FP32_ACC64's differences in two FP32 parts
    # must carry it.  Masking or mis-resolving the pair would cost about
    # |log r| ~ 20 at both points; the two-part difference is accurate to
    # about 2^-23 of itself, its log to about 1e-6 absolute.
    L = 1
    g = np.random.default_rng(777 + per_leaf + 1000 * across)
    n = 4 * per_leaf
    h = n // 2 - 1
    x = np.concatenate([[0.5, 0.5], g.uniform(0.0, 0.49, h), g.uniform(0.51, 1.0, n - 2 - h)])
    y = np.concatenate([[0.3, 0.3], g.random(n - 2)])
    q = g.uniform(-1.0, 1.0, n)
    q[0] = q[1] = 1.0
    t = orc.tree(x, y, L)
    R = float(np.asarray(t.geom)[orc.level_offset(L):, 2].max())
    r_pair = 2.0 ** -30 * R
    if across:
        x[0], x[1] = 0.5 - r_pair / 2, 0.5 + r_pair / 2
    else:
        x[1], y[1] = x[0] + r_pair * math.cos(0.7), y[0] + r_pair * math.sin(0.7)
        x[0] -= 0.25  # both in the low-x half, away from the split line
        x[1] -= 0.25
    t = orc.tree(x, y, L)
    pos = np.empty(n, dtype=np.int64)
    pos[np.asarray(t.perm)] = np.arange(n)
    leaf = np.searchsorted(np.asarray(t.leaf_start), pos[:2], side="right") - 1
    assert (leaf[0] != leaf[1]) == across
    _announce("two-part differences", per_leaf, across)
    fmm.build_tree(_dev(x), _dev(y), L)
    fmm.connectivity(0.5)
    phi = fmm.evaluate(_dev(q), 20, "fp32_acc64").cpu().numpy()
    ex = orc.direct(x, y, q)
    err = np.abs(phi - ex)
    assert err[:2].max() <= 1e-4, err[:2]
    assert err.max() <= 2e-5 * np.abs(ex).max()


def test_acc64_below_the_fp32_offset_floor(fmm, orc):
    # A held-out selector layout (26438 points) whose clustered leaves hold
    # pairs far closer than their leaf size: at 5 levels the FP32 offsets
    # alone leave about 8e-6 of max |phi| (the reduced mode FP32 measures
    # that); the two-part differences of FP32_ACC64 meet 1e-6.
    ps = W.selector_layout(90155, 4.0, 7.0)
    assert ps.n == 26438
    _announce("acc64 floor layout", ps.n)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), 5)
    fmm.connectivity(0.5, parent=True, swap="all")
    q = _dev(ps.q)
    ex = orc.direct(ps.x, ps.y, ps.q)
    e64, _ = orc.rel_errors(fmm.evaluate(q, 20, "fp32_acc64").cpu().numpy(), ex)
    e32, _ = orc.rel_errors(fmm.evaluate(q, 20, "fp32").cpu().numpy(), ex)
    assert e64 <= 1e-6 < e32, (e64, e32)
