"""GPU parity of the gradient (field) evaluation against the oracle FMM
with the same tree, lists and order, binary64: 1e-12 of the largest
component."""
import sys

import numpy as np
import pytest
import torch

from tests.gpu_cases import TREE_CASES

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


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


# leaves of 16, 125, 7, 50, 63 and 32 points; coincident points; a collinear
# set; a one-box tree
FIELD_CASES = ["uniform_1k_L3", "uniform_2000_L2", "clustered_scaled_30k_L6", "uniform_3200_L3",
               "duplicates_4k_L3", "vertical_2k_L3", "single_box_L0", "ring_scaled_20k_L6"]


@pytest.mark.parametrize("case", FIELD_CASES)
@pytest.mark.parametrize("p", [3, 12, 17])
def test_field_matches_oracle_fmm(fmm, orc, case, p):
    maker, L = TREE_CASES[case]
    ps = maker()
    _announce("field", case, ps.n, L, p)
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5)
    phi, gx, gy = (a.cpu().numpy() for a in fmm.evaluate_field(_dev(ps.q), p, "fp64"))
    rphi, rgx, rgy = orc.fmm_field(ps.x, ps.y, ps.q, L, p, 0.5)
    scale = max(np.abs(rgx).max(), np.abs(rgy).max())
    assert np.all(np.isfinite(gx)) and np.all(np.isfinite(gy))
    assert np.abs(gx - rgx).max() <= 1e-12 * scale
    assert np.abs(gy - rgy).max() <= 1e-12 * scale
    # the potential is the one fmm2d_evaluate gives
    np.testing.assert_array_equal(phi, fmm.evaluate(_dev(ps.q), p, "fp64").cpu().numpy())


def test_field_needs_binary64(fmm):
    from paper_1006_2269_amd.fmm import FMM2DError

    maker, L = TREE_CASES["uniform_1k_L3"]
    ps = maker()
    fmm.build_tree(_dev(ps.x), _dev(ps.y), L)
    fmm.connectivity(0.5)
    with pytest.raises(FMM2DError):
        fmm.evaluate_field(_dev(ps.q), 12, "fp32")


@pytest.mark.parametrize("case", ["uniform_10k_L5", "duplicates_4k_L4", "clustered_scaled_30k_L6"])
def test_direct_field_matches_oracle(fmm, orc, case):
    ps = TREE_CASES[case][0]()
    rng = np.random.default_rng(17)
    t = rng.choice(ps.n, min(ps.n, 700), replace=False).astype(np.int64)
    _announce("direct_field", case, ps.n)
    gx, gy = (a.cpu().numpy() for a in fmm.direct_field(_dev(ps.x), _dev(ps.y), _dev(ps.q), _dev(t)))
    rx, ry = orc.direct_field(ps.x, ps.y, ps.q, t)
    scale = max(np.abs(rx).max(), np.abs(ry).max())
    # both compensated: they differ in the summation order only
    assert np.abs(gx - rx).max() <= 1e-13 * scale
    assert np.abs(gy - ry).max() <= 1e-13 * scale
