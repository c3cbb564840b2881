"""Device memory through the caller's allocator (fmm2d_create's callbacks).

* With PyTorch's caching allocator behind the callbacks, every byte the
  library holds is a tensor the binding keeps, and the potentials equal those
  of a context that calls hipMalloc itself, bit for bit.
* An allocator that refuses makes the failing stage return FMM2D_ENOMEM;
  earlier stages stay valid, and once memory is available again the same
  context gives the oracle's tree, lists and binary64 potentials.
* Everything handed out is handed back by fmm2d_destroy.
"""
import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _path(ctx, ps, L, p, mode, theta=0.5):
    ctx.build_tree(_dev(ps.x), _dev(ps.y), L)
    ctx.connectivity(theta)
    out = ctx.evaluate(_dev(ps.q), p, mode)
    torch.cuda.synchronize()
    return out.cpu().numpy()


@pytest.mark.parametrize("mode", ["fp64", "fp32_acc64"])
def test_torch_allocator_same_results_as_hipmalloc(mode):
    from paper_1006_2269_amd.fmm import FMM2D

    ps = W.mixed_1m(scale=0.02)
    print("[case] allocator parity", mode, ps.n, flush=True)
    with FMM2D(0, allocator="hip") as a, FMM2D(0, allocator="torch") as b:
        ra = _path(a, ps, 5, 14, mode)
        rb = _path(b, ps, 5, 14, mode)
        assert b.allocator.bytes_held() > 0
        assert np.array_equal(ra.view(np.int64), rb.view(np.int64))


def test_refused_allocations_report_enomem_and_recover(orc):
    from paper_1006_2269_amd.fmm import FMM2D, FMM2DError

    ps = W.clustered_10m(scale=0.002)
    L, p, theta = 5, 12, 0.5
    ref_tree = orc.tree(ps.x, ps.y, L)
    ref_ls = orc.lists(ref_tree, theta)
    ref = orc.fmm_eval(ps.x, ps.y, ps.q, ref_tree, ref_ls, p)
    x, y, q = _dev(ps.x), _dev(ps.y), _dev(ps.q)
    print("[case] refused allocations", ps.n, flush=True)
    ctx = FMM2D(0)
    al = ctx.allocator
    # build_tree on a fresh context needs memory: refuse the first request
    al.refuse_after = 0
    with pytest.raises(FMM2DError) as e:
        ctx.build_tree(x, y, L)
    assert e.value.code == -2
    with pytest.raises(FMM2DError) as e:
        ctx.connectivity(theta)
    assert e.value.code == -4  # no tree
    al.refuse_after = None
    ctx.build_tree(x, y, L)
    # connectivity refused at its first, then at a later allocation: each time
    # ENOMEM, the tree kept, the lists discarded
    for k in (0, 3):
        al.refuse_after = k
        with pytest.raises(FMM2DError) as e:
            ctx.connectivity(theta)
        assert e.value.code == -2
        with pytest.raises(FMM2DError) as e:
            ctx.evaluate(q, p, "fp64")
        assert e.value.code == -4  # lists discarded
        al.refuse_after = None
    torch.cuda.synchronize()
    assert np.array_equal(ctx.perm().cpu().numpy().astype(np.int64), ref_tree.perm)
    ctx.connectivity(theta)
    for l in range(L + 1):
        sp, si, wp, wi = (t.cpu().numpy().astype(np.int64) for t in ctx.lists(l))
        assert np.array_equal(si, ref_ls.sidx[l]) and np.array_equal(wi, ref_ls.widx[l])
    # evaluate refused: ENOMEM, then the same context evaluates
    al.refuse_after = 0
    with pytest.raises(FMM2DError) as e:
        ctx.evaluate(q, p + 3, "fp64")
    assert e.value.code == -2
    al.refuse_after = None
    phi = ctx.evaluate(q, p, "fp64")
    torch.cuda.synchronize()
    got = phi.cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    ctx.close()
    assert al.bytes_held() == 0
