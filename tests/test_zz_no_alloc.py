"""fmm2d_direct_noalloc: the judge on the library's fixed device array.

Called through the C ABI on a fresh context whose allocator counts every
request, it must allocate nothing and give the same values as fmm2d_direct
(the same kernels: bit for bit), on two calls in a row, the second with
fewer sources and targets (the array keeps the first call's contents).
Sizes beyond the array and target indices out of range are refused.
"""
import ctypes

import numpy as np
import pytest

from paper_1006_2269_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_direct_noalloc_matches_direct_and_allocates_nothing():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1006_2269_amd.fmm import FMM2D, FMM2DError

    ref_ctx = FMM2D(0)
    ctx = FMM2D(0)
    ctx.allocator.refuse_after = 0   # any allocation request by the library would fail the call
    lib = ctx._lib
    for n, m, seed in ((200_000, 3000, 31), (5_000, 700, 32)):
        ps = W.mixed_1m(scale=n / 1e6, seed=1002 + seed)
        x, y, q = _dev(ps.x), _dev(ps.y), _dev(ps.q)
        tg = _dev(W.sample_targets(ps.n, m, seed=seed))
        print("[case] direct_noalloc n=%d m=%d" % (ps.n, m), flush=True)
        out = torch.full((m,), float("nan"), dtype=torch.float64, device="cuda")
        rc = lib.fmm2d_direct_noalloc(ctx._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                      ctypes.c_void_p(q.data_ptr()), ps.n, ctypes.c_void_p(tg.data_ptr()), m,
                                      ctypes.c_void_p(out.data_ptr()))
        assert rc == 0, lib.fmm2d_last_error(ctx._h)
        ref = ref_ctx.direct(x, y, q, tg)
        torch.cuda.synchronize()
        a, b = out.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a.view(np.int64), b.view(np.int64))
    assert ctx.allocator.bytes_held() == 0 and not ctx.allocator.blocks
    # refused sizes and indices; the context is still usable afterwards
    big = torch.zeros(262145, dtype=torch.int64, device="cuda")
    outb = torch.empty(262145, dtype=torch.float64, device="cuda")
    with pytest.raises(FMM2DError) as e:
        ctx.direct_noalloc(x, y, q, big, outb)
    assert e.value.code == -1
    bad = torch.tensor([0, ps.n], dtype=torch.int64, device="cuda")
    with pytest.raises(FMM2DError) as e:
        ctx.direct_noalloc(x, y, q, bad, outb)
    assert e.value.code == -1
    ok = ctx.direct_noalloc(x, y, q, tg, torch.empty(m, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert np.array_equal(ok.cpu().numpy().view(np.int64), b.view(np.int64))
    ctx.close()
    ref_ctx.close()
