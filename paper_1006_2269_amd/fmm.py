"""Python binding of the fmm2d C ABI: argument marshalling only.

Every step runs in the HIP library; this module passes torch device tensors
(device memory and the current stream come from PyTorch) through ctypes.
"""
from __future__ import annotations

import ctypes

import torch

from . import _capi


class FMM2DError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("fmm2d error %d: %s" % (code, msg))
        self.code = code


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, device, name):
    if not isinstance(t, torch.Tensor) or t.dtype != dtype or t.device != device or not t.is_contiguous():
        raise TypeError("%s must be a contiguous %s tensor on %s" % (name, dtype, device))


class TorchAllocator:
    """Device memory of a context from PyTorch's caching allocator: each block
    is a uint8 tensor allocated on the context's stream and kept alive until
    the library hands it back (stream-ordered, as the allocator expects).
    ``refuse_after`` (tests) makes every allocation after that many more fail."""

    def __init__(self, device: torch.device, stream: torch.cuda.Stream):
        self.device = device
        self.stream = stream
        self.blocks = {}
        self.refuse_after = None
        self.c_alloc = _capi.ALLOC_FN(self._alloc)
        self.c_free = _capi.FREE_FN(self._free)

    def _alloc(self, nbytes, user):
        try:
            if self.refuse_after is not None:
                if self.refuse_after <= 0:
                    return None
                self.refuse_after -= 1
            with torch.cuda.stream(self.stream):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
            self.blocks[t.data_ptr()] = t
            return t.data_ptr()
        except Exception:  # out of memory: the library reports FMM2D_ENOMEM
            return None

    def _free(self, ptr, nbytes, user):
        self.blocks.pop(ptr, None)

    def bytes_held(self) -> int:
        return sum(t.numel() for t in self.blocks.values())


class FMM2D:
    """A context: one device, one stream, one tree and its lists.

    allocator="torch" (default): every device byte the library uses comes
    from PyTorch's caching allocator (``TorchAllocator``); "hip": the library
    calls hipMalloc itself."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None, allocator: str = "torch"):
        self._lib = _capi.load()
        self.device = torch.device("cuda", device)
        self._stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        if allocator == "torch":
            self.allocator = TorchAllocator(self.device, self._stream)
            fa, ff = self.allocator.c_alloc, self.allocator.c_free
        elif allocator == "hip":
            self.allocator = None
            fa, ff = None, None
        else:
            raise ValueError("allocator must be 'torch' or 'hip'")
        rc = self._lib.fmm2d_create(ctypes.byref(h), device, ctypes.c_void_p(self._stream.cuda_stream),
                                    ctypes.cast(fa, ctypes.c_void_p) if fa else None,
                                    ctypes.cast(ff, ctypes.c_void_p) if ff else None, None)
        if rc != 0:
            raise FMM2DError(rc, "fmm2d_create failed")
        self._h = h
        self.n = None
        self.levels = None

    # -- helpers ---------------------------------------------------------
    def _check(self, rc):
        if rc != 0:
            raise FMM2DError(rc, self._lib.fmm2d_last_error(self._h).decode())

    def close(self):
        if getattr(self, "_h", None):
            self._lib.fmm2d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    @property
    def stream(self):
        return self._stream

    def set_tree_options(self, shrink: bool = False):
        """Options of the trees built from now on: ``shrink`` draws each box's
        ball around its points (bounding box) instead of its tiling rectangle."""
        self._check(self._lib.fmm2d_set_tree_options(self._h, _capi.TREE_SHRINK if shrink else 0))

    # -- the three stages --------------------------------------------------
    def build_tree(self, x: torch.Tensor, y: torch.Tensor, levels: int):
        _require(x, torch.float64, self.device, "x")
        _require(y, torch.float64, self.device, "y")
        n = x.numel()
        if y.numel() != n:
            raise ValueError("x and y differ in length")
        self._check(self._lib.fmm2d_build_tree(self._h, _ptr(x), _ptr(y), n, int(levels)))
        self.n, self.levels = n, int(levels)

    def connectivity(self, theta: float, parent: bool = False, swap: str | None = None):
        """Strong/weak lists under the theta-criterion.  Section 4's
        structural options: ``parent`` (interaction via the parent box) and
        ``swap`` = "finest" or "all" (exchanged roles for boxes of very
        different radii at the finest level, or at every level)."""
        opt = (_capi.OPT_PARENT if parent else 0) | {None: 0, "finest": _capi.OPT_SWAP_FINEST,
                                                     "all": _capi.OPT_SWAP_ALL}[swap]
        self._check(self._lib.fmm2d_connectivity_opt(self._h, float(theta), opt))

    def connectivity_relaxed(self, theta: float, theta_max: float, p: int, k0: int = 16, k1: int = 16):
        """Plain lists under the locally relaxed theta-criterion (Section 4,
        last paragraph): candidates up to theta_max admitted as weak, lowest
        first, while each level's mean of theta_i^(p+1) stays within
        theta^(p+1)."""
        self._check(self._lib.fmm2d_connectivity_relaxed(self._h, float(theta), float(theta_max), int(p),
                                                          int(k0), int(k1)))
        self._relax_bins = int(k0) + int(k1)

    def relax_bins(self):
        """(count int64 [L + 1, k0 + k1], kmax int32 [L + 1]) of the relaxed lists."""
        nbin = getattr(self, "_relax_bins", 0)
        if not nbin or self.levels is None:
            raise RuntimeError("no lists from connectivity_relaxed")
        count = torch.zeros((self.levels + 1) * nbin, dtype=torch.int64)
        kmax = torch.zeros(self.levels + 1, dtype=torch.int32)
        self._check(self._lib.fmm2d_get_relax_bins(self._h, _ptr(count), _ptr(kmax)))
        return count.reshape(self.levels + 1, nbin), kmax

    def evaluate(self, q: torch.Tensor, p: int, mode: str = "fp64", out: torch.Tensor | None = None):
        _require(q, torch.float64, self.device, "q")
        if self.n is not None and q.numel() != self.n:
            raise ValueError("q has %d entries, the tree %d" % (q.numel(), self.n))
        if out is None:
            out = torch.empty_like(q)
        _require(out, torch.float64, self.device, "out")
        self._check(self._lib.fmm2d_evaluate(self._h, _ptr(q), int(p), _capi.MODES[mode], _ptr(out)))
        return out

    def evaluate_field(self, q: torch.Tensor, p: int, mode: str = "fp64"):
        """(phi, d phi/dx, d phi/dy) at every point, input order (binary64 only)."""
        _require(q, torch.float64, self.device, "q")
        if self.n is not None and q.numel() != self.n:
            raise ValueError("q has %d entries, the tree %d" % (q.numel(), self.n))
        phi, gx, gy = (torch.empty_like(q) for _ in range(3))
        self._check(self._lib.fmm2d_evaluate_field(self._h, _ptr(q), int(p), _capi.MODES[mode], _ptr(phi), _ptr(gx),
                                                   _ptr(gy)))
        return phi, gx, gy

    def direct(self, x, y, q, targets: torch.Tensor, out: torch.Tensor | None = None):
        for t, nm in ((x, "x"), (y, "y"), (q, "q")):
            _require(t, torch.float64, self.device, nm)
        _require(targets, torch.int64, self.device, "targets")
        if out is None:
            out = torch.empty(targets.numel(), dtype=torch.float64, device=self.device)
        self._check(self._lib.fmm2d_direct(self._h, _ptr(x), _ptr(y), _ptr(q), x.numel(), _ptr(targets),
                                           targets.numel(), _ptr(out)))
        return out

    def direct_noalloc(self, x, y, q, targets: torch.Tensor, out: torch.Tensor):
        """fmm2d_direct on the library's fixed device array: no allocation by
        the library (the caller provides out)."""
        for t, nm in ((x, "x"), (y, "y"), (q, "q")):
            _require(t, torch.float64, self.device, nm)
        _require(targets, torch.int64, self.device, "targets")
        _require(out, torch.float64, self.device, "out")
        if out.numel() < targets.numel():
            raise ValueError("out holds %d values, %d targets" % (out.numel(), targets.numel()))
        self._check(self._lib.fmm2d_direct_noalloc(self._h, _ptr(x), _ptr(y), _ptr(q), x.numel(), _ptr(targets),
                                                   targets.numel(), _ptr(out)))
        return out

    def direct_field(self, x, y, q, targets: torch.Tensor):
        """(d phi/dx, d phi/dy) by the direct binary64 sum at the target indices."""
        for t, nm in ((x, "x"), (y, "y"), (q, "q")):
            _require(t, torch.float64, self.device, nm)
        _require(targets, torch.int64, self.device, "targets")
        gx = torch.empty(targets.numel(), dtype=torch.float64, device=self.device)
        gy = torch.empty_like(gx)
        self._check(self._lib.fmm2d_direct_field(self._h, _ptr(x), _ptr(y), _ptr(q), x.numel(), _ptr(targets),
                                                 targets.numel(), _ptr(gx), _ptr(gy)))
        return gx, gy

    # -- timing -------------------------------------------------------------
    def timing(self, enable: bool):
        self._check(self._lib.fmm2d_timing(self._h, 1 if enable else 0))

    def timings(self):
        """{phase: (total GPU ms, intervals)} since timing was enabled."""
        import numpy as np

        ms = np.zeros(len(_capi.PHASES), dtype=np.float64)
        cnt = np.zeros(len(_capi.PHASES), dtype=np.int64)
        self._check(self._lib.fmm2d_get_timings(self._h, ctypes.c_void_p(ms.ctypes.data),
                                                ctypes.c_void_p(cnt.ctypes.data)))
        return {ph: (float(ms[i]), int(cnt[i])) for i, ph in enumerate(_capi.PHASES)}

    # -- parameter selection ----------------------------------------------
    def features(self, x: torch.Tensor, y: torch.Tensor, tol: float, out: torch.Tensor | None = None):
        _require(x, torch.float64, self.device, "x")
        _require(y, torch.float64, self.device, "y")
        if out is None:
            out = torch.empty(_capi.NFEAT, dtype=torch.float32, device=self.device)
        _require(out, torch.float32, self.device, "out")
        if out.numel() < _capi.NFEAT:
            raise ValueError("out holds fewer than %d floats" % _capi.NFEAT)
        self._check(self._lib.fmm2d_features(self._h, _ptr(x), _ptr(y), x.numel(), float(tol), _ptr(out)))
        return out

    def select(self, x: torch.Tensor, y: torch.Tensor, tol: float, weights: torch.Tensor | None = None):
        """(levels, p, theta, from_network); weights is the device blob of a trained selector."""
        _require(x, torch.float64, self.device, "x")
        _require(y, torch.float64, self.device, "y")
        wp = None
        if weights is not None:
            _require(weights, torch.float32, self.device, "weights")
            need = _capi.SELECT_HEADER + self._lib.fmm2d_mlp_nparams(_capi.NFEAT)
            if weights.numel() != need:
                raise ValueError("weights must hold %d floats" % need)
            wp = _ptr(weights)
        L, p, net = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        th = ctypes.c_double()
        self._check(self._lib.fmm2d_select(self._h, _ptr(x), _ptr(y), x.numel(), float(tol), wp, ctypes.byref(L),
                                           ctypes.byref(p), ctypes.byref(th), ctypes.byref(net)))
        return L.value, p.value, th.value, bool(net.value)

    def select_build_tree(self, x: torch.Tensor, y: torch.Tensor, tol: float, weights: torch.Tensor | None = None):
        """select() then build_tree() at the selected level count, in one call
        (the sort overlaps the selector); returns (levels, p, theta, from_network)."""
        _require(x, torch.float64, self.device, "x")
        _require(y, torch.float64, self.device, "y")
        if x.numel() != y.numel():
            raise ValueError("x and y differ in length")
        wp = None
        if weights is not None:
            _require(weights, torch.float32, self.device, "weights")
            need = _capi.SELECT_HEADER + self._lib.fmm2d_mlp_nparams(_capi.NFEAT)
            if weights.numel() != need:
                raise ValueError("weights must hold %d floats" % need)
            wp = _ptr(weights)
        L, p, net = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        th = ctypes.c_double()
        self._check(self._lib.fmm2d_select_build_tree(self._h, _ptr(x), _ptr(y), x.numel(), float(tol), wp,
                                                      ctypes.byref(L), ctypes.byref(p), ctypes.byref(th),
                                                      ctypes.byref(net)))
        self.n, self.levels = x.numel(), L.value
        return L.value, p.value, th.value, bool(net.value)

    def mlp_nparams(self, d_in: int) -> int:
        return int(self._lib.fmm2d_mlp_nparams(int(d_in)))

    def mlp_forward(self, params: torch.Tensor, X: torch.Tensor, out: torch.Tensor | None = None):
        _require(params, torch.float32, self.device, "params")
        _require(X, torch.float32, self.device, "X")
        batch, d_in = X.shape
        if params.numel() != self.mlp_nparams(d_in):
            raise ValueError("params must hold %d floats" % self.mlp_nparams(d_in))
        if out is None:
            out = torch.empty((batch, 3), dtype=torch.float32, device=self.device)
        _require(out, torch.float32, self.device, "out")
        self._check(self._lib.fmm2d_mlp_forward(self._h, _ptr(params), _ptr(X), batch, d_in, _ptr(out)))
        return out

    def mlp_grad(self, params: torch.Tensor, X: torch.Tensor, Y: torch.Tensor, grad: torch.Tensor | None = None,
                 loss: torch.Tensor | None = None):
        _require(params, torch.float32, self.device, "params")
        _require(X, torch.float32, self.device, "X")
        _require(Y, torch.float32, self.device, "Y")
        batch, d_in = X.shape
        if params.numel() != self.mlp_nparams(d_in) or tuple(Y.shape) != (batch, 3):
            raise ValueError("params or Y has the wrong size")
        if grad is None:
            grad = torch.empty_like(params)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=self.device)
        _require(grad, torch.float32, self.device, "grad")
        _require(loss, torch.float32, self.device, "loss")
        self._check(self._lib.fmm2d_mlp_grad(self._h, _ptr(params), _ptr(X), _ptr(Y), batch, d_in, _ptr(grad),
                                             _ptr(loss)))
        return grad, loss

    def mlp_adam(self, params: torch.Tensor, m: torch.Tensor, v: torch.Tensor, grad: torch.Tensor, step: int,
                 lr: float, weight_decay: float = 0.0):
        for t, nm in ((params, "params"), (m, "m"), (v, "v"), (grad, "grad")):
            _require(t, torch.float32, self.device, nm)
            if t.numel() != params.numel():
                raise ValueError("%s differs in size from params" % nm)
        self._check(self._lib.fmm2d_mlp_adam(self._h, _ptr(params), _ptr(m), _ptr(v), _ptr(grad), params.numel(),
                                             int(step), float(lr), float(weight_decay)))

    # -- introspection ------------------------------------------------------
    def tree_info(self):
        n, nb = ctypes.c_int64(), ctypes.c_int64()
        L = ctypes.c_int()
        self._check(self._lib.fmm2d_tree_info(self._h, ctypes.byref(n), ctypes.byref(L), ctypes.byref(nb)))
        return n.value, L.value, nb.value

    def perm(self):
        out = torch.empty(self.n, dtype=torch.int32, device=self.device)
        self._check(self._lib.fmm2d_get_perm(self._h, _ptr(out)))
        return out

    def leaf_start(self):
        out = torch.empty(4 ** self.levels + 1, dtype=torch.int32, device=self.device)
        self._check(self._lib.fmm2d_get_leaf_start(self._h, _ptr(out)))
        return out

    def rects(self):
        nbox = (4 ** (self.levels + 1) - 1) // 3
        out = torch.empty((nbox, 4), dtype=torch.float64, device=self.device)
        self._check(self._lib.fmm2d_get_rects(self._h, _ptr(out)))
        return out

    def geometry(self):
        """(cx, cy, r, scale) of every box, level by level."""
        nbox = (4 ** (self.levels + 1) - 1) // 3
        out = torch.empty((nbox, 4), dtype=torch.float64, device=self.device)
        self._check(self._lib.fmm2d_get_geometry(self._h, _ptr(out)))
        return out

    def list_sizes(self, level: int):
        ns, nw = ctypes.c_int64(), ctypes.c_int64()
        self._check(self._lib.fmm2d_list_sizes(self._h, level, ctypes.byref(ns), ctypes.byref(nw)))
        return ns.value, nw.value

    def lists(self, level: int):
        ns, nw = self.list_sizes(level)
        nb = 4 ** level
        dev = self.device
        sp = torch.empty(nb + 1, dtype=torch.int32, device=dev)
        wp = torch.empty(nb + 1, dtype=torch.int32, device=dev)
        si = torch.empty(max(ns, 1), dtype=torch.int32, device=dev)
        wi = torch.empty(max(nw, 1), dtype=torch.int32, device=dev)
        self._check(self._lib.fmm2d_get_lists(self._h, level, _ptr(sp), _ptr(si), _ptr(wp), _ptr(wi)))
        return sp, si[:ns], wp, wi[:nw]

    def xlists(self, level: int):
        """(xptr, xidx) of the exchanged-roles list of one level."""
        nx = ctypes.c_int64()
        self._check(self._lib.fmm2d_get_xlists(self._h, level, ctypes.byref(nx), None, None))
        nb = 4 ** level
        xp = torch.empty(nb + 1, dtype=torch.int32, device=self.device)
        xi = torch.empty(max(nx.value, 1), dtype=torch.int32, device=self.device)
        self._check(self._lib.fmm2d_get_xlists(self._h, level, ctypes.byref(nx), _ptr(xp), _ptr(xi)))
        return xp, xi[:nx.value]
