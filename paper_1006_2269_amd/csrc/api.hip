// C ABI of the library: argument validation, call-order checks, error
// reporting, and the sequencing of the device passes on the context stream.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <new>

#include "devutil.h"
#include "evaluate.h"
#include "internal.h"

using namespace fmm2d;

namespace {

// Makes ctx's device current and ctx the owner of the device buffers that
// grow during the call (DevBuf::ensure); both are restored on exit.
thread_local fmm2d_ctx *tl_ctx = nullptr;

struct CtxScope {
    int prev = -1;
    fmm2d_ctx *prev_ctx;
    explicit CtxScope(fmm2d_ctx *c) : prev_ctx(tl_ctx) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != c->device) (void)hipSetDevice(c->device);
        tl_ctx = c;
    }
    ~CtxScope() {
        tl_ctx = prev_ctx;
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

int fail(fmm2d_ctx *c, int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
int fail(fmm2d_ctx *c, int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    c->err = buf;
    return code;
}

int hip_fail(fmm2d_ctx *c, hipError_t e, const char *where) {
    if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
        return fail(c, FMM2D_ENOMEM, "%s: device allocation failed (%s)", where, hipGetErrorString(e));
    return fail(c, FMM2D_EDEVICE, "%s: %s", where, hipGetErrorString(e));
}

// flags[1]: a target index out of range
__global__ void k_check_targets(const int64_t *__restrict__ t, int64_t m, int64_t n, int *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && (t[i] < 0 || t[i] >= n)) flags[1] = 1;
}
__global__ void k_zero_flags(int *flags) {
    flags[0] = 0;
    flags[1] = 0;
}

}  // namespace

namespace fmm2d {

static hipError_t dev_alloc(fmm2d_ctx *c, void **p, size_t bytes) {
    if (c->alloc) {
        *p = c->alloc(bytes, c->user);
        return *p ? hipSuccess : hipErrorOutOfMemory;
    }
    return hipMalloc(p, bytes);
}

static hipError_t dev_free(fmm2d_ctx *c, void *p, size_t bytes) {
    if (c->free) {
        // stream order: the context stream waits for the second stream's
        // last batch, and the callback returns the memory at that point
        const hipError_t e = side_join(c);
        c->free(p, bytes, c->user);
        return e;
    }
    hipError_t e = c->side ? hipStreamSynchronize(c->side) : hipSuccess;
    const hipError_t e2 = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = e2;
    const hipError_t e3 = hipFree(p);
    return e != hipSuccess ? e : e3;
}

hipError_t DevBuf::ensure(size_t bytes) {
    if (bytes <= cap && ptr) return hipSuccess;
    fmm2d_ctx *c = tl_ctx;
    if (!c) return hipErrorInvalidContext;
    if (ptr) {
        const hipError_t e = dev_free(c, ptr, cap);
        ptr = nullptr;
        cap = 0;
        if (e != hipSuccess) return e;
    }
    const size_t b = bytes < 256 ? 256 : bytes;
    void *q = nullptr;
    const hipError_t e = dev_alloc(c, &q, b);
    if (e != hipSuccess) return e;
    ptr = q;
    cap = b;
    return hipSuccess;
}

void DevBuf::release() {
    if (ptr && tl_ctx) (void)dev_free(tl_ctx, ptr, cap);
    ptr = nullptr;
    cap = 0;
}

}  // namespace fmm2d

extern "C" {

int fmm2d_version(void) { return 100; }

int fmm2d_create(fmm2d_ctx **out, int device, void *stream, fmm2d_alloc_fn alloc, fmm2d_free_fn free_fn,
                 void *user) {
    if (!out) return FMM2D_EINVAL;
    *out = nullptr;
    if ((alloc == nullptr) != (free_fn == nullptr)) return FMM2D_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return FMM2D_EINVAL;
    fmm2d_ctx *c = new (std::nothrow) fmm2d_ctx;
    if (!c) return FMM2D_ENOMEM;
    c->device = device;
    c->stream = static_cast<hipStream_t>(stream);
    c->alloc = alloc;
    c->free = free_fn;
    c->user = user;
    if (const char *lim = getenv("FMM2D_LIST_LIMIT")) {
        const long long v = atoll(lim);
        if (v > 0 && v < c->list_limit) c->list_limit = v;
    }
    *out = c;
    return FMM2D_OK;
}

int fmm2d_destroy(fmm2d_ctx *c) {
    if (!c) return FMM2D_EINVAL;
    {
        CtxScope g(c);
        (void)hipStreamSynchronize(c->stream);
        if (c->side) {
            (void)hipStreamSynchronize(c->side);
            (void)hipStreamDestroy(c->side);
            (void)hipEventDestroy(c->ev_side_in);
            (void)hipEventDestroy(c->ev_side_out);
            c->side = nullptr;
            c->side_pending = false;
        }
        if (c->hpin) {
            (void)hipEventDestroy(c->ev_keys);
            (void)hipEventDestroy(c->ev_sel);
            (void)hipHostFree(c->hpin);
        }
        TreeState &t = c->tree;
        for (DevBuf *b : {&t.xsorted, &t.ysorted, &t.xorder, &t.XLx, &t.XLy, &t.YLx, &t.YLy, &t.T0, &t.T1,
                          &t.starts, &t.rects, &t.prect, &t.geom, &t.perm, &t.leafid, &t.px, &t.py, &t.loc, &t.sptr, &t.wptr,
                          &t.sidx, &t.widx, &t.xptr, &t.xidx, &t.cnt_x, &t.cnt_s, &t.cnt_w, &t.pool_state, &t.nrec_j, &t.nrec_d, &t.bits,
                          &t.owner0, &t.owner1, &t.selfpos, &t.trans, &t.spart, &t.relax_tk, &t.relax_hist,
                          &t.relax_lv, &t.relax_k})
            b->release();
        EvalState &e = c->ev;
        c->tree.m2l_all.segoff.release();
        c->tree.m2l_all.table.release();
        c->tree.near_seg.segoff.release();
        c->tree.near_seg.table.release();
        c->tree.near_up.segoff.release();
        c->tree.near_up.table.release();
        c->tree.near_lo.segoff.release();
        c->tree.near_lo.table.release();
        c->tree.lsum.release();
        c->tree.x_items.release();
        c->tree.x_itemoff.release();
        c->tree.m_items.release();
        c->tree.m_itemoff.release();
        c->ev.xpart.release();
        c->ev.xsum.release();
        c->ev.mpart.release();
        for (DevBuf *b : {&e.binom, &e.mhat, &e.part, &e.npart, &e.gpart, &e.A, &e.B, &e.qs, &e.work,
                          &e.src, &e.srclo})
            b->release();
        Scratch &s = c->scr;
        for (hipEvent_t ev : c->timer.pool) (void)hipEventDestroy(ev);
        for (DevBuf *b : {&s.keys0, &s.keys1, &s.vals0, &s.vals1, &s.hist, &s.aux, &s.tiles, &s.tiles2, &s.segbase,
                          &s.thr, &s.split0, &s.split1, &s.flag, &s.segcnt, &s.mcnt, &s.sel, &s.sel2})
            b->release();
    }
    delete c;
    return FMM2D_OK;
}

const char *fmm2d_last_error(const fmm2d_ctx *c) {
    if (!c) return "fmm2d: NULL context";
    return c->err.c_str();
}

int fmm2d_set_stream(fmm2d_ctx *c, void *stream) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (s == c->stream) return FMM2D_OK;
    // the new stream starts after everything queued on the old one (and on
    // the second stream), so buffers handed back in stream order stay safe
    CtxScope g(c);
    hipEvent_t ev = nullptr;
    hipError_t e = side_join(c);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventRecord(ev, c->stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, ev, 0);
    if (ev) (void)hipEventDestroy(ev);
    if (e != hipSuccess) return hip_fail(c, e, "set_stream");
    c->stream = s;
    return FMM2D_OK;
}

int fmm2d_set_tree_options(fmm2d_ctx *c, int flags) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (flags & ~FMM2D_TREE_SHRINK) return fail(c, FMM2D_EINVAL, "set_tree_options: unknown bits 0x%x", flags);
    c->tree_opt = flags;
    return FMM2D_OK;
}

int fmm2d_build_tree(fmm2d_ctx *c, const double *x, const double *y, int64_t n, int levels) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y) return fail(c, FMM2D_EINVAL, "build_tree: x and y must be device pointers");
    if (levels < 0 || levels > FMM2D_MAX_LEVELS) return fail(c, FMM2D_EINVAL, "build_tree: levels %d not in [0, 13]", levels);
    if (n < 1 || n > 2147483647LL) return fail(c, FMM2D_EINVAL, "build_tree: n = %lld not in [1, 2^31-1]", (long long)n);
    if (n < (int64_t(1) << (2 * levels)))
        return fail(c, FMM2D_EINVAL, "build_tree: n = %lld < 4^levels = %lld", (long long)n,
                    (long long)(int64_t(1) << (2 * levels)));
    CtxScope g(c);
    hipError_t e;
    // validate the coordinates (and make the sort keys) before touching the
    // current tree
    bool bad = false;
    {
        PhaseScope ps(c, PH_TREE);
        e = sort_prepare(c, x, y, n, &bad);
    }
    if (e != hipSuccess) return hip_fail(c, e, "build_tree");
    if (bad) return fail(c, FMM2D_EINVAL, "build_tree: coordinates must be finite with |v| <= 2^500");
    TreeState &t = c->tree;
    t.has_lists = false;
    t.nrec_valid = false;
    t.n = n;
    t.L = levels;
    {
        PhaseScope ps(c, PH_TREE);
        e = side_join(c);  // second-stream work still reading the previous tree or lists
        if (e == hipSuccess) e = build_tree_device(c, x, y);
    }
    if (e != hipSuccess) {
        t.L = -1;
        return hip_fail(c, e, "build_tree");
    }
    return FMM2D_OK;
}

int fmm2d_select_build_tree(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol,
                            const float *weights, int *levels, int *p, double *theta, int *from_network) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y || !levels || !p || !theta) return fail(c, FMM2D_EINVAL, "select_build_tree: NULL pointer");
    if (n < 4 || n > 2147483647LL)
        return fail(c, FMM2D_EINVAL, "select_build_tree: n = %lld not in [4, 2^31-1]", (long long)n);
    if (!(tol > 0.0 && tol < 1.0)) return fail(c, FMM2D_EINVAL, "select_build_tree: tol must lie in (0, 1)");
    CtxScope g(c);
    TreeState &t = c->tree;
    hipError_t e = hipSuccess;
    if (!c->hpin) {
        if ((e = hipHostMalloc(&c->hpin, 128, hipHostMallocDefault)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&c->ev_keys, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&c->ev_sel, hipEventDisableTiming)) != hipSuccess)
            return hip_fail(c, e, "select_build_tree");
    }
    unsigned long long *h_andor = static_cast<unsigned long long *>(c->hpin);  // 6 words
    int *h_out = reinterpret_cast<int *>(static_cast<char *>(c->hpin) + 64);      // levels, p, network, bad
    double *h_theta = reinterpret_cast<double *>(static_cast<char *>(c->hpin) + 80);
    // The tree's sorted arrays are overwritten before the validation is read:
    // the current tree is given up from here on.
    t.has_lists = false;
    t.nrec_valid = false;
    t.L = -1;
    // second-stream work of earlier calls first; then the selector on the
    // second stream while the keys and all eight radix passes run here
    e = side_join(c);
    if (e == hipSuccess) e = side_begin(c);
    if (e == hipSuccess) {
        PhaseScope ps(c, PH_SELECT, c->side);
        e = select_launch(c, c->side, x, y, n, tol, weights, h_out, h_theta);
    }
    if (e == hipSuccess) e = hipEventRecord(c->ev_sel, c->side);
    if (e == hipSuccess) e = side_end(c);
    if (e == hipSuccess) {
        PhaseScope ps(c, PH_TREE);
        e = sort_prepare_async(c, x, y, n, h_andor, c->ev_keys);
        if (e == hipSuccess) e = tree_sort(c, n);
    }
    // one wait for the two small copies; the sort keeps running meanwhile
    if (e == hipSuccess) e = hipEventSynchronize(c->ev_keys);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev_sel);
    if (e != hipSuccess) return hip_fail(c, e, "select_build_tree");
    if ((h_andor[2] | h_andor[5]) != 0 || h_out[3])
        return fail(c, FMM2D_EINVAL, "select_build_tree: coordinates must be finite with |v| <= 2^500");
    const int L = h_out[0];
    t.n = n;
    t.L = L;
    {
        PhaseScope ps(c, PH_TREE);
        e = build_tree_device(c, x, y, true);
    }
    if (e != hipSuccess) {
        t.L = -1;
        return hip_fail(c, e, "select_build_tree");
    }
    *levels = L;
    *p = h_out[1];
    *theta = *h_theta;
    if (from_network) *from_network = h_out[2];
    return FMM2D_OK;
}

// The list build with its pool regrowth, shared by the connectivity calls
// (arguments already checked).
static int connectivity_impl(fmm2d_ctx *c, double theta, int opt, const RelaxRule *rx) {
    TreeState &t = c->tree;
    CtxScope g(c);
    const int64_t nbox = level_offset(t.L + 1);
    const bool swaps = (opt & (FMM2D_OPT_SWAP_FINEST | FMM2D_OPT_SWAP_ALL)) != 0;
    // start from the pool sizes that sufficed for the previous call (repeated
    // calls on similar point sets then build the lists in one pass)
    int64_t cap_s = std::max<int64_t>(32 * nbox + 64, c->cap_hint_s);
    int64_t cap_w = std::max<int64_t>(96 * nbox + 64, c->cap_hint_w);
    int64_t cap_x = swaps ? std::max<int64_t>(16 * nbox + 64, c->cap_hint_x) : 0;
    const int64_t pool_max = int64_t(1) << 34;  // entries per pool, all levels together
    for (int attempt = 0; attempt < 16; ++attempt) {
        int overflow = 0;
        hipError_t e;
        {
            PhaseScope ps(c, PH_LISTS);
            t.nrec_valid = false;
            e = build_lists_device(c, theta, opt, cap_s, cap_w, cap_x, c->list_limit, &overflow, rx);
        }
        if (e != hipSuccess) {
            t.has_lists = false;
            return hip_fail(c, e, "connectivity");
        }
        if (overflow == 0) {
            {
                PhaseScope ps(c, PH_LISTS);
                t.nrec_valid = true;  // written by the finest level's fill pass
                e = build_schedules(c);
            }
            if (e != hipSuccess) return hip_fail(c, e, "connectivity");
            // the root box's half diagonal, for the range check of the FP32 modes
            double4 g0;
            if ((e = hipMemcpyAsync(&g0, t.geom.as<double4>(), sizeof(g0), hipMemcpyDeviceToHost, c->stream)) !=
                    hipSuccess ||
                (e = hipStreamSynchronize(c->stream)) != hipSuccess)
                return hip_fail(c, e, "connectivity");
            t.root_r = g0.z;
            t.has_lists = true;
            t.theta = theta;
            c->cap_hint_s = cap_s;
            c->cap_hint_w = cap_w;
            if (swaps) c->cap_hint_x = cap_x;
            return FMM2D_OK;
        }
        if (overflow == 2) {
            t.has_lists = false;
            return fail(c, FMM2D_ECAPACITY,
                        "connectivity: a level's strong or weak list exceeds %lld entries (choose fewer levels or "
                        "another theta for this point set)",
                        (long long)c->list_limit);
        }
        // grow only the pools that were too small, to at least twice what the
        // levels built so far needed (the pool offsets read back with the flag)
        const int64_t need_s = *std::max_element(t.s_off.begin(), t.s_off.end());
        const int64_t need_w = *std::max_element(t.w_off.begin(), t.w_off.end());
        const int64_t need_x = *std::max_element(t.x_off.begin(), t.x_off.end());
        auto grown = [&](int64_t cap, int64_t need) { return std::min(pool_max, std::max(4 * cap, 2 * need)); };
        const int64_t old_s = cap_s, old_w = cap_w, old_x = cap_x;
        if (overflow & LIST_GROW_S) cap_s = grown(cap_s, need_s);
        if (overflow & LIST_GROW_W) cap_w = grown(cap_w, need_w);
        if (overflow & LIST_GROW_X) cap_x = grown(cap_x, need_x);
        if (overflow & LIST_GROW_CAND) cap_w = grown(cap_w, need_w);
        if (cap_s == old_s && cap_w == old_w && cap_x == old_x) break;  // at the 2^34 ceiling
    }
    t.has_lists = false;
    return fail(c, FMM2D_ECAPACITY, "connectivity: interaction lists exceed 2^34 entries");
}

int fmm2d_connectivity_opt(fmm2d_ctx *c, double theta, int opt) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!(theta > 0.0 && theta < 1.0)) return fail(c, FMM2D_EINVAL, "connectivity: theta must lie in (0, 1)");
    if (opt & ~(FMM2D_OPT_PARENT | FMM2D_OPT_SWAP_FINEST | FMM2D_OPT_SWAP_ALL))
        return fail(c, FMM2D_EINVAL, "connectivity: unknown option bits 0x%x", opt);
    if (c->tree.L < 0) return fail(c, FMM2D_ESTATE, "connectivity: no tree (call fmm2d_build_tree first)");
    return connectivity_impl(c, theta, opt, nullptr);
}

int fmm2d_connectivity(fmm2d_ctx *c, double theta) { return fmm2d_connectivity_opt(c, theta, 0); }

// t^(p+1) by p repeated products, each rounded (the sums of the admission
// test use the same values on the device).
static double power_p1(double t, int p) {
    double e = t;
    for (int i = 0; i < p; ++i) e *= t;
    return e;
}

int fmm2d_connectivity_relaxed(fmm2d_ctx *c, double theta, double theta_max, int p, int k0, int k1) {
#pragma clang fp contract(off)
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!(theta > 0.0 && theta <= theta_max && theta_max < 1.0))
        return fail(c, FMM2D_EINVAL, "connectivity_relaxed: need 0 < theta <= theta_max < 1");
    if (p < 0 || p > 1024 || k0 < 1 || k1 < 1 || k0 + k1 > RELAX_MAX_BINS)
        return fail(c, FMM2D_EINVAL, "connectivity_relaxed: need 0 <= p <= 1024, k0, k1 >= 1, k0 + k1 <= %d",
                    RELAX_MAX_BINS);
    TreeState &t = c->tree;
    if (t.L < 0) return fail(c, FMM2D_ESTATE, "connectivity_relaxed: no tree (call fmm2d_build_tree first)");
    const int nbin = k0 + k1;
    t.relax_host.assign(2 * nbin, 0.0);
    for (int k = 0; k < nbin; ++k) {
        const double tk = k < k0 ? theta * (double)(k + 1) / (double)k0
                                 : theta + (theta_max - theta) * (double)(k - k0 + 1) / (double)k1;
        t.relax_host[k] = tk;
        t.relax_host[nbin + k] = power_p1(tk, p);
    }
    RelaxRule rx{theta, theta_max, power_p1(theta, p), p, k0, k1};
    return connectivity_impl(c, theta, 0, &rx);
}

int fmm2d_get_relax_bins(fmm2d_ctx *c, int64_t *count, int32_t *kmax) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    TreeState &t = c->tree;
    if (!t.has_lists || t.relax_nbin == 0)
        return fail(c, FMM2D_ESTATE, "get_relax_bins: no lists from fmm2d_connectivity_relaxed");
    if (!count || !kmax) return fail(c, FMM2D_EINVAL, "get_relax_bins: NULL output");
    CtxScope g(c);
    const int nbin = t.relax_nbin, L = t.L;
    std::vector<uint32_t> h((size_t)(L + 1) * nbin);
    hipError_t e;
    if ((e = hipMemcpyAsync(h.data(), t.relax_hist.ptr, sizeof(uint32_t) * h.size(), hipMemcpyDeviceToHost,
                            c->stream)) != hipSuccess ||
        (e = hipMemcpyAsync(kmax, t.relax_k.ptr, sizeof(int32_t) * (L + 1), hipMemcpyDeviceToHost, c->stream)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, "get_relax_bins");
    for (size_t i = 0; i < h.size(); ++i) count[i] = h[i];
    return FMM2D_OK;
}

int fmm2d_evaluate(fmm2d_ctx *c, const double *q, int p, int mode, double *phi) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!q || !phi) return fail(c, FMM2D_EINVAL, "evaluate: q and phi must be device pointers");
    if (p < 1 || p > FMM2D_MAX_P) return fail(c, FMM2D_EINVAL, "evaluate: p = %d not in [1, 63]", p);
    if (mode < FMM2D_MODE_FP64 || mode > FMM2D_MODE_FP32_ACC64) return fail(c, FMM2D_EINVAL, "evaluate: unknown mode %d", mode);
    if (c->tree.L < 0 || !c->tree.has_lists)
        return fail(c, FMM2D_ESTATE, "evaluate: needs a tree and its lists (build_tree, connectivity)");
    // The FP32 modes work on offsets from leaf centres: their squares must
    // neither overflow nor underflow FP32 (a point set spanning zero is fine:
    // all its points coincide and contribute nothing)
    const double r0 = c->tree.root_r;
    if (mode != FMM2D_MODE_FP64 && r0 != 0.0 && !(r0 >= 0x1p-60 && r0 <= 0x1p56))
        return fail(c, FMM2D_EINVAL,
                    "evaluate: the FP32 modes need a root box whose half diagonal lies in [2^-60, 2^56] (this one: "
                    "%.3g); use FMM2D_MODE_FP64",
                    r0);
    CtxScope g(c);
    hipError_t e = evaluate_device(c, q, p, mode, phi);
    if (e != hipSuccess) return hip_fail(c, e, "evaluate");
    return FMM2D_OK;
}

int fmm2d_evaluate_field(fmm2d_ctx *c, const double *q, int p, int mode, double *phi, double *gx, double *gy) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!q || !phi || !gx || !gy) return fail(c, FMM2D_EINVAL, "evaluate_field: q, phi, gx and gy must be device pointers");
    if (p < 1 || p > FMM2D_MAX_P) return fail(c, FMM2D_EINVAL, "evaluate_field: p = %d not in [1, 63]", p);
    if (mode != FMM2D_MODE_FP64)
        return fail(c, FMM2D_EINVAL, "evaluate_field: the gradient is computed in binary64 only (FMM2D_MODE_FP64)");
    if (c->tree.opt != 0)
        return fail(c, FMM2D_EINVAL, "evaluate_field: needs the plain lists (fmm2d_connectivity without options)");
    if (c->tree.L < 0 || !c->tree.has_lists)
        return fail(c, FMM2D_ESTATE, "evaluate_field: needs a tree and its lists (build_tree, connectivity)");
    CtxScope g(c);
    hipError_t e = evaluate_device(c, q, p, mode, phi);
    if (e == hipSuccess) e = gradient_device(c, p, gx, gy);
    if (e != hipSuccess) return hip_fail(c, e, "evaluate_field");
    return FMM2D_OK;
}

// Checks (on the device, one host read) that every target index lies in
// [0, n); FMM2D_OK or the error code with the message set.
static int check_targets(fmm2d_ctx *c, const int64_t *targets, int64_t m, int64_t n, const char *who) {
    hipError_t e;
    if ((e = c->scr.aux.ensure(4096)) != hipSuccess) return hip_fail(c, e, who);
    int *flags = reinterpret_cast<int *>(c->scr.aux.as<char>() + 2048);
    hipLaunchKernelGGL(k_zero_flags, dim3(1), dim3(1), 0, c->stream, flags);
    hipLaunchKernelGGL(k_check_targets, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, targets, m, n, flags);
    int hf[2] = {0, 0};
    if ((e = hipMemcpyAsync(hf, flags, sizeof(hf), hipMemcpyDeviceToHost, c->stream)) != hipSuccess ||
        (e = hipStreamSynchronize(c->stream)) != hipSuccess)
        return hip_fail(c, e, who);
    if (hf[1]) return fail(c, FMM2D_EINVAL, "%s: a target index is outside [0, n)", who);
    return FMM2D_OK;
}

int fmm2d_direct(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n, const int64_t *targets,
                 int64_t m, double *phi_m) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y || !q || (m > 0 && (!targets || !phi_m))) return fail(c, FMM2D_EINVAL, "direct: NULL pointer");
    if (n < 1 || m < 0) return fail(c, FMM2D_EINVAL, "direct: need n >= 1 and m >= 0");
    if (m == 0) return FMM2D_OK;
    CtxScope g(c);
    hipError_t e;
    if (int rc = check_targets(c, targets, m, n, "direct")) return rc;
    {
        PhaseScope ps(c, PH_JUDGE);
        e = direct_device(c, x, y, q, n, targets, m, phi_m);
    }
    if (e != hipSuccess) return hip_fail(c, e, "direct");
    return FMM2D_OK;
}

int fmm2d_direct_noalloc(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                         const int64_t *targets, int64_t m, double *phi_m) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y || !q || (m > 0 && (!targets || !phi_m))) return fail(c, FMM2D_EINVAL, "direct_noalloc: NULL pointer");
    if (n < 1 || m < 0) return fail(c, FMM2D_EINVAL, "direct_noalloc: need n >= 1 and m >= 0");
    if (m == 0) return FMM2D_OK;
    if (m > (int64_t(1) << 18) || !noalloc_fits(n, m))
        return fail(c, FMM2D_EINVAL, "direct_noalloc: m = %lld exceeds 262144 targets (the fixed 4 MiB scratch)",
                    (long long)m);
    CtxScope g(c);
    void *scr = nullptr;
    hipError_t e = noalloc_scratch(c->device, &scr);
    bool bad = false;
    if (e == hipSuccess) e = direct_noalloc_device(c, scr, x, y, q, n, targets, m, phi_m, &bad);
    if (e != hipSuccess) return hip_fail(c, e, "direct_noalloc");
    if (bad) return fail(c, FMM2D_EINVAL, "direct_noalloc: a target index is outside [0, %lld)", (long long)n);
    return FMM2D_OK;
}

int fmm2d_direct_field(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                       const int64_t *targets, int64_t m, double *gx_m, double *gy_m) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y || !q || (m > 0 && (!targets || !gx_m || !gy_m)))
        return fail(c, FMM2D_EINVAL, "direct_field: NULL pointer");
    if (n < 1 || m < 0) return fail(c, FMM2D_EINVAL, "direct_field: need n >= 1 and m >= 0");
    if (m == 0) return FMM2D_OK;
    CtxScope g(c);
    if (int rc = check_targets(c, targets, m, n, "direct_field")) return rc;
    hipError_t e;
    {
        PhaseScope ps(c, PH_JUDGE);
        e = direct_grad_device(c, x, y, q, n, targets, m, gx_m, gy_m);
    }
    if (e != hipSuccess) return hip_fail(c, e, "direct_field");
    return FMM2D_OK;
}

int fmm2d_features(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol, float *feat) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y || !feat) return fail(c, FMM2D_EINVAL, "features: NULL pointer");
    if (n < 1 || n > 2147483647LL) return fail(c, FMM2D_EINVAL, "features: n = %lld not in [1, 2^31-1]", (long long)n);
    if (!(tol > 0.0 && tol < 1.0)) return fail(c, FMM2D_EINVAL, "features: tol must lie in (0, 1)");
    CtxScope g(c);
    hipError_t e = features_device(c, x, y, n, tol, feat, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "features");
    return FMM2D_OK;
}

int fmm2d_select(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol, const float *weights,
                 int *levels, int *p, double *theta, int *from_network) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!x || !y || !levels || !p || !theta) return fail(c, FMM2D_EINVAL, "select: NULL pointer");
    if (n < 4 || n > 2147483647LL) return fail(c, FMM2D_EINVAL, "select: n = %lld not in [4, 2^31-1]", (long long)n);
    if (!(tol > 0.0 && tol < 1.0)) return fail(c, FMM2D_EINVAL, "select: tol must lie in (0, 1)");
    CtxScope g(c);
    int out[4] = {0, 0, 0, 0};
    double th = 0.0;
    hipError_t e;
    {
        PhaseScope ps(c, PH_SELECT);
        e = select_device(c, x, y, n, tol, weights, out, &th);
    }
    if (e != hipSuccess) return hip_fail(c, e, "select");
    if (out[3]) return fail(c, FMM2D_EINVAL, "select: coordinates must be finite with |v| <= 2^500");
    *levels = out[0];
    *p = out[1];
    *theta = th;
    if (from_network) *from_network = out[2];
    return FMM2D_OK;
}

int64_t fmm2d_mlp_nparams(int d_in) {
    if (d_in < 1 || d_in > FMM2D_MLP_MAX_IN) return -1;
    return mlp_nparams(d_in);
}

int fmm2d_mlp_forward(fmm2d_ctx *c, const float *params, const float *X, int64_t batch, int d_in, float *Y) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!params || !X || !Y) return fail(c, FMM2D_EINVAL, "mlp_forward: NULL pointer");
    if (d_in < 1 || d_in > FMM2D_MLP_MAX_IN || batch < 1 || batch > (int64_t(1) << 30))
        return fail(c, FMM2D_EINVAL, "mlp_forward: need 1 <= d_in <= %d and 1 <= batch <= 2^30", FMM2D_MLP_MAX_IN);
    CtxScope g(c);
    hipError_t e = mlp_forward(c, params, X, batch, d_in, Y);
    if (e != hipSuccess) return hip_fail(c, e, "mlp_forward");
    return FMM2D_OK;
}

int fmm2d_mlp_grad(fmm2d_ctx *c, const float *params, const float *X, const float *Y, int64_t batch, int d_in,
                   float *grad, float *loss) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!params || !X || !Y || !grad || !loss) return fail(c, FMM2D_EINVAL, "mlp_grad: NULL pointer");
    if (d_in < 1 || d_in > FMM2D_MLP_MAX_IN || batch < 1 || batch > (int64_t(1) << 24))
        return fail(c, FMM2D_EINVAL, "mlp_grad: need 1 <= d_in <= %d and 1 <= batch <= 2^24", FMM2D_MLP_MAX_IN);
    CtxScope g(c);
    hipError_t e = mlp_grad(c, params, X, Y, batch, d_in, grad, loss);
    if (e != hipSuccess) return hip_fail(c, e, "mlp_grad");
    return FMM2D_OK;
}

int fmm2d_mlp_adam(fmm2d_ctx *c, float *params, float *m, float *v, const float *grad, int64_t nparams, int step,
                   float lr, float weight_decay) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!params || !m || !v || !grad) return fail(c, FMM2D_EINVAL, "mlp_adam: NULL pointer");
    if (nparams < 1 || step < 1 || !(lr > 0.0f) || !(weight_decay >= 0.0f))
        return fail(c, FMM2D_EINVAL, "mlp_adam: need nparams >= 1, step >= 1, lr > 0, weight_decay >= 0");
    CtxScope g(c);
    hipError_t e = mlp_adam(c, params, m, v, grad, nparams, step, lr, weight_decay);
    if (e != hipSuccess) return hip_fail(c, e, "mlp_adam");
    return FMM2D_OK;
}

int fmm2d_tree_info(const fmm2d_ctx *c, int64_t *n, int *levels, int64_t *nbox) {
    if (!c) return FMM2D_EINVAL;
    if (c->tree.L < 0) return FMM2D_ESTATE;
    if (n) *n = c->tree.n;
    if (levels) *levels = c->tree.L;
    if (nbox) *nbox = level_offset(c->tree.L + 1);
    return FMM2D_OK;
}

int fmm2d_get_perm(fmm2d_ctx *c, int32_t *perm) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!perm) return fail(c, FMM2D_EINVAL, "get_perm: NULL pointer");
    if (c->tree.L < 0) return fail(c, FMM2D_ESTATE, "get_perm: no tree");
    CtxScope g(c);
    hipError_t e = hipMemcpyAsync(perm, c->tree.perm.ptr, sizeof(int32_t) * c->tree.n, hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? FMM2D_OK : hip_fail(c, e, "get_perm");
}

int fmm2d_get_leaf_start(fmm2d_ctx *c, int32_t *start) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!start) return fail(c, FMM2D_EINVAL, "get_leaf_start: NULL pointer");
    if (c->tree.L < 0) return fail(c, FMM2D_ESTATE, "get_leaf_start: no tree");
    CtxScope g(c);
    const int L = c->tree.L;
    hipError_t e = hipMemcpyAsync(start, c->tree.starts.as<int32_t>() + depth_offset(2 * L),
                                  sizeof(int32_t) * ((int64_t(1) << (2 * L)) + 1), hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? FMM2D_OK : hip_fail(c, e, "get_leaf_start");
}

int fmm2d_get_rects(fmm2d_ctx *c, double *rects) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    if (!rects) return fail(c, FMM2D_EINVAL, "get_rects: NULL pointer");
    if (c->tree.L < 0) return fail(c, FMM2D_ESTATE, "get_rects: no tree");
    CtxScope g(c);
    hipError_t e = hipMemcpyAsync(rects, c->tree.rects.ptr, sizeof(double) * 4 * level_offset(c->tree.L + 1),
                                  hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? FMM2D_OK : hip_fail(c, e, "get_rects");
}

int fmm2d_list_sizes(const fmm2d_ctx *c, int level, int64_t *ns, int64_t *nw) {
    if (!c) return FMM2D_EINVAL;
    const TreeState &t = c->tree;
    if (t.L < 0 || !t.has_lists) return FMM2D_ESTATE;
    if (level < 0 || level > t.L) return FMM2D_EINVAL;
    if (ns) *ns = t.s_off[level + 1] - t.s_off[level];
    if (nw) *nw = t.w_off[level + 1] - t.w_off[level];
    return FMM2D_OK;
}

int fmm2d_get_lists(fmm2d_ctx *c, int level, int32_t *sptr, int32_t *sidx, int32_t *wptr, int32_t *widx) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    TreeState &t = c->tree;
    if (t.L < 0 || !t.has_lists) return fail(c, FMM2D_ESTATE, "get_lists: no lists");
    if (level < 0 || level > t.L) return fail(c, FMM2D_EINVAL, "get_lists: level %d not in [0, %d]", level, t.L);
    CtxScope g(c);
    const int64_t nb = int64_t(1) << (2 * level);
    const int64_t ns = t.s_off[level + 1] - t.s_off[level], nw = t.w_off[level + 1] - t.w_off[level];
    hipError_t e = hipSuccess;
    if (sptr && e == hipSuccess)
        e = hipMemcpyAsync(sptr, t.sptr.as<int32_t>() + ptr_offset(level), sizeof(int32_t) * (nb + 1),
                           hipMemcpyDeviceToDevice, c->stream);
    if (wptr && e == hipSuccess)
        e = hipMemcpyAsync(wptr, t.wptr.as<int32_t>() + ptr_offset(level), sizeof(int32_t) * (nb + 1),
                           hipMemcpyDeviceToDevice, c->stream);
    if (sidx && ns > 0 && e == hipSuccess)
        e = hipMemcpyAsync(sidx, t.sidx.as<int32_t>() + t.s_off[level], sizeof(int32_t) * ns, hipMemcpyDeviceToDevice,
                           c->stream);
    if (widx && nw > 0 && e == hipSuccess)
        e = hipMemcpyAsync(widx, t.widx.as<int32_t>() + t.w_off[level], sizeof(int32_t) * nw, hipMemcpyDeviceToDevice,
                           c->stream);
    return e == hipSuccess ? FMM2D_OK : hip_fail(c, e, "get_lists");
}

int fmm2d_get_geometry(fmm2d_ctx *c, double *geom) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    const TreeState &t = c->tree;
    if (t.L < 0) return fail(c, FMM2D_ESTATE, "get_geometry: no tree");
    if (!geom) return fail(c, FMM2D_EINVAL, "get_geometry: NULL pointer");
    CtxScope g(c);
    const hipError_t e = hipMemcpyAsync(geom, t.geom.ptr, sizeof(double4) * level_offset(t.L + 1),
                                        hipMemcpyDeviceToDevice, c->stream);
    return e == hipSuccess ? FMM2D_OK : hip_fail(c, e, "get_geometry");
}

int fmm2d_get_xlists(fmm2d_ctx *c, int level, int64_t *nx, int32_t *xptr, int32_t *xidx) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    const TreeState &t = c->tree;
    if (!t.has_lists) return fail(c, FMM2D_ESTATE, "get_xlists: no lists");
    if (level < 0 || level > t.L) return fail(c, FMM2D_EINVAL, "get_xlists: level %d not in [0, %d]", level, t.L);
    const int64_t n = t.x_off[level + 1] - t.x_off[level];
    if (nx) *nx = n;
    CtxScope g(c);
    hipError_t e = hipSuccess;
    const int64_t rows = (int64_t(1) << (2 * level)) + 1;
    if (xptr) {
        const bool swaps = (t.opt & (FMM2D_OPT_SWAP_FINEST | FMM2D_OPT_SWAP_ALL)) != 0;
        e = swaps ? hipMemcpyAsync(xptr, t.xptr.as<int32_t>() + ptr_offset(level), sizeof(int32_t) * rows,
                                   hipMemcpyDeviceToDevice, c->stream)
                  : hipMemsetAsync(xptr, 0, sizeof(int32_t) * rows, c->stream);
    }
    if (xidx && n > 0 && e == hipSuccess)
        e = hipMemcpyAsync(xidx, t.xidx.as<int32_t>() + t.x_off[level], sizeof(int32_t) * n, hipMemcpyDeviceToDevice,
                           c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "get_xlists");
    return FMM2D_OK;
}

int fmm2d_timing(fmm2d_ctx *c, int enable) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    CtxScope g(c);
    if (enable) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return hip_fail(c, e, "timing");
        c->timer.marks.clear();
        c->timer.used = 0;
    }
    c->timer.on = enable != 0;
    return FMM2D_OK;
}

int fmm2d_get_timings(fmm2d_ctx *c, double *ms, int64_t *count) {
    if (!c) return FMM2D_EINVAL;
    c->err.clear();
    CtxScope g(c);
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess && c->side) e = hipStreamSynchronize(c->side);  // marks recorded on the second stream
    if (e != hipSuccess) return hip_fail(c, e, "get_timings");
    double acc[PH_COUNT] = {0};
    int64_t cnt[PH_COUNT] = {0};
    for (const auto &m : c->timer.marks) {
        float t = 0.f;
        if ((e = hipEventElapsedTime(&t, m.a, m.b)) != hipSuccess) return hip_fail(c, e, "get_timings");
        acc[m.phase] += t;
        cnt[m.phase] += 1;
    }
    for (int k = 0; k < PH_COUNT; ++k) {
        if (ms) ms[k] = acc[k];
        if (count) count[k] = cnt[k];
    }
    return FMM2D_OK;
}

}  // extern "C"
