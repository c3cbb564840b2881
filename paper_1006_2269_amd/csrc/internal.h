// Internal declarations of the fmm2d HIP library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/fmm2d.h"

namespace fmm2d {

constexpr int WAVE = 64;

// Global id of the first box of level l: (4^l - 1) / 3.
__host__ __device__ inline int64_t level_offset(int l) { return ((int64_t(1) << (2 * l)) - 1) / 3; }
// Offset of level l in an array holding (4^m + 1) entries per level m.
__host__ __device__ inline int64_t ptr_offset(int l) { return level_offset(l) + l; }
// Level of global box id g (levels stored one after the other).
__host__ __device__ inline int level_of(int64_t g) {
    int l = 0;
    while (level_offset(l + 1) <= g) ++l;
    return l;
}
// Offset of depth d in an array holding (2^e + 1) entries per depth e.
__host__ __device__ inline int64_t depth_offset(int d) { return ((int64_t(1) << d) - 1) + d; }

// Growable device buffer owned by the context.  Its memory comes from the
// allocator of the context whose API call is running on this thread (the
// callbacks given to fmm2d_create, else hipMalloc); see CtxScope in api.hip.
// A regrown buffer's old memory is returned only after all work queued on
// either stream that may still use it: with callbacks, the context stream
// first waits for the second stream and the memory is handed back in stream
// order; with hipMalloc, the host waits for both streams before hipFree.
struct DevBuf {
    void *ptr = nullptr;
    size_t cap = 0;
    hipError_t ensure(size_t bytes);  // at least `bytes`; old contents are not kept
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// Segments of a CSR list for the list-driven kernels (sched.hip).
struct Schedule {
    DevBuf segoff;          // int32 [rows + 1]: first segment of each row; [rows] = count
    DevBuf table;           // int2 [bound]: (row, first entry) of each segment
    int64_t bound = 0;      // upper bound of the segment count (launch size)
};
constexpr int M2L_SEG = 256;   // weak-list entries per M2L segment
constexpr int NEAR_SEG = 64;   // strong-list entries per near-field segment

// Everything a tree and its lists leave on the device.
struct TreeState {
    int64_t n = 0;
    int L = -1;
    // sorted coordinates and the x-order permutation
    DevBuf xsorted, ysorted, xorder;
    // rank lists (structure of arrays): XL sorted by x rank within segments,
    // YL sorted by y rank within segments; each holds (x rank, y rank)
    DevBuf XLx, XLy, YLx, YLy, T0, T1;
    DevBuf starts;          // int32, all depths 0..2L, (2^d + 1) entries each
    DevBuf rects;           // double [nbox][4]
    DevBuf prect;           // double [nbox][4]: bounding box of each box's points (tree option SHRINK)
    bool shrink = false;    // geometry (balls, leaf offsets) from the points' bounding boxes
    DevBuf geom;            // double4 [nbox]: cx, cy, r, scale
    DevBuf perm;            // int32 [n]
    DevBuf leafid;          // int32 [n]: leaf of each leaf-ordered point
    DevBuf px, py;          // double [n], leaf order
    DevBuf loc;             // float2 [n], offsets from the leaf centre
    // lists: row pointers of every level (ptr_offset), index pools
    DevBuf sptr, wptr, sidx, widx, cnt_s, cnt_w;
    // exchanged-roles lists (structural option): row pointers of every level,
    // index pool, per-word counts
    DevBuf xptr, xidx, cnt_x;
    int opt = 0;            // FMM2D_OPT_* flags the lists were built with
    DevBuf bits;            // uint64: theta decisions of one level's candidates
    DevBuf owner0, owner1;  // int32: row (box) of each S entry of a level, by level parity
    DevBuf selfpos;         // int32 [4^L]: position of leaf b in S_L(b) (level-relative)
    DevBuf trans;           // int32 per S_L record t = (b, c) with c > b: the position of b in S_L(c)
    DevBuf spart;           // float: source-side near-field partial sums per S_L record and source lane
    DevBuf pool_state;      // int64 [3 (L+2) + 1]: s, w, x offsets, overflow
    DevBuf nrec_j, nrec_d;  // per finest-level strong entry: source range; 2 float4 (FP32 centre offset, thresholds, low part)
    // relaxed criterion (fmm2d_connectivity_relaxed): thresholds t_k and
    // t_k^(p+1) (double [nbin] each), candidates per bin and level (uint32
    // [(L+1) nbin]), each level's admitted threshold (double [L+1]) and last
    // admitted bin (int32 [L+1]); relax_nbin 0 when the lists are plain
    DevBuf relax_tk, relax_hist, relax_lv, relax_k;
    std::vector<double> relax_host;  // t_k then t_k^(p+1), the source of the copy to relax_tk
    int relax_nbin = 0, relax_k0 = 0;
    bool nrec_valid = false;
    Schedule m2l_all;               // weak lists of all levels (rows = global box ids)
    Schedule near_seg;              // finest-level strong lists (built on first use)
    bool near_seg_ready = false;
    Schedule near_up;               // finest-level strong lists from each leaf's own entry on
    Schedule near_lo;               // the same lists before each leaf's own entry
    // exchanged roles: P2L work items int4 (target box, source box, first
    // point, end point), global ids; per global box its first item (+ count)
    DevBuf x_items, x_itemoff;
    int64_t x_bound_wave = 0;       // upper bound of the wavefront-per-item P2L items (launch size)
    int64_t x_bound_lane = 0;       // ... of the lane-per-item ones
    int x_lane_level = 0;           // first level of lane-per-item P2L (all deeper levels too)
    // M2P work items int4 (target box, first point, row span start, end) per
    // box, level by level; per global box its first item (+ count)
    DevBuf m_items, m_itemoff;
    int m_wide_level = 0;           // first level whose M2P pass is narrower than 64 points
    int64_t m_bound_wide = 0;       // upper bound of the M2P items of the levels before it (launch size)
    int64_t m_bound_narrow = 0;     // ... of the levels from it on
    bool x_ready = false;
    DevBuf lsum;                    // double: per near_lo segment and source lane, its entries' source sums
    std::vector<int64_t> s_off, w_off, x_off;  // host copy: pool offset of each level
    bool has_lists = false;
    double theta = 0.0;
    double root_r = 0.0;            // half diagonal of the root box (host copy, read with the lists)
};

// The M2P sums of the exchanged-roles items for the near-field reduction
// (a kernel argument): per global box its first M2P item (+ count), each
// item's sums at its points (64 doubles), and every level's pass width; no
// M2P sums when itemoff is null.
struct M2PSum {
    const int32_t *itemoff = nullptr;
    const double *mpart = nullptr;
    int32_t w[FMM2D_MAX_LEVELS + 1] = {};
};

struct EvalState {
    DevBuf binom;           // double [128][128] binomial coefficients
    bool binom_ready = false;
    DevBuf mhat;            // double [64][64] rescaled constant M2L matrix
    bool mhat_ready = false;
    DevBuf A, B;            // expansions, complex<double> [nbox][p+1]
    DevBuf qs;              // double [n] charges in leaf order
    DevBuf work;            // mode-dependent scratch
    DevBuf src;             // float4 [n]: FP32 local offsets and charge
    DevBuf srclo;           // float2 [n]: low parts of the offsets (FP32_ACC64's two-part differences)
    DevBuf part;            // partial sums of the M2L's list segments
    DevBuf npart;           // near-field partial sums (written on the second stream while the far field runs)
    DevBuf gpart;           // near-field gradient partial sums (fmm2d_evaluate_field)
    DevBuf xpart;           // P2L partial expansions of the exchanged-roles items
    DevBuf xsum;            // their sum per target box (boxes with items)
    DevBuf mpart;           // double [M2P items][64]: each item's sums at its points
    M2PSum m2p;             // the M2P sums of this evaluation (set before the leaf pass finishes)
};

// Per-phase GPU time, measured with HIP events recorded on the context stream
// around each phase's launches while timing is enabled.
enum Phase {
    PH_TREE = 0, PH_LISTS, PH_UPWARD, PH_M2L, PH_L2L, PH_LEAF, PH_OTHER, PH_JUDGE, PH_SELECT,
    PH_NEAR_KERNEL, PH_M2L_KERNEL,  // single launches inside PH_LEAF / PH_M2L
    PH_EXCHANGE,                    // P2L and M2P of the exchanged-roles pairs
    PH_P2L_KERNEL, PH_M2P_KERNEL,   // single launches inside PH_EXCHANGE
    PH_COUNT
};

struct PhaseTimer {
    bool on = false;
    struct Mark {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    std::vector<Mark> marks;
    hipEvent_t next() {
        if (used == pool.size()) {
            hipEvent_t e = nullptr;
            if (hipEventCreate(&e) != hipSuccess) return nullptr;
            pool.push_back(e);
        }
        return pool[used++];
    }
};

struct Scratch {
    DevBuf keys0, keys1, vals0, vals1, hist, aux, tiles, tiles2, segbase, thr, split0, split1, flag, segcnt, mcnt;
    DevBuf sel, sel2;        // selector: counts and features; decision
    int64_t sort_n = -1;     // size of the validated keys waiting in keys0 / vals0, or -1
    uint64_t sort_differ = 0;  // bits in which the keys of either coordinate differ
};

}  // namespace fmm2d

struct fmm2d_ctx {
    int device = 0;
    // device memory: the caller's callbacks, or hipMalloc / hipFree when NULL
    fmm2d_alloc_fn alloc = nullptr;
    fmm2d_free_fn free = nullptr;
    void *user = nullptr;
    int64_t list_limit = 2147483647LL;  // entries per level and list (FMM2D_LIST_LIMIT lowers it)
    int64_t cap_hint_s = 0, cap_hint_w = 0, cap_hint_x = 0;  // list pool sizes that sufficed last time
    int tree_opt = 0;       // FMM2D_TREE_* for the next trees (fmm2d_set_tree_options)
    hipStream_t stream = nullptr;
    // internal stream for work that may overlap the caller's stream (created
    // on first use, default priority); ev_side_out marks the end of the last
    // batch, which the caller's stream waits for before using its results
    hipStream_t side = nullptr;
    hipEvent_t ev_side_in = nullptr, ev_side_out = nullptr;
    bool side_pending = false;
    // fmm2d_select_build_tree: pinned host words for the two decisions read
    // back without a stream-wide wait, and the events after their copies
    void *hpin = nullptr;
    hipEvent_t ev_keys = nullptr, ev_sel = nullptr;
    std::string err;
    fmm2d::TreeState tree;
    fmm2d::EvalState ev;
    fmm2d::Scratch scr;
    fmm2d::PhaseTimer timer;
};

namespace fmm2d {

// ---- launchers (each returns the launch's hipError_t) ---------------------
// sort.hip: stable sort of both coordinates by (value, index).  sort_prepare
// validates (finite, |v| <= 2^500) and touches scratch memory only;
// sort_finish completes the sort of the keys sort_prepare left.
hipError_t sort_prepare(fmm2d_ctx *c, const double *x, const double *y, int64_t n, bool *bad_input);
hipError_t sort_finish(fmm2d_ctx *c, int64_t n, double *xs, double *ys, int32_t *xorder, int32_t *yorder,
                       int32_t *xrank, int32_t *yrank);
// The keys and the validation without waiting: the AND / OR / bad words of
// both coordinates (6 x u64) are copied to host memory h_andor and event ev
// recorded after the copy; then every digit is treated as differing, so that
// sort_finish can be queued before the host has read them.
hipError_t sort_prepare_async(fmm2d_ctx *c, const double *x, const double *y, int64_t n,
                              unsigned long long *h_andor, hipEvent_t ev);
// sched.hip: the side stream (see fmm2d_ctx): begin a batch after the work
// queued so far on the caller's stream, end it, and make the caller's stream
// wait for the last batch
hipError_t side_begin(fmm2d_ctx *c);
hipError_t side_end(fmm2d_ctx *c);
hipError_t side_join(fmm2d_ctx *c);
// scan.hip: exclusive scan of int32 in[n] into out[n+1] (out[n] = total)
hipError_t scan_exclusive(fmm2d_ctx *c, const int32_t *in, int64_t n, int32_t *out);
// the same for k (1 or 2) arrays of one length, in the same launches
hipError_t scan_exclusive_n(fmm2d_ctx *c, int k, const int32_t *const *in, int64_t n, int32_t *const *out);
// select.hip: density features and the parameter decision (host outputs)
hipError_t features_device(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol, float *feat,
                           const float *blob, float *xin, double **box_out, hipStream_t st = nullptr);
hipError_t select_device(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol, const float *blob,
                         int out[4], double *theta);
hipError_t select_launch(fmm2d_ctx *c, hipStream_t st, const double *x, const double *y, int64_t n, double tol,
                         const float *blob, int *h_out, double *h_theta);
// mlp.hip: the selector network
int64_t mlp_nparams(int d_in);
hipError_t mlp_forward(fmm2d_ctx *c, const float *P, const float *X, int64_t batch, int d_in, float *Y,
                       hipStream_t st = nullptr);
hipError_t mlp_grad(fmm2d_ctx *c, const float *P, const float *X, const float *Y, int64_t batch, int d_in,
                    float *grad, float *loss);
hipError_t mlp_adam(fmm2d_ctx *c, float *P, float *m, float *v, const float *g, int64_t np, int step, float lr,
                    float wd);
// tree.hip: the tree at t.n points and t.L levels; `sorted`: tree_sort(c,
// t.n) is already queued on the context stream
hipError_t tree_sort(fmm2d_ctx *c, int64_t n);
hipError_t build_tree_device(fmm2d_ctx *c, const double *x, const double *y, bool sorted = false);
// lists.hip
// overflow: 0 ok, 2 a level exceeds `limit` entries, else the LIST_GROW_* bits of the pools
// to grow before a retry;
// opt: FMM2D_OPT_* (0: the plain lists)
constexpr int LIST_GROW_S = 4, LIST_GROW_W = 8, LIST_GROW_X = 16, LIST_GROW_CAND = 32;
// rx (plain lists with the relaxed criterion) or nullptr
struct RelaxRule {
    double theta, theta_max, etheta;  // etheta = theta^(p+1) by p repeated products
    int p, k0, k1;
};
constexpr int RELAX_MAX_BINS = 256;
hipError_t build_lists_device(fmm2d_ctx *c, double theta, int opt, int64_t cap_s, int64_t cap_w, int64_t cap_x,
                              int64_t limit, int *overflow, const RelaxRule *rx = nullptr);
// expand.hip
hipError_t evaluate_device(fmm2d_ctx *c, const double *q, int p, int mode, double *phi);
// judge.hip
hipError_t direct_device(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                         const int64_t *targets, int64_t m, double *phi);
// the judge on the fixed per-device array (fmm2d_direct_noalloc): its
// address on `device` (looked up on first use, that device current), whether
// the partials of n sources and m targets fit, and the launches (target check first:
// *bad_target and nothing queued when an index is outside [0, n))
hipError_t noalloc_scratch(int device, void **ptr);
bool noalloc_fits(int64_t n, int64_t m);
hipError_t direct_noalloc_device(fmm2d_ctx *c, void *scr, const double *x, const double *y, const double *q,
                                 int64_t n, const int64_t *targets, int64_t m, double *phi, bool *bad_target);
hipError_t direct_grad_device(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                              const int64_t *targets, int64_t m, double *gx, double *gy);

// Brackets the launches of one phase with two events when timing is on.
struct PhaseScope {
    fmm2d_ctx *c;
    int phase;
    hipEvent_t a = nullptr;
    hipStream_t s;
    // ph < 0: not timed; stream: the context stream unless given
    PhaseScope(fmm2d_ctx *ctx, int ph, hipStream_t stream = nullptr) : c(ctx), phase(ph), s(stream) {
        if (!s) s = c->stream;
        if (ph >= 0 && c->timer.on && (a = c->timer.next())) (void)hipEventRecord(a, s);
    }
    ~PhaseScope() {
        if (a) {
            hipEvent_t b = c->timer.next();
            if (b && hipEventRecord(b, s) == hipSuccess) c->timer.marks.push_back({phase, a, b});
        }
    }
};

inline unsigned grid_for(int64_t work, int per_block) {
    int64_t g = (work + per_block - 1) / per_block;
    return (unsigned)(g < 1 ? 1 : g);
}

}  // namespace fmm2d

#define FMM2D_TRY(expr)                          \
    do {                                         \
        hipError_t e__ = (expr);                 \
        if (e__ != hipSuccess) return e__;       \
    } while (0)
