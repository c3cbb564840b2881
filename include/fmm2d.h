/*
 * fmm2d.h -- C ABI of an MI355X (gfx950) implementation of the asymmetric
 * adaptive fast multipole method for the 2D logarithmic potential, after
 * S. Engblom, "On well-separated sets and fast multipole methods".
 *
 * The library computes, for points z_i = (x_i, y_i) with real charges q_i,
 *
 *     phi_i = sum_{j : z_j != z_i} q_j log|z_i - z_j|                  (1.1)
 *
 * (the interaction sum of eq. (1.1) with G = log|x - y| and charges; pairs at
 * one location are left out like j == i).  The three stages of Section 4 are
 * separate calls: the balanced median-split tree, the strong/weak
 * connectivity under the theta-criterion (Criterion 2.1), and the
 * evaluation of the expansions and of the near field.
 *
 * Conventions for every function:
 *  - Every function returns an int status: FMM2D_OK or a negative code.
 *    Nothing throws across the ABI.  On error, fmm2d_last_error() describes
 *    the failure.  Arguments are validated on the host before any launch,
 *    and a call that fails validation leaves the context unchanged.
 *  - Pointers documented as "device" are HIP device pointers on the
 *    context's device; the caller owns them.  Work is enqueued on the
 *    context's stream; device inputs must stay valid, and device outputs are
 *    complete, once that stream has passed the call (synchronise the stream
 *    before reading them on the host).  Pointers documented as "host" are
 *    ordinary host memory, read or written before the call returns.
 *  - A context is not thread-safe; use one context per host thread.
 *  - Device memory.  Every device byte the context uses (its tree, lists,
 *    expansions and scratch, kept and reused across calls) comes from the
 *    allocator given to fmm2d_create (e.g. a framework's caching allocator),
 *    or from hipMalloc when none is given; it is returned by fmm2d_destroy
 *    or when a buffer has to grow.  The only other memory is 128 bytes of
 *    pinned host memory (fmm2d_select_build_tree).
 *  - FMM2D_ENOMEM (an allocation failed) discards the results of the failing
 *    call's stage (a failing build_tree discards the tree, a failing
 *    connectivity the lists); earlier stages stay valid and the context
 *    stays usable.
 */
#ifndef FMM2D_H
#define FMM2D_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define FMM2D_OK          0
#define FMM2D_EINVAL     -1  /* an argument is out of range or NULL          */
#define FMM2D_ENOMEM     -2  /* a device allocation failed                    */
#define FMM2D_EDEVICE    -3  /* a HIP runtime error; see fmm2d_last_error()   */
#define FMM2D_ESTATE     -4  /* wrong call order (e.g. evaluate before lists) */
#define FMM2D_ECAPACITY  -5  /* a level's list exceeds what int32 list       */
                             /* offsets can address (fewer levels, or another */
                             /* theta, for this point set)                    */

/* Precision modes of fmm2d_evaluate.  In every mode the tree, the lists,
 * P2M, M2M, L2L and L2P run in binary64; the modes differ in the two hot
 * steps, the M2L conversion along the weak lists and the near-field sum.
 *   FP64        M2L and near field in binary64.
 *   FP32        M2L as an FP32 matrix product on the matrix cores with FP32
 *               accumulation and FP32 power scaling; near field in FP32 on
 *               box-local coordinates; FP32 accumulation.
 *   BF16X3      as FP32, with the M2L product done as three BF16 products of
 *               a two-way BF16 split of both operands.
 *   FP32_ACC64  as FP32, with the per-pair power scaling in binary64 and the
 *               M2L and near-field sums accumulated in binary64.           */
#define FMM2D_MODE_FP64        0
#define FMM2D_MODE_FP32        1
#define FMM2D_MODE_BF16X3      2
#define FMM2D_MODE_FP32_ACC64  3

#define FMM2D_MAX_LEVELS 13
#define FMM2D_MAX_P      63

typedef struct fmm2d_ctx fmm2d_ctx;

/* Library version (major*10000 + minor*100 + patch). */
int fmm2d_version(void);

/* Device memory callbacks.  alloc returns `bytes` of device memory on the
 * context's device, aligned to at least 256 bytes, or NULL when it cannot
 * (the call then fails with FMM2D_ENOMEM).  free returns a block alloc gave
 * (with the same size) in stream order: work the context queued on its
 * stream before the call may still be using it, so the block may be handed
 * out again only for work ordered after that point of the context stream
 * (the rule of a stream-ordered caching allocator that allocates on that
 * stream).  Work of the context's internal second stream is always ordered
 * before the context stream when free is called.  user is passed through. */
typedef void *(*fmm2d_alloc_fn)(size_t bytes, void *user);
typedef void (*fmm2d_free_fn)(void *ptr, size_t bytes, void *user);

/* Creates a context on HIP device `device` that enqueues all work on
 * `stream` (a hipStream_t; NULL means the device's null stream).  alloc and
 * free: both NULL (hipMalloc and hipFree, the host waiting for the
 * context's streams before a block is freed) or both set (see
 * fmm2d_alloc_fn).  *out receives the context.  FMM2D_EINVAL for a NULL
 * out, one callback without the other, or a device that does not exist. */
int fmm2d_create(fmm2d_ctx **out, int device, void *stream, fmm2d_alloc_fn alloc, fmm2d_free_fn free,
                 void *user);

/* Frees the context and returns all its device memory.  Synchronises its
 * streams first. */
int fmm2d_destroy(fmm2d_ctx *ctx);

/* Message of the last failing call on ctx (owned by ctx, valid until the
 * next call on it).  Returns "" when there was none, or a fixed message when
 * ctx is NULL. */
const char *fmm2d_last_error(const fmm2d_ctx *ctx);

/* Replaces the stream used by later calls; the new stream is made to wait
 * for the work queued so far on the old one. */
int fmm2d_set_stream(fmm2d_ctx *ctx, void *stream);

/* Options of the trees built from now on (fmm2d_build_tree,
 * fmm2d_select_build_tree), combined with |:
 *   FMM2D_TREE_SHRINK  the ball of each box in Criterion 2.1, and the centre
 *                      and scale of its expansions, are those of its points'
 *                      bounding box (centre, half diagonal) instead of its
 *                      tiling rectangle: the smallest axis-aligned box
 *                      around the points (Criterion 2.1 is stated for any
 *                      balls enclosing the two sets).  The boxes and their
 *                      points are unchanged.
 * FMM2D_EINVAL for unknown bits. */
#define FMM2D_TREE_SHRINK 1
int fmm2d_set_tree_options(fmm2d_ctx *ctx, int flags);

/* Builds the balanced pyramid (Section 4 and Fig. 1.1).  x, y: device,
 * binary64 [n], every value finite with |value| <= 2^500.  levels: 0..13,
 * with n >= 4^levels (every box must split) and n <= 2^31 - 1.
 *
 * Each box is split along x so that its floor(m/2) first members in
 * (x, original index) order go low, then each half is split along y the same
 * way with (y, index); the children of box b are 4b + 2*[x high] + [y high]
 * and a split line is the midpoint of the two straddling coordinates.  The
 * root is the tight bounding box.  Inside each leaf, points are kept in
 * (x, index) order.  Replaces any earlier tree and invalidates the lists. */
int fmm2d_build_tree(fmm2d_ctx *ctx, const double *x, const double *y,
                     int64_t n, int levels);

/* Builds the strong and weak interaction lists of every level (Section 4)
 * with the theta-criterion R + theta r <= theta d on the boxes' enclosing
 * balls (centre of the rectangle, half its diagonal).  0 < theta < 1.
 * Needs a tree.  Synchronises the stream once (to size the lists), more
 * often when the lists outgrow the pools of earlier calls.
 * FMM2D_ECAPACITY when a level's candidates (16 times the previous level's
 * strong entries) exceed 2^31 - 1, or all lists together 2^34 entries. */
int fmm2d_connectivity(fmm2d_ctx *ctx, double theta);

/* Structural options of the connectivity (Section 4's optional
 * optimisations), combined with |:
 *   FMM2D_OPT_PARENT       a box b for which all four children of a box q of
 *                          S(parent(b)) pass the criterion, and q itself
 *                          passes it against b, interacts with q (a box of
 *                          the level above) instead of the four children:
 *                          the weak list of b then holds q | FMM2D_VFLAG.
 *   FMM2D_OPT_SWAP_FINEST  at the finest level, a strong pair of boxes whose
 *                          criterion holds with the radii's roles exchanged,
 *                          r + theta R <= theta d (R the larger radius), on
 *                          disjoint balls (d > R + r), leaves the strong list
 *                          for the exchanged list X: the sources of the larger
 *                          box become a local expansion about the smaller
 *                          (P2L) and the multipole of the smaller is evaluated
 *                          at the points of the larger (M2P).
 *   FMM2D_OPT_SWAP_ALL     the same at every level; an exchanged pair is not
 *                          refined further (its children are no candidates).
 * Every list stays ascending (a V entry sorts as its box q among the
 * children of the level above's boxes). */
#define FMM2D_OPT_PARENT       1
#define FMM2D_OPT_SWAP_FINEST  2
#define FMM2D_OPT_SWAP_ALL     4
#define FMM2D_VFLAG            0x40000000

/* fmm2d_connectivity with structural options `opt` (FMM2D_OPT_*, 0 gives
 * exactly fmm2d_connectivity).  Later evaluations use the extra lists.
 * FMM2D_EINVAL for unknown bits.  fmm2d_evaluate_field needs opt = 0. */
int fmm2d_connectivity_opt(fmm2d_ctx *ctx, double theta, int opt);

/* The plain lists under a locally relaxed theta-criterion (Section 4, last
 * paragraph: differing theta_i are admissible while the mean of
 * theta_i^(p+1) over the observed values stays at most theta^(p+1)).
 * A pair's theta_i is read on a grid of k0 + k1 thresholds,
 *     t_k = theta (k + 1) / k0                             k < k0
 *     t_k = theta + (theta_max - theta) (k - k0 + 1) / k1   k >= k0
 * (binary64, evaluated as written; t_{k0-1} = theta): a candidate's bin is
 * the least k at which the criterion holds.  On every level the bins are
 * counted, and bins 0..K are weak for the largest K >= k0 - 1 such that for
 * each k from k0 - 1 to K
 *     sum_{j<=k} count_j t_j^(p+1) <= theta^(p+1) sum_{j<=k} count_j
 * (powers by p repeated products, sums in bin order, binary64); the other
 * candidates are strong.  theta_max = theta gives fmm2d_connectivity's
 * lists.  p is the expansion order the lists are meant for (later
 * evaluations may use any order).  0 < theta <= theta_max < 1,
 * 0 <= p <= 1024, k0, k1 >= 1, k0 + k1 <= 256; FMM2D_EINVAL otherwise,
 * FMM2D_ESTATE without a tree, FMM2D_ECAPACITY as fmm2d_connectivity.
 * Synchronises the stream as fmm2d_connectivity does. */
int fmm2d_connectivity_relaxed(fmm2d_ctx *ctx, double theta, double theta_max, int p, int k0, int k1);

/* The bin counts and admitted bins of the lists built by
 * fmm2d_connectivity_relaxed.  count: host int64 [(L + 1) (k0 + k1)], level
 * by level (level 0 all zero); kmax: host int32 [L + 1], the last weak bin
 * of each level (k0 - 1 for level 0).  FMM2D_ESTATE unless the current
 * lists came from fmm2d_connectivity_relaxed.  Synchronises the stream. */
int fmm2d_get_relax_bins(fmm2d_ctx *ctx, int64_t *count, int32_t *kmax);

/* Evaluates phi (eq. (1.1)) with expansion order p (degrees 0..p, so p + 1
 * coefficients per expansion), 1 <= p <= 63, in precision `mode`
 * (FMM2D_MODE_*).  q: device binary64 [n] charges in input order.  phi:
 * device binary64 [n] output in input order.  Needs tree and lists.
 * The FP32 modes (FP32, BF16X3, FP32_ACC64) compute on offsets from leaf
 * centres and need the root box's half diagonal in [2^-60, 2^56] (or 0):
 * FMM2D_EINVAL otherwise (FMM2D_MODE_FP64 has no such limit).
 * Asynchronous on the stream. */
int fmm2d_evaluate(fmm2d_ctx *ctx, const double *q, int p, int mode, double *phi);

/* As fmm2d_evaluate, and the gradient of phi at every point: gx = d phi/dx,
 * gy = d phi/dy, i.e. sum over j with z_j != z_i of q_j (z_i - z_j) /
 * |z_i - z_j|^2 componentwise (the field of the logarithmic kernel; Section
 * 5's first experiment measures the corresponding force kernel).  The far
 * part is the derivative of each leaf's local expansion, the near part the
 * direct sum over the finest strong list.  Binary64 only: mode must be
 * FMM2D_MODE_FP64 (FMM2D_EINVAL otherwise).  q, phi, gx, gy: device binary64
 * [n], input order; phi equals what fmm2d_evaluate writes.  Needs tree and
 * lists.  Asynchronous on the stream. */
int fmm2d_evaluate_field(fmm2d_ctx *ctx, const double *q, int p, int mode, double *phi, double *gx, double *gy);

/* Direct binary64 sum (eq. (1.1)) at m target indices, with compensated
 * summation: the error judge.  x, y, q: device binary64 [n]; targets: device
 * int64 [m] with values in [0, n); phi_m: device binary64 [m].  Independent
 * of any tree.  Synchronises the stream once (the target check: FMM2D_EINVAL
 * for an index outside [0, n)); the sum itself is queued. */
int fmm2d_direct(fmm2d_ctx *ctx, const double *x, const double *y, const double *q,
                 int64_t n, const int64_t *targets, int64_t m, double *phi_m);

/* fmm2d_direct without any device allocation, for callers that cannot
 * allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid it).  Same arguments, results and target check as
 * fmm2d_direct (the same kernels, so bit-identical results); the chunk
 * partials and the check flag live in a fixed device array of 4 MiB + 256
 * bytes that the library holds on every device it runs on until the process
 * ends.  m <= 262144 (FMM2D_EINVAL beyond).  Every call on a device
 * shares that device's array: calls that overlap on one device (several
 * contexts or streams) race and must be serialised by the caller.  No
 * timing is recorded.  Synchronises the stream once (the target check). */
int fmm2d_direct_noalloc(fmm2d_ctx *ctx, const double *x, const double *y, const double *q,
                         int64_t n, const int64_t *targets, int64_t m, double *phi_m);

/* The direct gradient of the same sum at m target indices, the judge of
 * fmm2d_evaluate_field: gx_m, gy_m (device binary64 [m]) receive the sums over
 * j with z_j != z_i of q_j (x_i - x_j) / |z_i - z_j|^2 and q_j (y_i - y_j) /
 * |z_i - z_j|^2, compensated.  Arguments and errors as fmm2d_direct. */
int fmm2d_direct_field(fmm2d_ctx *ctx, const double *x, const double *y, const double *q,
                       int64_t n, const int64_t *targets, int64_t m, double *gx_m, double *gy_m);

/* ---- parameter selection -------------------------------------------------- */

/* Density features of a point set (the selector's input), FMM2D_NFEAT floats:
 *   [0] log10 n, [1] log10 tol, then for each level l = 1..10 of a uniform
 *   2^l x 2^l grid over the points' tight bounding box, 9 values:
 *   the fraction of occupied cells, then the fractions of the n points whose
 *   cell has relative density r = count 4^l / n in bin k = 0..7, where k is
 *   the number of the edges 1/8, 1/4, 1/2, 1, 2, 4, 8 that are <= r.
 * A point's cell along x is floor((x - xmin) 1024 / (xmax - xmin)) clamped
 * to [0, 1023] at level 10 (0 when xmax = xmin), shifted right by 10 - l for
 * level l; likewise along y (bounding box of all points).  Cells are counted
 * over every s-th point, s = ceil(n / 2^18) (all points when n <= 2^18); the
 * densities and fractions then refer to that sample's size.  Counts are
 * exact integers, so the output is deterministic.
 * x, y: device double [n]; feat: device float [FMM2D_NFEAT].
 * 1 <= n <= 2^31 - 1, 0 < tol < 1.  Coordinates are not validated here. */
#define FMM2D_NFEAT 92
int fmm2d_features(fmm2d_ctx *ctx, const double *x, const double *y, int64_t n, double tol, float *feat);

/* Chooses (levels, p, theta) for tolerance tol on the points x, y.
 * weights: device float blob of a trained selector, or NULL:
 *   [0, 92)    mean of each feature
 *   [92, 184)  1 / standard deviation of each feature (network input is
 *              (feature - mean) * scale)
 *   [184, 187) mean of the three targets (levels - L0, log10 C, theta)
 *   [187, 190) standard deviation of the three targets
 *   [190, 194) trained range: log10 n low, high, log10 tol low, high
 *   [194, 194 + fmm2d_mlp_nparams(92)) network parameters (see fmm2d_mlp_forward)
 * With weights and inputs inside the trained range, the network's outputs
 * (de-standardised) give levels = round(L0 + out0) with L0 =
 * round(log4(n / 16)), theta = out2 snapped to {0.35, 0.45, 0.55, 0.65,
 * 0.75}, and, with out1 = log10 C of an error model e(p) = C theta^(p+1)
 * (the form of the truncation bound of Section 3), p = ceil((log10(tol / 2)
 * - out1) / log10 theta) - 1: the least order the model says meets tol / 2
 * (a safety factor of 2 on the error).
 * Otherwise (NULL weights, n or tol outside the range, non-finite output)
 * the a-priori rule, the practical choice at the end of Section 4: theta =
 * 1/2, levels = round(log4(n / 20)) (about 20 points per leaf), p = the least
 * p with 0.1 theta^(p+1) / (1 - theta)^2 <= tol (the truncation bound of
 * Section 3 with a calibrated constant).  round() is round-half-up.  levels is clamped to
 * [1, min(13, floor(log4 n))] and p to [1, 63].
 * Host outputs levels, p, theta; from_network (may be NULL) is 1 when the
 * network decided, 0 for the rule.  4 <= n <= 2^31 - 1, 0 < tol < 1.
 * Returns FMM2D_EINVAL for non-finite coordinates or |v| > 2^500.
 * Synchronises the context stream. */
#define FMM2D_SELECT_HEADER 194
int fmm2d_select(fmm2d_ctx *ctx, const double *x, const double *y, int64_t n, double tol, const float *weights,
                 int *levels, int *p, double *theta, int *from_network);

/* fmm2d_select followed by fmm2d_build_tree(x, y, n, *levels): the same
 * decision and the same tree (Section 2's partition at the selected level
 * count), in one call.  The sort of the coordinates, which does not depend on
 * the level count, runs on the context stream while the features and the
 * network run on the context's second stream, and the host waits once, for
 * the decision and the validation together (pinned host words owned by the
 * context); then the partition is queued.  All eight radix digits are sorted
 * (fmm2d_build_tree skips digits on which all keys agree, which it learns
 * from an extra wait).  Arguments and outputs as fmm2d_select; 4 <= n <=
 * 2^31 - 1, 0 < tol < 1.  FMM2D_EINVAL for non-finite coordinates or
 * |v| > 2^500: unlike fmm2d_build_tree, the previous tree is then discarded
 * (the sort has already overwritten its sorted arrays), and connectivity or
 * evaluate fail until a tree is built.  Returns with the partition queued on
 * the context stream. */
int fmm2d_select_build_tree(fmm2d_ctx *ctx, const double *x, const double *y, int64_t n, double tol,
                            const float *weights, int *levels, int *p, double *theta, int *from_network);

/* The selector network: d_in -> 64 -> 64 -> 64 -> 3, tanh on the hidden
 * layers, linear output, FP32.  The flat parameter vector holds each layer
 * in turn as its weight matrix [fan_out][fan_in] (row-major) followed by its
 * bias.  Returns the parameter count, or -1 for d_in outside [1, 128]. */
#define FMM2D_MLP_MAX_IN 128
int64_t fmm2d_mlp_nparams(int d_in);

/* Y[batch][3] = network(X[batch][d_in]).  All device float, row-major. */
int fmm2d_mlp_forward(fmm2d_ctx *ctx, const float *params, const float *X, int64_t batch, int d_in, float *Y);

/* Mean-squared error over all batch x 3 outputs against Y, into *loss
 * (device float [1]), and its gradient with respect to params into grad
 * (device float [nparams]).  The sum over samples has a fixed order.
 * batch <= 2^24. */
int fmm2d_mlp_grad(fmm2d_ctx *ctx, const float *params, const float *X, const float *Y, int64_t batch, int d_in,
                   float *grad, float *loss);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected moments;
 * step counts from 1) on params with moments m, v, all device float
 * [nparams], updated in place.  weight_decay >= 0 adds the gradient of the
 * L2 penalty (weight_decay / 2) |params|^2 before the moments are updated
 * (0: plain Adam).  FMM2D_EINVAL for lr <= 0, weight_decay < 0 or NaN. */
int fmm2d_mlp_adam(fmm2d_ctx *ctx, float *params, float *m, float *v, const float *grad, int64_t nparams, int step,
                   float lr, float weight_decay);

/* ---- introspection (used by the parity tests) ---------------------------- */

/* Host outputs: number of points, levels and boxes of the current tree. */
int fmm2d_tree_info(const fmm2d_ctx *ctx, int64_t *n, int *levels, int64_t *nbox);

/* Device output int32 [n]: original index of each point in leaf order. */
int fmm2d_get_perm(fmm2d_ctx *ctx, int32_t *perm);

/* Device output int32 [4^levels + 1]: first position of each leaf in perm. */
int fmm2d_get_leaf_start(fmm2d_ctx *ctx, int32_t *start);

/* Device output binary64 [nbox][4]: (xlo, xhi, ylo, yhi) of every box, level
 * by level, level l starting at box (4^l - 1)/3. */
int fmm2d_get_rects(fmm2d_ctx *ctx, double *rects);

/* Device output binary64 [nbox][4]: (cx, cy, r, scale) of every box: the
 * centre and radius of its ball (Criterion 2.1) and the scale of its
 * expansions (r, or 1 for a box of zero size). */
int fmm2d_get_geometry(fmm2d_ctx *ctx, double *geom);

/* Host outputs: number of strong and weak list entries at `level`. */
int fmm2d_list_sizes(const fmm2d_ctx *ctx, int level, int64_t *n_strong, int64_t *n_weak);

/* Device outputs for one level: CSR row pointers int32 [4^level + 1] and
 * column indices (box numbers within the level, ascending per row) of the
 * strong list S and the weak list W (with FMM2D_OPT_PARENT, entries with
 * FMM2D_VFLAG set are boxes of level - 1).  Any pointer may be NULL to skip
 * it. */
int fmm2d_get_lists(fmm2d_ctx *ctx, int level, int32_t *sptr, int32_t *sidx,
                    int32_t *wptr, int32_t *widx);

/* Exchanged-roles list of one level (empty unless the lists were built with
 * a swap option): host output *nx (entry count); device outputs xptr int32
 * [4^level + 1] and xidx (box numbers within the level, ascending per row),
 * either may be NULL. */
int fmm2d_get_xlists(fmm2d_ctx *ctx, int level, int64_t *nx, int32_t *xptr, int32_t *xidx);

/* ---- per-phase GPU timing ------------------------------------------------ */

/* Phases timed by fmm2d_get_timings (index into its output arrays). */
#define FMM2D_PHASE_TREE    0  /* build_tree: sorts, splits, geometry, gather */
#define FMM2D_PHASE_LISTS   1  /* connectivity                                */
#define FMM2D_PHASE_UPWARD  2  /* P2M and M2M                                 */
#define FMM2D_PHASE_M2L     3  /* M2L along the weak lists (all levels)       */
#define FMM2D_PHASE_L2L     4  /* L2L, with the M2L sums added into B         */
#define FMM2D_PHASE_LEAF    5  /* L2P plus the near field (one launch)        */
#define FMM2D_PHASE_OTHER   6  /* charge gather, scatter to input order       */
#define FMM2D_PHASE_JUDGE   7  /* fmm2d_direct                                */
#define FMM2D_PHASE_SELECT  8  /* parameter selection                         */
/* Single kernel launches, also counted in their phase above:                 */
#define FMM2D_PHASE_NEAR_KERNEL  9  /* the near-field kernel (in LEAF)       */
#define FMM2D_PHASE_M2L_KERNEL  10  /* the M2L kernel, all levels (in M2L)   */
#define FMM2D_PHASE_EXCHANGE    11  /* P2L and M2P of exchanged-roles pairs  */
#define FMM2D_PHASE_P2L_KERNEL  12  /* the P2L kernels (in EXCHANGE)         */
#define FMM2D_PHASE_M2P_KERNEL  13  /* the M2P kernels (in EXCHANGE; their  */
                                    /* sums are added per point in LEAF)    */
#define FMM2D_NPHASE       14

/* enable = 1 clears the accumulated timings and starts recording HIP events
 * on the context stream around each phase; enable = 0 stops recording. */
int fmm2d_timing(fmm2d_ctx *ctx, int enable);

/* Host outputs ms[FMM2D_NPHASE] (accumulated GPU milliseconds) and
 * count[FMM2D_NPHASE] (number of timed intervals) since timing was enabled.
 * Synchronises the context stream.  Either pointer may be NULL. */
int fmm2d_get_timings(fmm2d_ctx *ctx, double *ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* FMM2D_H */
