// Pieces of the evaluation pass shared between the binary64 operators and the
// reduced-precision hot kernels.
#pragma once
#include "devutil.h"
#include "internal.h"

namespace fmm2d {

hipError_t ensure_binomials(fmm2d_ctx *c);
// constant M2L matrix (m2l.hip)
hipError_t ensure_mhat(fmm2d_ctx *c);
// M2L of all levels along their weak lists, in precision `mode`, into the
// segment partial sums ev.part that the L2L pass adds into B (m2l.hip).
hipError_t m2l_all(fmm2d_ctx *c, int p, int mode);
// L2P plus the near field at the leaves in precision `mode`; writes the
// potentials to phi in input order (near.hip).
// The leaf pass in three stages: NEAR_PREP packs the sources (and builds
// the full near-field schedule where it is needed) on the context stream and
// makes the context's second stream wait for that point; NEAR_LAUNCH queues
// the near-field kernels on the second stream (they need neither expansion);
// NEAR_FINISH makes the context stream wait for them and adds L2P and the
// near-field sums.  The far field runs in between.
enum { NEAR_PREP = 0, NEAR_LAUNCH = 1, NEAR_FINISH = 2 };
hipError_t leaf_pass(fmm2d_ctx *c, int p, int mode, int stage, double *phi);
// the gradient of the potential at every point, input order, after a
// binary64 evaluation with the same p (field.hip)
hipError_t gradient_device(fmm2d_ctx *c, int p, double *gx, double *gy);
// Exchanged roles (structural option, exchange.hip): the work items of the
// P2L side (target box, source box, point range), built with the schedules;
// per global box the range of its items (nullptr when the lists have no
// exchanged pair); P2L partials into ev.xpart (before the L2L pass, which
// adds them into B); M2P of the smaller boxes' multipoles: m2p_partials
// writes each item's sums at its points and describes them in ev.m2p (the
// leaf pass adds them per point, m2p_point_sum); above order 32, m2p_direct
// adds them into phi after the leaf pass instead.
hipError_t exchange_schedule(fmm2d_ctx *c);
const int32_t *exchange_item_offsets(fmm2d_ctx *c);
hipError_t p2l_all(fmm2d_ctx *c, int p);
hipError_t m2p_partials(fmm2d_ctx *c, int p);
hipError_t m2p_direct(fmm2d_ctx *c, int p, double *phi);

// The M2P sums at point i (leaf order) of leaf `leaf`: level by level, and
// within a level in item order (the row spans of the point's pass).  The item
// ranges and box starts of all levels are loaded before any is used.
__device__ inline double m2p_point_sum(const M2PSum &ms, int L, int64_t i, int64_t leaf,
                                       const int32_t *__restrict__ stL) {
    int32_t r0[FMM2D_MAX_LEVELS + 1], r1[FMM2D_MAX_LEVELS + 1], a0[FMM2D_MAX_LEVELS + 1];
#pragma unroll
    for (int l = 1; l <= FMM2D_MAX_LEVELS; ++l) {
        r0[l] = r1[l] = a0[l] = 0;
        if (l <= L) {
            const int64_t b = leaf >> (2 * (L - l)), g = level_offset(l) + b;
            r0[l] = ms.itemoff[g];
            r1[l] = ms.itemoff[g + 1];
            a0[l] = stL[b << (2 * (L - l))];  // the box's first point
        }
    }
    double acc = 0.0;
#pragma unroll
    for (int l = 1; l <= FMM2D_MAX_LEVELS; ++l) {
        if (l > L || r0[l] == r1[l]) continue;
        const int64_t b = leaf >> (2 * (L - l));
        const int32_t e = stL[(b + 1) << (2 * (L - l))];
        const int32_t a = a0[l], step = ms.w[l];
        const int32_t npc = (e - a + step - 1) / step, nsp = (r1[l] - r0[l]) / npc;
        const int32_t pc = ((int32_t)i - a) / step, o = (int32_t)i - a - pc * step;
        const double *row = ms.mpart + (int64_t)(r0[l] + pc * nsp) * 64 + o;
        for (int32_t s = 0; s < nsp; ++s) acc += row[(int64_t)s * 64];
    }
    return acc;
}
// list segments for the M2L and near-field kernels (sched.hip)
hipError_t build_schedules(fmm2d_ctx *c);
hipError_t ensure_near_full_schedule(fmm2d_ctx *c);
// Leaves of 17 to 64 points: the FP32 near field takes each leaf pair once
// (a leaf pair's 256 to 4096 point pairs then outweigh the per-record cost of
// the transposed positions); smaller leaves take every ordered pair.
inline bool pair_once_leaves(int64_t maxleaf) { return maxleaf > 16 && maxleaf <= 64; }

}  // namespace fmm2d
