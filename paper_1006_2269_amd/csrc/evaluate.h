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
// adds them into B); M2P of the smaller boxes' multipoles added into phi.
hipError_t exchange_schedule(fmm2d_ctx *c);
const int32_t *exchange_item_offsets(fmm2d_ctx *c);
hipError_t p2l_all(fmm2d_ctx *c, int p);
hipError_t m2p_all(fmm2d_ctx *c, int p, double *phi);
// list segments for the M2L and near-field kernels (sched.hip)
hipError_t build_schedules(fmm2d_ctx *c);
hipError_t ensure_near_full_schedule(fmm2d_ctx *c);
// Leaves of 17 to 64 points: the FP32 near field takes each leaf pair once
// (a leaf pair's 256 to 4096 point pairs then outweigh the per-record cost of
// the transposed positions); smaller leaves take every ordered pair.
inline bool pair_once_leaves(int64_t maxleaf) { return maxleaf > 16 && maxleaf <= 64; }

}  // namespace fmm2d
