// Pieces of the evaluation pass shared between the binary64 operators and the
// reduced-precision hot kernels.
#pragma once
#include "devutil.h"
#include "internal.h"

namespace fmm2d {

hipError_t ensure_binomials(fmm2d_ctx *c);
// M2L of level l in a reduced-precision mode (FP32, BF16X3, FP32_ACC64).
hipError_t m2l_reduced_level(fmm2d_ctx *c, int l, int p, int mode);
// L2P plus the near field at the leaves in a reduced-precision mode; writes
// the leaf-ordered potentials to ev.phi_leaf.
hipError_t leaf_reduced(fmm2d_ctx *c, int p, int mode);

}  // namespace fmm2d
