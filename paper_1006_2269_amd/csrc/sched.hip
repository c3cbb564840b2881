// Work schedules for the two list-driven kernels.
//
// Interaction lists of clustered point sets are heavy-tailed (a few boxes
// couple to thousands of others).  If one wavefront walked a whole list, the
// longest list would set the kernel's duration.  Each list is therefore cut
// into segments of at most SEG entries; a wavefront handles one segment and
// writes partial sums, which a second kernel adds per box (or per point) in
// segment order, so results do not depend on scheduling.  The tables depend
// only on the lists and are built once, after connectivity.
#include "evaluate.h"

namespace fmm2d {
namespace {

__global__ void k_seg_count(const int32_t *__restrict__ ptr, int64_t nb, int seg, int32_t *__restrict__ cnt) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) cnt[b] = (ptr[b + 1] - ptr[b] + seg - 1) / seg;
}

__global__ void k_seg_fill(const int32_t *__restrict__ ptr, int64_t nb, int seg, const int32_t *__restrict__ segoff,
                           int2 *__restrict__ table) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t p0 = ptr[b], p1 = ptr[b + 1];
    int32_t k = segoff[b];
    for (int32_t t = p0; t < p1; t += seg) table[k++] = make_int2((int32_t)b, t);
}

// Segments of one CSR list (nb rows, `entries` entries): table[i] = (row,
// first entry), segoff[nb + 1] (row -> first segment; segoff[nb] is the
// count).  The host only needs an upper bound (entries / seg + rows) to size
// the table and the launch grids, so no synchronisation is needed.
hipError_t segment_list(fmm2d_ctx *c, const int32_t *ptr, int64_t nb, int64_t entries, int seg, Schedule &s) {
    s.bound = entries / seg + nb;
    FMM2D_TRY(c->scr.segcnt.ensure(sizeof(int32_t) * nb));
    FMM2D_TRY(s.segoff.ensure(sizeof(int32_t) * (nb + 1)));
    FMM2D_TRY(s.table.ensure(sizeof(int2) * s.bound));
    hipLaunchKernelGGL(k_seg_count, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, ptr, nb, seg,
                       c->scr.segcnt.as<int32_t>());
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(scan_exclusive(c, c->scr.segcnt.as<int32_t>(), nb, s.segoff.as<int32_t>()));
    hipLaunchKernelGGL(k_seg_fill, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, ptr, nb, seg,
                       s.segoff.as<int32_t>(), s.table.as<int2>());
    return hipGetLastError();
}

}  // namespace

hipError_t build_schedules(fmm2d_ctx *c) {
    TreeState &t = c->tree;
    const int L = t.L;
    t.m2l_seg.resize(L + 1);
    for (int l = 1; l <= L; ++l) {
        Schedule &s = t.m2l_seg[l];
        const int64_t nw = t.w_off[l + 1] - t.w_off[l];
        s.bound = 0;
        if (nw == 0) continue;
        FMM2D_TRY(segment_list(c, t.wptr.as<int32_t>() + ptr_offset(l), int64_t(1) << (2 * l), nw, M2L_SEG, s));
    }
    FMM2D_TRY(segment_list(c, t.sptr.as<int32_t>() + ptr_offset(L), int64_t(1) << (2 * L),
                           t.s_off[L + 1] - t.s_off[L], NEAR_SEG, t.near_seg));
    return hipSuccess;
}

}  // namespace fmm2d
