// Work schedules for the two list-driven kernels.
//
// Interaction lists of clustered point sets are heavy-tailed (a few boxes
// couple to thousands of others).  If one wavefront walked a whole list, the
// longest list would set the kernel's duration.  Each list is therefore cut
// into segments of at most SEG entries; a wavefront handles one segment and
// writes partial sums, which a later kernel adds per box (or per point) in
// segment order, so results do not depend on scheduling.  The tables depend
// only on the lists and are built once, after connectivity.
//
// The M2L table covers the weak lists of all levels at once (rows are the
// global box ids, level after level), so that one launch converts every
// level; the near-field table covers the finest strong lists.
#include "evaluate.h"

namespace fmm2d {
namespace {

// segments per row; rows are global box ids [0, nbox) with level-relative
// CSR row pointers at ptr_offset(level) (rows of level 0 have none)
__global__ void k_seg_count(const int32_t *__restrict__ ptr_all, int64_t nbox, int first_level, int seg,
                            int32_t *__restrict__ cnt) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbox) return;
    const int l = level_of(g);
    if (l < first_level) {
        cnt[g] = 0;
        return;
    }
    const int32_t *ptr = ptr_all + ptr_offset(l);
    const int64_t b = g - level_offset(l);
    cnt[g] = (ptr[b + 1] - ptr[b] + seg - 1) / seg;
}

__global__ void k_seg_fill(const int32_t *__restrict__ ptr_all, int64_t nbox, int first_level, int seg,
                           const int32_t *__restrict__ segoff, int2 *__restrict__ table) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbox) return;
    const int l = level_of(g);
    if (l < first_level) return;
    const int32_t *ptr = ptr_all + ptr_offset(l);
    const int64_t b = g - level_offset(l);
    const int32_t p0 = ptr[b], p1 = ptr[b + 1];
    int32_t k = segoff[g];
    for (int32_t t = p0; t < p1; t += seg) table[k++] = make_int2((int32_t)g, t);
}

// Segments of the rows [level_offset(first_level), nbox) of a level-wise CSR
// list: table[i] = (global row, first level-relative entry), segoff[nbox + 1]
// (row -> first segment; segoff[nbox] is the count).  The host only needs an
// upper bound (entries / seg + rows) to size the table and the launch grids,
// so no synchronisation is needed.
hipError_t segment_rows(fmm2d_ctx *c, const int32_t *ptr_all, int64_t nbox, int first_level, int64_t entries,
                        int seg, Schedule &s) {
    s.bound = entries / seg + (nbox - level_offset(first_level));
    FMM2D_TRY(c->scr.segcnt.ensure(sizeof(int32_t) * nbox));
    FMM2D_TRY(s.segoff.ensure(sizeof(int32_t) * (nbox + 1)));
    FMM2D_TRY(s.table.ensure(sizeof(int2) * (s.bound > 0 ? s.bound : 1)));
    hipLaunchKernelGGL(k_seg_count, dim3(grid_for(nbox, 256)), dim3(256), 0, c->stream, ptr_all, nbox, first_level,
                       seg, c->scr.segcnt.as<int32_t>());
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(scan_exclusive(c, c->scr.segcnt.as<int32_t>(), nbox, s.segoff.as<int32_t>()));
    hipLaunchKernelGGL(k_seg_fill, dim3(grid_for(nbox, 256)), dim3(256), 0, c->stream, ptr_all, nbox, first_level,
                       seg, s.segoff.as<int32_t>(), s.table.as<int2>());
    return hipGetLastError();
}

__global__ void k_seg_count_level(const int32_t *__restrict__ ptr, int64_t nb, int seg, int32_t *__restrict__ cnt) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b < nb) cnt[b] = (ptr[b + 1] - ptr[b] + seg - 1) / seg;
}

__global__ void k_seg_fill_level(const int32_t *__restrict__ ptr, int64_t nb, int seg,
                                 const int32_t *__restrict__ segoff, int2 *__restrict__ table) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t p0 = ptr[b], p1 = ptr[b + 1];
    int32_t k = segoff[b];
    for (int32_t t = p0; t < p1; t += seg) table[k++] = make_int2((int32_t)b, t);
}

// The same for one level's CSR list (nb rows, level-relative rows).
hipError_t segment_level(fmm2d_ctx *c, const int32_t *ptr, int64_t nb, int64_t entries, int seg, Schedule &s) {
    s.bound = entries / seg + nb;
    FMM2D_TRY(c->scr.segcnt.ensure(sizeof(int32_t) * nb));
    FMM2D_TRY(s.segoff.ensure(sizeof(int32_t) * (nb + 1)));
    FMM2D_TRY(s.table.ensure(sizeof(int2) * (s.bound > 0 ? s.bound : 1)));
    hipLaunchKernelGGL(k_seg_count_level, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, ptr, nb, seg,
                       c->scr.segcnt.as<int32_t>());
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(scan_exclusive(c, c->scr.segcnt.as<int32_t>(), nb, s.segoff.as<int32_t>()));
    hipLaunchKernelGGL(k_seg_fill_level, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, ptr, nb, seg,
                       s.segoff.as<int32_t>(), s.table.as<int2>());
    return hipGetLastError();
}

}  // namespace

hipError_t build_schedules(fmm2d_ctx *c) {
    TreeState &t = c->tree;
    const int L = t.L;
    const int64_t nbox = level_offset(L + 1);
    // all levels' weak lists (rows of levels >= 1)
    const int64_t nw = t.w_off[L + 1] - t.w_off[1];
    FMM2D_TRY(segment_rows(c, t.wptr.as<int32_t>(), nbox, 1, nw, M2L_SEG, t.m2l_all));
    // finest strong lists (leaf-relative rows)
    FMM2D_TRY(segment_level(c, t.sptr.as<int32_t>() + ptr_offset(L), int64_t(1) << (2 * L),
                            t.s_off[L + 1] - t.s_off[L], NEAR_SEG, t.near_seg));
    return hipSuccess;
}

}  // namespace fmm2d
