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
// level; the near-field tables cover the finest strong lists, whole or from
// each leaf's own entry on.
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

// The finest strong lists split at each leaf's own entry (the lists are
// ascending): entries from it on (c >= b) and entries before it (c < b),
// each cut into segments; both tables in the same launches.
__global__ void k_seg_count_updown(const int32_t *__restrict__ ptr, const int32_t *__restrict__ self, int64_t nb,
                                   int seg, int32_t *__restrict__ cnt_up, int32_t *__restrict__ cnt_lo) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    cnt_up[b] = (ptr[b + 1] - self[b] + seg - 1) / seg;
    cnt_lo[b] = (self[b] - ptr[b] + seg - 1) / seg;
}

__global__ void k_seg_fill_updown(const int32_t *__restrict__ ptr, const int32_t *__restrict__ self, int64_t nb,
                                  int seg, const int32_t *__restrict__ off_up, const int32_t *__restrict__ off_lo,
                                  int2 *__restrict__ tab_up, int2 *__restrict__ tab_lo) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t p0 = ptr[b], p1 = ptr[b + 1], sb = self[b];
    int32_t k = off_up[b];
    for (int32_t t = sb; t < p1; t += seg) tab_up[k++] = make_int2((int32_t)b, t);
    k = off_lo[b];
    for (int32_t t = p0; t < sb; t += seg) tab_lo[k++] = make_int2((int32_t)b, t);
}

hipError_t segment_updown(fmm2d_ctx *c, const int32_t *ptr, const int32_t *self, int64_t nb, int64_t entries,
                          int seg, Schedule &up, Schedule &lo) {
    up.bound = entries / seg + nb;
    lo.bound = entries / seg + nb;
    FMM2D_TRY(c->scr.segcnt.ensure(sizeof(int32_t) * 2 * nb));
    for (Schedule *s : {&up, &lo}) {
        FMM2D_TRY(s->segoff.ensure(sizeof(int32_t) * (nb + 1)));
        FMM2D_TRY(s->table.ensure(sizeof(int2) * (s->bound > 0 ? s->bound : 1)));
    }
    int32_t *cu = c->scr.segcnt.as<int32_t>(), *cl = cu + nb;
    hipLaunchKernelGGL(k_seg_count_updown, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, ptr, self, nb, seg, cu,
                       cl);
    FMM2D_TRY(hipGetLastError());
    {
        const int32_t *ins[2] = {cu, cl};
        int32_t *outs[2] = {up.segoff.as<int32_t>(), lo.segoff.as<int32_t>()};
        FMM2D_TRY(scan_exclusive_n(c, 2, ins, nb, outs));
    }
    hipLaunchKernelGGL(k_seg_fill_updown, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, ptr, self, nb, seg,
                       up.segoff.as<int32_t>(), lo.segoff.as<int32_t>(), up.table.as<int2>(), lo.table.as<int2>());
    return hipGetLastError();
}

// For every finest strong entry u (row c, entry b) with b < c: the position
// t of c in S_L(b), and transU[t] = u, so that the near field can write the
// source-side sums of record t (target leaf b, source leaf c) where leaf c's
// reduction reads them in order.  The lists are symmetric (the criterion is)
// and ascending; c is located by eight evenly spaced samples of S_L(b) (one
// round of independent loads), then bisection of the interval between two.
__global__ void k_near_trans(const int32_t *__restrict__ sptr, const int32_t *__restrict__ sidx,
                             const int32_t *__restrict__ owner, int64_t ns, int32_t *__restrict__ transU) {
    const int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ns) return;
    const int32_t c = owner[u], b = sidx[u];
    if (b >= c) return;
    const int32_t lo = sptr[b], n = sptr[b + 1] - lo;
    const int32_t step = (n + 7) / 8;
    // number of samples sidx[lo + k step] (k < 8, inside the row) below c
    int32_t below = 0;
#pragma unroll
    for (int k = 1; k < 8; ++k) {
        const int32_t i = k * step;
        below += (i < n && sidx[lo + i] < c) ? 1 : 0;
    }
    // entries before i0 = below * step are all below c (the sample at i0 is,
    // when below > 0) and entries from i0 + step on are not: bisect
    // [i0, i0 + step) for the first entry not below c
    int32_t a0 = below * step, a1 = a0 + step < n ? a0 + step : n;
    while (a0 < a1) {
        const int32_t mid = a0 + ((a1 - a0) >> 1);
        if (sidx[lo + mid] < c) a0 = mid + 1;
        else a1 = mid;
    }
    const int32_t pos = a0;
    if (pos < n && sidx[lo + pos] == c) transU[lo + pos] = (int32_t)u;  // always found: the lists are symmetric
}

}  // namespace

hipError_t build_schedules(fmm2d_ctx *c) {
    TreeState &t = c->tree;
    const int L = t.L;
    FMM2D_TRY(exchange_schedule(c));  // P2L work items of the exchanged-roles lists (structural option)
    const int64_t nbox = level_offset(L + 1);
    const int64_t nleaf = int64_t(1) << (2 * L);
    // all levels' weak lists (rows of levels >= 1)
    const int64_t nw = t.w_off[L + 1] - t.w_off[1];
    FMM2D_TRY(segment_rows(c, t.wptr.as<int32_t>(), nbox, 1, nw, M2L_SEG, t.m2l_all));
    const int64_t ns = t.s_off[L + 1] - t.s_off[L];
    const int32_t *sptrL = t.sptr.as<int32_t>() + ptr_offset(L);
    t.near_seg_ready = false;
    const int64_t maxleaf = (t.n + nleaf - 1) >> (2 * L);
    if (!pair_once_leaves(maxleaf)) return ensure_near_full_schedule(c);  // every ordered pair
    // finest strong lists from each leaf's own entry on (and before it), and
    // the transposed positions, for the near field that takes each leaf pair
    // once; the full-list schedule (binary64 mode) is built when first needed
    FMM2D_TRY(segment_updown(c, sptrL, t.selfpos.as<int32_t>(), nleaf, ns, NEAR_SEG, t.near_up, t.near_lo));
    // the transposed positions only read the lists: on the side stream, so
    // that their (latency-bound) search overlaps the upward pass and M2L; the
    // near field waits for it
    FMM2D_TRY(t.trans.ensure(sizeof(int32_t) * (ns > 0 ? ns : 1)));  // transU
    FMM2D_TRY(side_begin(c));
    hipLaunchKernelGGL(k_near_trans, dim3(grid_for(ns, 256)), dim3(256), 0, c->side, sptrL,
                       t.sidx.as<int32_t>() + t.s_off[L], (L & 1) ? t.owner1.as<int32_t>() : t.owner0.as<int32_t>(),
                       ns, t.trans.as<int32_t>());
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(side_end(c));
    return hipSuccess;
}

hipError_t ensure_near_full_schedule(fmm2d_ctx *c) {
    TreeState &t = c->tree;
    if (t.near_seg_ready) return hipSuccess;
    const int L = t.L;
    FMM2D_TRY(segment_level(c, t.sptr.as<int32_t>() + ptr_offset(L), int64_t(1) << (2 * L),
                            t.s_off[L + 1] - t.s_off[L], NEAR_SEG, t.near_seg));
    t.near_seg_ready = true;
    return hipSuccess;
}

hipError_t side_begin(fmm2d_ctx *c) {
    if (!c->side) {
        FMM2D_TRY(hipStreamCreateWithFlags(&c->side, hipStreamNonBlocking));
        FMM2D_TRY(hipEventCreateWithFlags(&c->ev_side_in, hipEventDisableTiming));
        FMM2D_TRY(hipEventCreateWithFlags(&c->ev_side_out, hipEventDisableTiming));
    }
    FMM2D_TRY(hipEventRecord(c->ev_side_in, c->stream));
    return hipStreamWaitEvent(c->side, c->ev_side_in, 0);
}

hipError_t side_end(fmm2d_ctx *c) {
    FMM2D_TRY(hipEventRecord(c->ev_side_out, c->side));
    c->side_pending = true;
    return hipSuccess;
}

hipError_t side_join(fmm2d_ctx *c) {
    if (!c->side_pending) return hipSuccess;
    return hipStreamWaitEvent(c->stream, c->ev_side_out, 0);
}

}  // namespace fmm2d
