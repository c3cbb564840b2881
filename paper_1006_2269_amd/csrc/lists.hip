// Strong / weak connectivity of every level (Section 4) under the
// theta-criterion (Criterion 2.1).
//
// For box b at level l with parent P, the candidates are the four children of
// every box in S_{l-1}(P); they are visited in ascending order by the 64
// lanes of one wavefront, tested, and compacted with ballots into S_l(b)
// (criterion false) or W_l(b) (criterion true), so both lists come out
// ascending.  Each level is a count pass, an exclusive scan of the counts
// (the CSR row pointers) and a fill pass.  The index lists of all levels live
// in two pools; the pool offset of each level is advanced on the device, and
// the host reads the offsets (and an overflow flag) at the end.
//
// Row pointers are int32.  A level's candidates number 16 |S_{l-1}| (four
// children of each of the four children's parents' strong boxes).  The host
// carries an upper bound of |S_{l-1}| (16^(l-1) until a level's exact total
// has been read) and reads the exact total back only when 16 times the bound
// exceeds the entry limit; it refuses a level whose candidate count could
// exceed the limit before launching it, so no int32 prefix sum can wrap.
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int LW = 4;  // wavefronts (boxes) per block

// pool_state layout: [0, L+2): S pool offsets, [L+2, 2L+4): W pool offsets,
// [2L+4]: overflow flag.
__device__ inline bool theta_separated(double theta, double4 gb, double4 gc) {
#pragma clang fp contract(off)
    const double dx = gb.x - gc.x;
    const double dy = gb.y - gc.y;
    const double dx2 = dx * dx;
    const double dy2 = dy * dy;
    const double d = sqrt(dx2 + dy2);
    const double R = gb.z > gc.z ? gb.z : gc.z;
    const double r = gb.z > gc.z ? gc.z : gb.z;
    const double lhs = R + theta * r;
    const double rhs = theta * d;
    // balls must be disjoint: two zero-size boxes at one point (d = 0) never are
    return lhs <= rhs && rhs > 0.0;
}

__global__ void k_lists_init(int32_t *sptr0, int32_t *wptr0, int32_t *sidx_pool, int64_t *pool_state, int L) {
    sptr0[0] = 0;
    sptr0[1] = 1;
    wptr0[0] = 0;
    wptr0[1] = 0;
    sidx_pool[0] = 0;
    for (int k = 0; k < 2 * L + 5; ++k) pool_state[k] = 0;
    pool_state[1] = 1;  // S offset of level 1
}

// First word of box b's decision bits: candidates of b are preceded by
// cand(b) = 16 sptr_prev[P] + (b mod 4) 4 |S_{l-1}(P)| candidates of the
// level, and b needs ceil(ncand / 64) words, so floor(cand(b) / 64) + b never
// overlaps the words of box b - 1.
__device__ inline int64_t bits_base(int64_t b, int32_t s0, int32_t s1) {
    const int64_t cand = 16 * (int64_t)s0 + (b & 3) * 4 * (int64_t)(s1 - s0);
    return (cand >> 6) + b;
}

// Count pass (FILL = false): one wavefront per box tests its candidates,
// stores the decisions (bit set: weak) and the two counts.  Fill pass: the
// same candidates, the stored decisions, ballot compaction into the lists.
template <bool FILL>
__global__ void __launch_bounds__(LW * 64) k_lists_level(int l, int L, double theta, const double4 *__restrict__ geomL,
                                                        const int32_t *__restrict__ sptr_prev,
                                                        const int32_t *__restrict__ sidx_pool,
                                                        const int64_t *__restrict__ pool_state, int64_t nb,
                                                        int32_t *__restrict__ ns, int32_t *__restrict__ nw,
                                                        uint64_t *__restrict__ bits,
                                                        const int32_t *__restrict__ sptr_cur,
                                                        const int32_t *__restrict__ wptr_cur,
                                                        int32_t *__restrict__ sidx_out, int32_t *__restrict__ widx_out) {
    const int64_t b = (int64_t)blockIdx.x * LW + threadIdx.x / 64;
    const uint32_t lane = lane_id();
    if (b >= nb) return;
    const bool overflow = pool_state[2 * L + 4] != 0;
    if (overflow) {
        if (!FILL && lane == 0) { ns[b] = 0; nw[b] = 0; }
        return;
    }
    const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
    const int64_t P = b >> 2;
    const int32_t s0 = sptr_prev[P], s1 = sptr_prev[P + 1];
    const int32_t ncand = 4 * (s1 - s0);
    uint64_t *bw = bits + bits_base(b, s0, s1);
    double4 gb;
    if (!FILL) gb = geomL[b];
    int32_t cs = 0, cw = 0;
    int32_t *so = nullptr, *wo = nullptr;
    if (FILL) {
        so = sidx_out + pool_state[l] + sptr_cur[b];
        wo = widx_out + pool_state[(L + 2) + l] + wptr_cur[b];
    }
    for (int32_t base = 0; base < ncand; base += 64) {
        const int32_t j = base + (int32_t)lane;
        const bool ok = j < ncand;
        int32_t cbox = 0;
        uint64_t mw;
        if (FILL) {
            mw = bw[base >> 6];
            if (ok) cbox = 4 * sidx_prev[s0 + (j >> 2)] + (j & 3);
        } else {
            bool weak = false;
            if (ok) {
                cbox = 4 * sidx_prev[s0 + (j >> 2)] + (j & 3);
                weak = theta_separated(theta, gb, geomL[cbox]);
            }
            mw = __ballot(ok && weak);
            if (lane == 0) bw[base >> 6] = mw;
        }
        const uint64_t okm = __ballot(ok);
        const uint64_t ms = okm & ~mw;
        if (FILL && ok) {
            if ((mw >> lane) & 1) wo[cw + (int32_t)popc_below(mw)] = cbox;
            else so[cs + (int32_t)popc_below(ms)] = cbox;
        }
        cw += (int32_t)__popcll(mw);
        cs += (int32_t)__popcll(ms);
    }
    if (!FILL && lane == 0) {
        ns[b] = cs;
        nw[b] = cw;
    }
}

__global__ void k_lists_advance(int l, int L, int64_t nb, const int32_t *sptr_cur, const int32_t *wptr_cur,
                                int64_t *pool_state, int64_t cap_s, int64_t cap_w) {
    if (pool_state[2 * L + 4]) return;
    const int64_t so = pool_state[l] + sptr_cur[nb];
    const int64_t wo = pool_state[(L + 2) + l] + wptr_cur[nb];
    pool_state[l + 1] = so;
    pool_state[(L + 2) + l + 1] = wo;
    if (so > cap_s || wo > cap_w) pool_state[2 * L + 4] = 1;
}

}  // namespace

hipError_t build_lists_device(fmm2d_ctx *c, double theta, int64_t cap_s, int64_t cap_w, int64_t limit,
                              int *overflow) {
    TreeState &t = c->tree;
    const int L = t.L;
    const int64_t nptr = ptr_offset(L + 1);
    const int64_t maxnb = int64_t(1) << (2 * L);
    FMM2D_TRY(t.sptr.ensure(sizeof(int32_t) * nptr));
    FMM2D_TRY(t.wptr.ensure(sizeof(int32_t) * nptr));
    FMM2D_TRY(t.sidx.ensure(sizeof(int32_t) * cap_s));
    FMM2D_TRY(t.widx.ensure(sizeof(int32_t) * cap_w));
    FMM2D_TRY(t.cnt_s.ensure(sizeof(int32_t) * maxnb));
    FMM2D_TRY(t.cnt_w.ensure(sizeof(int32_t) * maxnb));
    FMM2D_TRY(t.pool_state.ensure(sizeof(int64_t) * (2 * L + 5)));
    int32_t *sptr = t.sptr.as<int32_t>(), *wptr = t.wptr.as<int32_t>();
    int64_t *ps = t.pool_state.as<int64_t>();
    hipLaunchKernelGGL(k_lists_init, dim3(1), dim3(1), 0, c->stream, sptr, wptr, t.sidx.as<int32_t>(), ps, L);
    const double4 *geom = t.geom.as<double4>();
    // Upper bound of the entries of S at level l-1 (exact at level 0: the
    // root).  |S_l| <= 16 |S_{l-1}|, so the bound grows by 16 per level; only
    // when it reaches the limit is the exact total read back (one copy and a
    // synchronisation).
    int64_t s_prev = 1;
    for (int l = 1; l <= L; ++l) {
        const int64_t nb = int64_t(1) << (2 * l);
        int32_t *sp_prev = sptr + ptr_offset(l - 1), *sp_cur = sptr + ptr_offset(l), *wp_cur = wptr + ptr_offset(l);
        if (16 * s_prev > limit) {
            int32_t tot = 0;
            FMM2D_TRY(hipMemcpyAsync(&tot, sp_prev + (nb >> 2), sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
            FMM2D_TRY(hipStreamSynchronize(c->stream));
            s_prev = tot;
            if (16 * s_prev > limit) {
                *overflow = 2;
                return hipSuccess;
            }
        }
        const double4 *gL = geom + level_offset(l);
        const unsigned grid = grid_for(nb, LW);
        // decision words: at most 16 s_prev candidates / 64 + one spare per box
        FMM2D_TRY(t.bits.ensure(sizeof(uint64_t) * (size_t)((16 * s_prev) / 64 + nb + 1)));
        uint64_t *bits = t.bits.as<uint64_t>();
        hipLaunchKernelGGL(k_lists_level<false>, dim3(grid), dim3(LW * 64), 0, c->stream, l, L, theta, gL, sp_prev,
                           t.sidx.as<int32_t>(), ps, nb, t.cnt_s.as<int32_t>(), t.cnt_w.as<int32_t>(), bits, sp_cur, wp_cur,
                           t.sidx.as<int32_t>(), t.widx.as<int32_t>());
        {
            const int32_t *ins[2] = {t.cnt_s.as<int32_t>(), t.cnt_w.as<int32_t>()};
            int32_t *outs[2] = {sp_cur, wp_cur};
            FMM2D_TRY(scan_exclusive_n(c, 2, ins, nb, outs));
        }
        s_prev *= 16;
        hipLaunchKernelGGL(k_lists_advance, dim3(1), dim3(1), 0, c->stream, l, L, nb, sp_cur, wp_cur, ps, cap_s,
                           cap_w);
        hipLaunchKernelGGL(k_lists_level<true>, dim3(grid), dim3(LW * 64), 0, c->stream, l, L, theta, gL, sp_prev,
                           t.sidx.as<int32_t>(), ps, nb, t.cnt_s.as<int32_t>(), t.cnt_w.as<int32_t>(), bits, sp_cur, wp_cur,
                           t.sidx.as<int32_t>(), t.widx.as<int32_t>());
        FMM2D_TRY(hipGetLastError());
    }
    std::vector<int64_t> h(2 * L + 5);
    FMM2D_TRY(hipMemcpyAsync(h.data(), ps, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    *overflow = h[2 * L + 4] != 0 ? 1 : 0;
    t.s_off.assign(h.begin(), h.begin() + (L + 2));
    t.w_off.assign(h.begin() + (L + 2), h.begin() + (2 * L + 4));
    return hipSuccess;
}

}  // namespace fmm2d
