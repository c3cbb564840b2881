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
// children of each of the four children's parents' strong boxes), and each
// becomes one entry of S or W.  After each level a one-thread kernel checks
// the next level's candidate count against the entry limit and the free pool
// space and raises a flag that stops all later levels, so no int32 prefix
// sum can wrap; the host reads the flag with the pool offsets at the end.
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int LW = 4;  // wavefronts (boxes) per block

// pool_state layout: [0, L+2): S pool offsets, [L+2, 2L+4): W pool offsets,
// [2L+4]: overflow flag.
// Criterion 2.1, R + theta r <= theta d, evaluated exactly as written
// (binary64, no contraction, correctly rounded sqrt).  Most candidates are
// decided without the square root: with L = R + theta r and s = d^2 as
// computed, L^2 and theta^2 s differ from L^2 and (theta d)^2 of the exact
// expression by a few units of the last place, so when they differ by more
// than a relative 1e-14 the exact comparison cannot come out differently;
// the narrow band in between, and magnitudes near the underflow range, take
// the exact path.
__device__ inline bool theta_separated(double theta, double theta2, double4 gb, double4 gc) {
#pragma clang fp contract(off)
    const double dx = gb.x - gc.x;
    const double dy = gb.y - gc.y;
    const double dx2 = dx * dx;
    const double dy2 = dy * dy;
    const double s = dx2 + dy2;
    const double R = gb.z > gc.z ? gb.z : gc.z;
    const double r = gb.z > gc.z ? gc.z : gb.z;
    const double lhs = R + theta * r;
    const double L2 = lhs * lhs;
    const double S2 = theta2 * s;
    if (s >= 0x1p-900 && L2 >= 0x1p-900) {
        if (L2 <= S2 * (1.0 - 1e-14)) return true;
        if (L2 >= S2 * (1.0 + 1e-14)) return false;
    }
    const double d = sqrt(s);
    const double rhs = theta * d;
    // balls must be disjoint: two zero-size boxes at one point (d = 0) never are
    return lhs <= rhs && rhs > 0.0;
}

// Level 0: S_0(root) = {root}, W_0(root) empty; for a one-level tree
// (L = 0) also the near-field record of that single strong entry, written
// as the finest fill pass writes the others.
__global__ void k_lists_init(int32_t *sptr0, int32_t *wptr0, int32_t *sidx_pool, int64_t *pool_state, int L,
                             const int32_t *stL, const double4 *geom0, int2 *recj, float4 *recd) {
    sptr0[0] = 0;
    sptr0[1] = 1;
    wptr0[0] = 0;
    wptr0[1] = 0;
    sidx_pool[0] = 0;
    for (int k = 0; k < 2 * L + 5; ++k) pool_state[k] = 0;
    pool_state[1] = 1;  // S offset of level 1
    if (L == 0) {
        const double4 g = geom0[0];
        const float dxc = (float)(g.x - g.x), dyc = (float)(g.y - g.y);
        const float mag = fabsf(dxc) + fabsf(dyc) + (float)g.z + (float)g.z;
        recj[0] = make_int2(stL[0], stL[1]);
        recd[0] = make_float4(dxc, dyc, (mag * 0x1p-20f) * (mag * 0x1p-20f), 0.f);
    }
}

// First word of box b's decision bits: candidates of b are preceded by
// cand(b) = 16 sptr_prev[P] + (b mod 4) 4 |S_{l-1}(P)| candidates of the
// level, and b needs ceil(ncand / 64) words, so floor(cand(b) / 64) + b never
// overlaps the words of box b - 1.
__device__ inline int64_t bits_base(int64_t b, int32_t s0, int32_t s1) {
    const int64_t cand = 16 * (int64_t)s0 + (b & 3) * 4 * (int64_t)(s1 - s0);
    return (cand >> 6) + b;
}

// One wavefront, box b of level l (candidates: the four children of each box
// of S_{l-1}(parent)).  Count pass (FILL = false): the theta test of every
// candidate, the two counts, and (BITS) the decisions stored as bits (set:
// weak).  Fill pass: the same candidates, their decisions (from the bits, or
// the test again), ballot compaction into the lists; on the finest level
// also the near-field record of each strong entry (source leaf's point
// range; FP32 centre offset c_b - c_c and the coincidence threshold
// (2^-20 of the magnitudes)^2 for the FP32 path).
template <bool FILL, bool BITS>
__device__ inline void box_lists(int l, int L, double theta, const double4 *__restrict__ geomL, int64_t b,
                                 const int32_t *__restrict__ sptr_prev, const int32_t *__restrict__ sidx_prev,
                                 uint64_t *__restrict__ bits, int32_t &cs, int32_t &cw, int32_t tS,
                                 int32_t *__restrict__ so, int32_t *__restrict__ wo, const int32_t *__restrict__ stL,
                                 int2 *__restrict__ recj, float4 *__restrict__ recd) {
    // Chunks of 64 candidates are taken CB at a time: the loads of a batch
    // (box numbers, then geometry, leaf ranges or decision words) are all
    // issued before any is waited for, so a box costs a few memory round trips
    // rather than two per chunk.
    constexpr int CB = 4;
    const uint32_t lane = lane_id();
    const int64_t P = b >> 2;
    const int32_t s0 = sptr_prev[P], s1 = sptr_prev[P + 1];
    const int32_t ncand = 4 * (s1 - s0);
    uint64_t *bw = BITS ? bits + bits_base(b, s0, s1) : nullptr;
    const bool records = FILL && l == L && recj != nullptr;
    const bool test = !FILL || !BITS;
    double4 gb = make_double4(0.0, 0.0, 0.0, 0.0);
    if (test || records) gb = geomL[b];
    cs = 0;
    cw = 0;
    for (int32_t base = 0; base < ncand; base += 64 * CB) {
        int32_t cbox[CB];
        bool ok[CB];
        uint64_t mw[CB];
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const int32_t j = base + 64 * u + (int32_t)lane;
            ok[u] = j < ncand;
            cbox[u] = ok[u] ? 4 * sidx_prev[s0 + (j >> 2)] + (j & 3) : 0;
            if (!test) mw[u] = base + 64 * u < ncand ? bw[(base >> 6) + u] : 0;
        }
        if (test) {
            double4 gc[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) gc[u] = ok[u] ? geomL[cbox[u]] : gb;
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                const bool weak = ok[u] && theta_separated(theta, theta * theta, gb, gc[u]);
                mw[u] = __ballot(weak);
                if (BITS && !FILL && lane == 0 && base + 64 * u < ncand) bw[(base >> 6) + u] = mw[u];
            }
        }
        // records of the finest level: geometry and leaf range of the strong entries
        double4 gr[CB];
        int2 rr[CB];
        if (records) {
#pragma unroll
            for (int u = 0; u < CB; ++u) {
                const bool strong = ok[u] && !((mw[u] >> lane) & 1);
                gr[u] = strong ? geomL[cbox[u]] : gb;
                rr[u] = strong ? make_int2(stL[cbox[u]], stL[cbox[u] + 1]) : make_int2(0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < CB; ++u) {
            const uint64_t okm = __ballot(ok[u]);
            const uint64_t ms = okm & ~mw[u];
            if (FILL && ok[u]) {
                if ((mw[u] >> lane) & 1) {
                    wo[cw + (int32_t)popc_below(mw[u])] = cbox[u];
                } else {
                    const int32_t pos = cs + (int32_t)popc_below(ms);
                    so[pos] = cbox[u];
                    if (records) {
                        const int32_t t = tS + pos;
                        const double4 gc = gr[u];
                        const float dxc = (float)(gb.x - gc.x), dyc = (float)(gb.y - gc.y);
                        const float mag = fabsf(dxc) + fabsf(dyc) + (float)gb.z + (float)gc.z;
                        recj[t] = rr[u];
                        recd[t] = make_float4(dxc, dyc, (mag * 0x1p-20f) * (mag * 0x1p-20f), 0.f);
                    }
                }
            }
            cw += (int32_t)__popcll(mw[u]);
            cs += (int32_t)__popcll(ms);
        }
    }
}

// One level, one wavefront per box.  The count pass stores the decisions as
// bits, the fill pass replays them.
template <bool FILL>
__global__ void __launch_bounds__(LW * 64) k_lists_level(int l, int L, double theta, const double4 *__restrict__ geomL,
                                                        const int32_t *__restrict__ sptr_prev,
                                                        const int32_t *__restrict__ sidx_pool,
                                                        const int64_t *__restrict__ pool_state, int64_t nb,
                                                        int32_t *__restrict__ ns, int32_t *__restrict__ nw,
                                                        uint64_t *__restrict__ bits,
                                                        const int32_t *__restrict__ sptr_cur,
                                                        const int32_t *__restrict__ wptr_cur,
                                                        int32_t *__restrict__ sidx_out, int32_t *__restrict__ widx_out,
                                                        const int32_t *__restrict__ stL, int2 *__restrict__ recj,
                                                        float4 *__restrict__ recd) {
    const int64_t b = (int64_t)blockIdx.x * LW + threadIdx.x / 64;
    const uint32_t lane = lane_id();
    if (b >= nb) return;
    const bool overflow = pool_state[2 * L + 4] != 0;
    if (overflow) {
        if (!FILL && lane == 0) { ns[b] = 0; nw[b] = 0; }
        return;
    }
    const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
    int32_t cs, cw;
    if (FILL) {
        box_lists<true, true>(l, L, theta, geomL, b, sptr_prev, sidx_prev, bits, cs, cw, sptr_cur[b],
                              sidx_out + pool_state[l] + sptr_cur[b], widx_out + pool_state[(L + 2) + l] + wptr_cur[b],
                              stL, recj, recd);
    } else {
        box_lists<false, true>(l, L, theta, geomL, b, sptr_prev, sidx_prev, bits, cs, cw, 0, nullptr, nullptr, stL,
                               nullptr, nullptr);
        if (lane == 0) {
            ns[b] = cs;
            nw[b] = cw;
        }
    }
}

// Pool offsets of level l + 1, and the checks that guard the next level:
// flag 1 when a pool is too small (the host retries with larger pools),
// flag 2 when level l + 1's candidates, 16 |S_l| (each becomes one entry of
// S or W), exceed the entry limit.  A flagged level is not examined, so no
// int32 prefix sum can wrap and no decision bit lies beyond the buffer
// (sized for cap_s + cap_w candidates).
__device__ inline void advance_pools(int l, int L, int64_t nb, const int32_t *sptr_cur, const int32_t *wptr_cur,
                                     int64_t *pool_state, int64_t cap_s, int64_t cap_w, int64_t limit) {
    if (pool_state[2 * L + 4]) return;
    const int64_t so = pool_state[l] + sptr_cur[nb];
    const int64_t wo = pool_state[(L + 2) + l] + wptr_cur[nb];
    pool_state[l + 1] = so;
    pool_state[(L + 2) + l + 1] = wo;
    if (so > cap_s || wo > cap_w) {
        pool_state[2 * L + 4] = 1;
        return;
    }
    if (l < L) {
        const int64_t cand = 16 * (int64_t)sptr_cur[nb];
        if (cand > limit) pool_state[2 * L + 4] = 2;
        else if (cand > (cap_s - so) + (cap_w - wo)) pool_state[2 * L + 4] = 1;
    }
}

__global__ void k_lists_advance(int l, int L, int64_t nb, const int32_t *sptr_cur, const int32_t *wptr_cur,
                                int64_t *pool_state, int64_t cap_s, int64_t cap_w, int64_t limit) {
    advance_pools(l, L, nb, sptr_cur, wptr_cur, pool_state, cap_s, cap_w, limit);
}

// Levels 1..K (4^K <= SMALL_BOXES boxes each) in one workgroup, which saves
// the launches of the coarse levels: the geometry of levels 0..K staged in
// LDS, and per level a count pass over the boxes (one wavefront per box), the
// two row-pointer scans in LDS, the pool offsets and checks, and a fill pass
// that tests the candidates again (cheaper here than storing the decisions).
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_BOXES = 64;
constexpr int SMALL_GEOM = 85;  // boxes of levels 0..3
__global__ void __launch_bounds__(SMALL_THREADS) k_lists_small(int K, int L, double theta,
                                                              const double4 *__restrict__ geom,
                                                              int32_t *__restrict__ sptr, int32_t *__restrict__ wptr,
                                                              int32_t *__restrict__ sidx_pool,
                                                              int32_t *__restrict__ widx_pool,
                                                              int64_t *__restrict__ pool_state, int64_t cap_s,
                                                              int64_t cap_w, int64_t limit,
                                                              const int32_t *__restrict__ stL, int2 *__restrict__ recj,
                                                              float4 *__restrict__ recd) {
    __shared__ int32_t ns[SMALL_BOXES], nw[SMALL_BOXES];
    __shared__ int32_t tmp[SMALL_THREADS / 64];
    __shared__ int flag;
    __shared__ double4 g_s[SMALL_GEOM];
    const int t = threadIdx.x, wv = t / 64;
    constexpr int NWV = SMALL_THREADS / 64;
    if (t < level_offset(K + 1)) g_s[t] = geom[t];
    for (int l = 1; l <= K; ++l) {
        if (t == 0) flag = (int)pool_state[2 * L + 4];
        __syncthreads();
        if (flag) return;  // uniform: every thread read the same flag
        const int64_t nb = int64_t(1) << (2 * l);
        const double4 *gL = g_s + level_offset(l);
        const int32_t *sp_prev = sptr + ptr_offset(l - 1);
        int32_t *sp_cur = sptr + ptr_offset(l), *wp_cur = wptr + ptr_offset(l);
        const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
        for (int64_t b = wv; b < nb; b += NWV) {
            int32_t cs, cw;
            box_lists<false, false>(l, L, theta, gL, b, sp_prev, sidx_prev, nullptr, cs, cw, 0, nullptr, nullptr,
                                    stL, nullptr, nullptr);
            if (lane_id() == 0) {
                ns[b] = cs;
                nw[b] = cw;
            }
        }
        __syncthreads();
        int32_t tot_s, tot_w;
        const int32_t vs = t < nb ? ns[t] : 0, vw = t < nb ? nw[t] : 0;
        const int32_t es = block_excl_scan<SMALL_THREADS>(vs, tmp, tot_s);
        const int32_t ew = block_excl_scan<SMALL_THREADS>(vw, tmp, tot_w);
        if (t < nb) {
            sp_cur[t] = es;
            wp_cur[t] = ew;
        }
        if (t == 0) {
            sp_cur[nb] = tot_s;
            wp_cur[nb] = tot_w;
        }
        __threadfence_block();
        __syncthreads();
        if (t == 0) {
            advance_pools(l, L, nb, sp_cur, wp_cur, pool_state, cap_s, cap_w, limit);
            flag = (int)pool_state[2 * L + 4];
        }
        __syncthreads();
        // a flagged level is not filled (the host discards or retries the lists)
        if (flag) return;
        const int64_t so0 = pool_state[l], wo0 = pool_state[(L + 2) + l];
        for (int64_t b = wv; b < nb; b += NWV) {
            int32_t cs, cw;
            box_lists<true, false>(l, L, theta, gL, b, sp_prev, sidx_prev, nullptr, cs, cw, sp_cur[b],
                                   sidx_pool + so0 + sp_cur[b], widx_pool + wo0 + wp_cur[b], stL, recj, recd);
        }
        __syncthreads();
    }
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
    const double4 *geom = t.geom.as<double4>();
    // Level 1 has 16 candidates (the root's children, four per box); later
    // levels are guarded on the device by k_lists_advance, so the host never
    // waits inside the level loop.
    if (L >= 1 && 16 > limit) {
        *overflow = 2;
        return hipSuccess;
    }
    FMM2D_TRY(t.bits.ensure(sizeof(uint64_t) * (size_t)((cap_s + cap_w) / 64 + maxnb + 2)));
    uint64_t *bits = t.bits.as<uint64_t>();
    // near-field records of the finest level's strong entries (<= cap_s)
    FMM2D_TRY(t.nrec_j.ensure(sizeof(int2) * cap_s));
    FMM2D_TRY(t.nrec_d.ensure(sizeof(float4) * cap_s));
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    hipLaunchKernelGGL(k_lists_init, dim3(1), dim3(1), 0, c->stream, sptr, wptr, t.sidx.as<int32_t>(), ps, L, stL,
                       geom, t.nrec_j.as<int2>(), t.nrec_d.as<float4>());
    // levels of at most 1024 boxes: one workgroup, one launch
    int K = 0;
    while (K < L && (int64_t(1) << (2 * (K + 1))) <= SMALL_BOXES) ++K;
    if (K >= 1)
        hipLaunchKernelGGL(k_lists_small, dim3(1), dim3(SMALL_THREADS), 0, c->stream, K, L, theta, geom, sptr, wptr,
                           t.sidx.as<int32_t>(), t.widx.as<int32_t>(), ps, cap_s, cap_w, limit, stL,
                           t.nrec_j.as<int2>(), t.nrec_d.as<float4>());
    for (int l = K + 1; l <= L; ++l) {
        const int64_t nb = int64_t(1) << (2 * l);
        int32_t *sp_prev = sptr + ptr_offset(l - 1), *sp_cur = sptr + ptr_offset(l), *wp_cur = wptr + ptr_offset(l);
        const double4 *gL = geom + level_offset(l);
        const unsigned grid = grid_for(nb, LW);
        hipLaunchKernelGGL(k_lists_level<false>, dim3(grid), dim3(LW * 64), 0, c->stream, l, L, theta, gL, sp_prev,
                           t.sidx.as<int32_t>(), ps, nb, t.cnt_s.as<int32_t>(), t.cnt_w.as<int32_t>(), bits, sp_cur, wp_cur,
                           t.sidx.as<int32_t>(), t.widx.as<int32_t>(), stL, nullptr, nullptr);
        {
            const int32_t *ins[2] = {t.cnt_s.as<int32_t>(), t.cnt_w.as<int32_t>()};
            int32_t *outs[2] = {sp_cur, wp_cur};
            FMM2D_TRY(scan_exclusive_n(c, 2, ins, nb, outs));
        }
        hipLaunchKernelGGL(k_lists_advance, dim3(1), dim3(1), 0, c->stream, l, L, nb, sp_cur, wp_cur, ps, cap_s,
                           cap_w, limit);
        hipLaunchKernelGGL(k_lists_level<true>, dim3(grid), dim3(LW * 64), 0, c->stream, l, L, theta, gL, sp_prev,
                           t.sidx.as<int32_t>(), ps, nb, t.cnt_s.as<int32_t>(), t.cnt_w.as<int32_t>(), bits, sp_cur, wp_cur,
                           t.sidx.as<int32_t>(), t.widx.as<int32_t>(), stL, t.nrec_j.as<int2>(), t.nrec_d.as<float4>());
        FMM2D_TRY(hipGetLastError());
    }
    std::vector<int64_t> h(2 * L + 5);
    FMM2D_TRY(hipMemcpyAsync(h.data(), ps, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    *overflow = (int)h[2 * L + 4];
    t.s_off.assign(h.begin(), h.begin() + (L + 2));
    t.w_off.assign(h.begin() + (L + 2), h.begin() + (2 * L + 4));
    return hipSuccess;
}

}  // namespace fmm2d
