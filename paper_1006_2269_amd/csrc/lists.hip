// Strong / weak connectivity of every level (Section 4) under the
// theta-criterion (Criterion 2.1).
//
// For box b at level l with parent P, the candidates are the four children of
// every box in S_{l-1}(P), in ascending order; each is tested and goes to
// S_l(b) (criterion false) or W_l(b) (criterion true), so both lists come out
// ascending.  The index lists of all levels live in two pools; the pool
// offset of each level is advanced on the device, and the host reads the
// offsets (and an overflow flag) at the end.
//
// Levels of at most 64 boxes run in one workgroup (one launch).  Finer levels
// are flat passes over the level's candidate space: candidate q of parent P
// is q = 16 sptr_{l-1}[P] + 4 |S_{l-1}(P)| c + j for child box b = 4P + c and
// its j-th candidate, so the candidates of consecutive boxes are consecutive
// and, with the owner of every entry of S_{l-1} (its row), q decodes in a few
// loads.  A count pass writes the decisions as one bit per candidate and the
// per-word counts; a scan over the words gives, for every candidate, the
// number of strong and weak candidates before it, which is its position in
// the level's S or W pool and, at a box's first candidate, the box's row
// pointer.  The work per wavefront is the same for every word, so boxes with
// very long lists (clustered inputs) do not serialise a pass.
//
// Row pointers are int32.  A level's candidates number 16 |S_{l-1}|, and each
// becomes one entry of S or W.  After each level a check compares the next
// level's candidate count with the entry limit and the free pool space and
// raises a flag that stops all later levels, so no int32 prefix sum can wrap;
// the host reads the flag with the pool offsets at the end.
#include <algorithm>

#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {


// pool_state layout: [0, L+2): S pool offsets, [L+2, 2L+4): W pool offsets,
// [2L+4, 3L+6): X pool offsets (exchanged roles), [3L+6]: overflow flag.
__host__ __device__ inline int slot_x(int L, int l) { return 2 * (L + 2) + l; }
__host__ __device__ inline int slot_flag(int L) { return 3 * (L + 2); }

// Structural options (Section 4): interaction via the parent, and exchanged
// roles at the finest level or at every level.
__host__ __device__ inline bool opt_parent(int opt) { return (opt & FMM2D_OPT_PARENT) != 0; }
__host__ __device__ inline bool opt_swap(int opt, int l, int L) {
    return (opt & FMM2D_OPT_SWAP_ALL) != 0 || ((opt & FMM2D_OPT_SWAP_FINEST) != 0 && l == L);
}
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

// The criterion with the radii's roles exchanged, r + theta R <= theta d, on
// disjoint balls (d > R + r), evaluated as written (binary64, no
// contraction, correctly rounded sqrt); the same guarded shortcut as above.
__device__ inline bool exchange_separated(double theta, double theta2, double4 gb, double4 gc) {
#pragma clang fp contract(off)
    const double dx = gb.x - gc.x;
    const double dy = gb.y - gc.y;
    const double dx2 = dx * dx;
    const double dy2 = dy * dy;
    const double s = dx2 + dy2;
    const double R = gb.z > gc.z ? gb.z : gc.z;
    const double r = gb.z > gc.z ? gc.z : gb.z;
    const double lhs = r + theta * R;
    const double sum = R + r;
    const double L2 = lhs * lhs, S2 = theta2 * s, Q2 = sum * sum;
    if (s >= 0x1p-900 && L2 >= 0x1p-900 && Q2 >= 0x1p-900) {
        const bool a_true = L2 <= S2 * (1.0 - 1e-14), a_false = L2 >= S2 * (1.0 + 1e-14);
        const bool b_true = s >= Q2 * (1.0 + 1e-14), b_false = s <= Q2 * (1.0 - 1e-14);
        if (a_false || b_false) return false;
        if (a_true && b_true) return true;
    }
    const double d = sqrt(s);
    const double rhs = theta * d;
    return lhs <= rhs && d > sum;
}

// A weak-list entry that is a box of the level above (interaction via the
// parent) carries this bit on its level-local index.
constexpr int32_t VFLAG = FMM2D_VFLAG;

// The four-lane groups of a word (the four children of one box of the level
// above) whose lanes are all set in m, marked at the group's first lane.
__device__ inline uint64_t full_groups(uint64_t m) {
    return m & (m >> 1) & (m >> 2) & (m >> 3) & 0x1111111111111111ull;
}
__device__ inline uint64_t expand_groups(uint64_t g) { return g | (g << 1) | (g << 2) | (g << 3); }

// The FP32 near-field record of target leaf b and source leaf c, two float4
// at 2t and 2t + 1 for strong entry t.  The first: the centre offset
// c_b - c_c rounded to FP32 and the squared distance below which a pair
// counts as coincident.  In b's own leaf both sides of a pair subtract the
// same rounded offsets, so duplicates give exactly r^2 = 0 and only r^2
// below the smallest normal float is masked (the logarithm's argument stays
// normal).  Across leaves a coincident pair shows a rounding distance: with
// u = 2^-24, the offsets x - c_b and x - c_c, the FP32 c_b - c_c, the source
// offset in b's frame and the difference are each rounded once, so
// |dx| + |dy| <= u (2 sqrt2 R_b + sqrt2 R_c + |dxc| + |dyc|) <= 3 u mag;
// the threshold 2^-21 mag = 8 u mag keeps a factor above 2 on that bound.
// The fourth component flags a separated pair of leaves: when the gap
// between the two rectangles (rb, rc: xlo, xhi, ylo, yhi) along x or y
// exceeds 2^-20 mag = 16 u mag, every pair is at least that far apart, its
// FP32 offsets are off by at most u (2 R_b + 4 R_c + 2 |dxc| + 2 |dyc|)
// <= 4 u mag, so its FP32 r^2 exceeds (12 u mag)^2 > threshold and the near
// kernels may skip the coincidence test for the record.
// The second, for the differences in two FP32 parts (mode FP32_ACC64): the
// low part of the centre offset (c_b - c_c minus its FP32 rounding) and the
// coincidence threshold of that form.  There the offsets carry about 48
// bits, the source offset in b's frame is formed by an exact two-term
// difference, and a pair's difference is off by at most about
// u |dx| + 2^-45 mag; pairs closer than 2^-42 mag count as coincident.
__device__ inline void near_record(float4 *__restrict__ recd, int64_t t, double4 gb, double4 gc, double4 rb,
                                   double4 rc, bool self) {
    const double ddx = gb.x - gc.x, ddy = gb.y - gc.y;
    const float dxc = (float)ddx, dyc = (float)ddy;
    const float mag = fabsf(dxc) + fabsf(dyc) + (float)gb.z + (float)gc.z;
    const float thr = self ? 0x1p-126f : (mag * 0x1p-21f) * (mag * 0x1p-21f);
    const float thr2 = self ? 0x1p-126f : fmaxf((mag * 0x1p-42f) * (mag * 0x1p-42f), 0x1p-126f);
    const double gap = fmax(fmax(rb.x - rc.y, rc.x - rb.y), fmax(rb.z - rc.w, rc.z - rb.w));
    const bool sep = !self && gap > 0x1p-20 * (double)mag;
    recd[2 * t] = make_float4(dxc, dyc, thr, sep ? 1.f : 0.f);
    recd[2 * t + 1] = make_float4((float)(ddx - (double)dxc), (float)(ddy - (double)dyc), thr2, 0.f);
}

// Level 0: S_0(root) = {root}, W_0(root) empty; for a one-level tree
// (L = 0) also the near-field record of that single strong entry, written
// as the finest fill pass writes the others.
__global__ void k_lists_init(int32_t *sptr0, int32_t *wptr0, int32_t *xptr0, int32_t *sidx_pool, int64_t *pool_state,
                             int L,
                             const int32_t *stL, const double4 *geom0, const double4 *rect0, int2 *recj, float4 *recd,
                             int32_t *owner0, int32_t *selfpos) {
    sptr0[0] = 0;
    sptr0[1] = 1;
    wptr0[0] = 0;
    wptr0[1] = 0;
    xptr0[0] = 0;
    xptr0[1] = 0;
    sidx_pool[0] = 0;
    for (int k = 0; k <= slot_flag(L); ++k) pool_state[k] = 0;
    pool_state[1] = 1;  // S offset of level 1
    owner0[0] = 0;      // row of level 0's one strong entry (a flat level 1 decodes by it)
    if (L == 0) {
        selfpos[0] = 0;
        recj[0] = make_int2(stL[0], stL[1]);
        near_record(recd, 0, geom0[0], geom0[0], rect0[0], rect0[0], true);
    }
}

// One wavefront, box b of level l (candidates: the four children of each box
// of S_{l-1}(parent)), for the levels done in one workgroup.  Count pass
// (FILL = false): the decisions of every candidate and the three counts.
// Fill pass: the same decisions, ballot compaction into the lists, the owner
// (row) of every strong entry when the next level needs it, and on the
// finest level the near-field record of each strong entry (source leaf's
// point range and near_record's offset and threshold for the FP32 path).
// A candidate is weak (criterion holds), exchanged (opt: the criterion with
// the radii exchanged holds), or strong; with the parent option a group of
// four weak children whose parent q passes the criterion too becomes one
// weak entry q | VFLAG (a box of the level above).  Groups of four are
// aligned to four lanes: each box has 4 |S_{l-1}(P)| candidates.
struct ListDecision {
    uint64_t ms, mwo, mx, mv;  // strong, W output (weak or group head), exchanged, group heads
};
__device__ inline ListDecision decide(bool ok, bool weak, bool exch, bool vhead_ok) {
    ListDecision d;
    const uint64_t okm = __ballot(ok);
    const uint64_t mw = __ballot(weak);
    d.mx = __ballot(exch);
    // a group head passes when its four lanes are weak and the parent test holds
    const uint64_t cand_heads = full_groups(mw);
    const uint32_t lane = lane_id();
    d.mv = __ballot(vhead_ok && ((cand_heads >> lane) & 1));
    d.mwo = (mw & ~expand_groups(d.mv)) | d.mv;
    d.ms = okm & ~mw & ~d.mx;
    return d;
}

template <bool FILL>
__device__ inline void box_lists(int l, int L, int opt, double theta, const double4 *__restrict__ geomL,
                                 const double4 *__restrict__ geomP, int64_t b,
                                 const int32_t *__restrict__ sptr_prev, const int32_t *__restrict__ sidx_prev,
                                 int32_t &cs, int32_t &cw, int32_t &cx, int32_t tS, int32_t *__restrict__ so,
                                 int32_t *__restrict__ wo, int32_t *__restrict__ xo, int32_t *__restrict__ own,
                                 int32_t *__restrict__ self, const int32_t *__restrict__ stL,
                                 const double4 *__restrict__ rectL, int2 *__restrict__ recj,
                                 float4 *__restrict__ recd) {
    const uint32_t lane = lane_id();
    const int64_t P = b >> 2;
    const int32_t s0 = sptr_prev[P], s1 = sptr_prev[P + 1];
    const int32_t ncand = 4 * (s1 - s0);
    const bool records = FILL && l == L && recj != nullptr;
    const bool swap = opt_swap(opt, l, L), par = opt_parent(opt);
    const double4 gb = geomL[b];
    cs = 0;
    cw = 0;
    cx = 0;
    for (int32_t base = 0; base < ncand; base += 64) {
        const int32_t j = base + (int32_t)lane;
        const bool ok = j < ncand;
        int32_t cbox = 0, ent = 0;
        double4 gc = gb;
        if (ok) {
            ent = sidx_prev[s0 + (j >> 2)];
            cbox = 4 * ent + (j & 3);
            gc = geomL[cbox];
        }
        const bool weak = ok && theta_separated(theta, theta * theta, gb, gc);
        const bool exch = swap && ok && !weak && exchange_separated(theta, theta * theta, gb, gc);
        const bool vtest = par && ok && (j & 3) == 0 && theta_separated(theta, theta * theta, gb, geomP[ent]);
        const ListDecision d = decide(ok, weak, exch, vtest);
        if (FILL && ok) {
            if ((d.mwo >> lane) & 1) {
                wo[cw + (int32_t)popc_below(d.mwo)] = ((d.mv >> lane) & 1) ? (ent | VFLAG) : cbox;
            } else if ((d.mx >> lane) & 1) {
                xo[cx + (int32_t)popc_below(d.mx)] = cbox;
            } else if ((d.ms >> lane) & 1) {
                const int32_t pos = cs + (int32_t)popc_below(d.ms);
                so[pos] = cbox;
                if (own) own[tS + pos] = (int32_t)b;
                if (self && cbox == b) self[b] = tS + pos;
                if (records) {
                    const int32_t t = tS + pos;
                    recj[t] = make_int2(stL[cbox], stL[cbox + 1]);
                    near_record(recd, t, gb, gc, rectL[b], rectL[cbox], cbox == b);
                }
            }
        }
        cw += (int32_t)__popcll(d.mwo);
        cs += (int32_t)__popcll(d.ms);
        cx += (int32_t)__popcll(d.mx);
    }
}

// Pool offsets of level l + 1, and the checks that guard the next level:
// the LIST_GROW_* bits of the pools that are too small (the host retries
// with larger ones; LIST_GROW_CAND: level l + 1's candidates exceed the free
// space, which bounds the decision words), 2 when level l + 1's candidates,
// 16 |S_l| (each becomes at most one entry), exceed the entry limit.  A flagged level is not examined, so no
// int32 prefix sum can wrap and no decision bit lies beyond the buffer
// (sized for cap_s + cap_w candidates).
__device__ inline void advance_pools(int l, int L, int64_t nb, const int32_t *sptr_cur, const int32_t *wptr_cur,
                                     const int32_t *xptr_cur, int64_t *pool_state, int64_t cap_s, int64_t cap_w,
                                     int64_t cap_x, int64_t limit) {
    if (pool_state[slot_flag(L)]) return;
    const int64_t so = pool_state[l] + sptr_cur[nb];
    const int64_t wo = pool_state[(L + 2) + l] + wptr_cur[nb];
    const int64_t xo = pool_state[slot_x(L, l)] + (xptr_cur ? xptr_cur[nb] : 0);
    pool_state[l + 1] = so;
    pool_state[(L + 2) + l + 1] = wo;
    pool_state[slot_x(L, l + 1)] = xo;
    // which pool is too small (the host grows only those), or the next
    // level's candidates exceed the entry limit (2)
    const int64_t grow = (so > cap_s ? LIST_GROW_S : 0) | (wo > cap_w ? LIST_GROW_W : 0) |
                         (xo > cap_x ? LIST_GROW_X : 0);
    if (grow) {
        pool_state[slot_flag(L)] = grow;
        return;
    }
    if (l < L) {
        const int64_t cand = 16 * (int64_t)sptr_cur[nb];
        if (cand > limit) pool_state[slot_flag(L)] = 2;
        else if (cand > (cap_s - so) + (cap_w - wo)) pool_state[slot_flag(L)] = LIST_GROW_CAND;
    }
}

__global__ void k_lists_advance(int l, int L, int64_t nb, const int32_t *sptr_cur, const int32_t *wptr_cur,
                                const int32_t *xptr_cur, int64_t *pool_state, int64_t cap_s, int64_t cap_w,
                                int64_t cap_x, int64_t limit) {
    advance_pools(l, L, nb, sptr_cur, wptr_cur, xptr_cur, pool_state, cap_s, cap_w, cap_x, limit);
}

// Levels 1..K (4^K <= SMALL_BOXES boxes each) in one workgroup, which saves
// the launches of the coarse levels: the geometry of levels 0..K staged in
// LDS, and per level a count pass over the boxes (one wavefront per box), the
// two row-pointer scans in LDS, the pool offsets and checks, and a fill pass
// that tests the candidates again (cheaper here than storing the decisions).
constexpr int SMALL_THREADS = 1024;
constexpr int SMALL_BOXES = 64;
constexpr int SMALL_GEOM = 85;  // boxes of levels 0..3
__global__ void __launch_bounds__(SMALL_THREADS) k_lists_small(int K, int L, int opt, double theta,
                                                              const double4 *__restrict__ geom,
                                                              int32_t *__restrict__ sptr, int32_t *__restrict__ wptr,
                                                              int32_t *__restrict__ xptr,
                                                              int32_t *__restrict__ sidx_pool,
                                                              int32_t *__restrict__ widx_pool,
                                                              int32_t *__restrict__ xidx_pool,
                                                              int64_t *__restrict__ pool_state, int64_t cap_s,
                                                              int64_t cap_w, int64_t cap_x, int64_t limit,
                                                              const int32_t *__restrict__ stL,
                                                              const double4 *__restrict__ rectL,
                                                              int2 *__restrict__ recj, float4 *__restrict__ recd,
                                                              int32_t *__restrict__ owner,
                                                              int32_t *__restrict__ selfpos) {
    __shared__ int32_t ns[SMALL_BOXES], nw[SMALL_BOXES], nx[SMALL_BOXES];
    __shared__ int32_t tmp[SMALL_THREADS / 64];
    __shared__ int flag;
    __shared__ double4 g_s[SMALL_GEOM];
    const int t = threadIdx.x, wv = t / 64;
    constexpr int NWV = SMALL_THREADS / 64;
    if (t < level_offset(K + 1)) g_s[t] = geom[t];
    for (int l = 1; l <= K; ++l) {
        if (t == 0) flag = (int)pool_state[slot_flag(L)];
        __syncthreads();
        if (flag) return;  // uniform: every thread read the same flag
        const int64_t nb = int64_t(1) << (2 * l);
        const double4 *gL = g_s + level_offset(l);
        const double4 *gP = g_s + level_offset(l - 1);
        const int32_t *sp_prev = sptr + ptr_offset(l - 1);
        int32_t *sp_cur = sptr + ptr_offset(l), *wp_cur = wptr + ptr_offset(l), *xp_cur = xptr + ptr_offset(l);
        const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
        for (int64_t b = wv; b < nb; b += NWV) {
            int32_t cs, cw, cx;
            box_lists<false>(l, L, opt, theta, gL, gP, b, sp_prev, sidx_prev, cs, cw, cx, 0, nullptr, nullptr,
                             nullptr, nullptr, nullptr, stL, nullptr, nullptr, nullptr);
            if (lane_id() == 0) {
                ns[b] = cs;
                nw[b] = cw;
                nx[b] = cx;
            }
        }
        __syncthreads();
        int32_t tot_s, tot_w, tot_x;
        const int32_t vs = t < nb ? ns[t] : 0, vw = t < nb ? nw[t] : 0, vx = t < nb ? nx[t] : 0;
        const int32_t es = block_excl_scan<SMALL_THREADS>(vs, tmp, tot_s);
        const int32_t ew = block_excl_scan<SMALL_THREADS>(vw, tmp, tot_w);
        const int32_t ex = block_excl_scan<SMALL_THREADS>(vx, tmp, tot_x);
        if (t < nb) {
            sp_cur[t] = es;
            wp_cur[t] = ew;
            xp_cur[t] = ex;
        }
        if (t == 0) {
            sp_cur[nb] = tot_s;
            wp_cur[nb] = tot_w;
            xp_cur[nb] = tot_x;
        }
        __threadfence_block();
        __syncthreads();
        if (t == 0) {
            advance_pools(l, L, nb, sp_cur, wp_cur, xp_cur, pool_state, cap_s, cap_w, cap_x, limit);
            flag = (int)pool_state[slot_flag(L)];
        }
        __syncthreads();
        // a flagged level is not filled (the host discards or retries the lists)
        if (flag) return;
        const int64_t so0 = pool_state[l], wo0 = pool_state[(L + 2) + l], xo0 = pool_state[slot_x(L, l)];
        for (int64_t b = wv; b < nb; b += NWV) {
            int32_t cs, cw, cx;
            box_lists<true>(l, L, opt, theta, gL, gP, b, sp_prev, sidx_prev, cs, cw, cx, sp_cur[b],
                            sidx_pool + so0 + sp_cur[b], widx_pool + wo0 + wp_cur[b], xidx_pool + xo0 + xp_cur[b],
                            l == K ? owner : nullptr, l == L ? selfpos : nullptr, stL, rectL, recj, recd);
        }
        __syncthreads();
    }
}

// ---- flat passes (levels with more than 64 boxes) -----------------------
constexpr int FB = 4;                 // words (chunks of 64 candidates) per wavefront step
constexpr unsigned FLAT_BLOCKS = 2048;  // 8192 wavefronts
constexpr int WS_T = 256, WS_PER = 16, WS_TILE = WS_T * WS_PER;  // word scan tiles

// Decodes FB words of candidates: box b, candidate box cbox (child of the
// level above's box ent), and whether q is its box's first candidate.  The
// loads of each step are issued for all FB words before any is used.
struct FlatCand {
    bool ok[FB], first[FB];
    int32_t b[FB], cbox[FB], ent[FB];
};
__device__ inline void flat_decode(int64_t w0, int64_t NC, const int32_t *__restrict__ owner_prev,
                                   const int32_t *__restrict__ sptr_prev, const int32_t *__restrict__ sidx_prev,
                                   FlatCand &fc) {
    const uint32_t lane = lane_id();
    int32_t P[FB], s0[FB], s1[FB], child[FB];
#pragma unroll
    for (int u = 0; u < FB; ++u) {
        const int64_t q = (w0 + u) * 64 + lane;
        fc.ok[u] = q < NC;
        P[u] = fc.ok[u] ? owner_prev[q >> 4] : 0;
    }
#pragma unroll
    for (int u = 0; u < FB; ++u) {
        s0[u] = fc.ok[u] ? sptr_prev[P[u]] : 0;
        s1[u] = fc.ok[u] ? sptr_prev[P[u] + 1] : 1;
    }
#pragma unroll
    for (int u = 0; u < FB; ++u) {
        const int64_t q = (w0 + u) * 64 + lane;
        const int32_t r = fc.ok[u] ? (int32_t)(q - 16 * (int64_t)s0[u]) : 0;
        const int32_t m4 = 4 * (s1[u] - s0[u]);  // candidates per child box
        const int c = (r >= m4 ? 1 : 0) + (r >= 2 * m4 ? 1 : 0) + (r >= 3 * m4 ? 1 : 0);
        const int32_t j = r - c * m4;
        fc.b[u] = 4 * P[u] + c;
        fc.first[u] = fc.ok[u] && j == 0;
        child[u] = j & 3;
        fc.ent[u] = fc.ok[u] ? sidx_prev[s0[u] + (j >> 2)] : 0;
    }
#pragma unroll
    for (int u = 0; u < FB; ++u) fc.cbox[u] = 4 * fc.ent[u] + child[u];
}

// Candidates of level l: 16 |S_{l-1}| (the previous level's total).
__device__ inline int64_t level_candidates(const int32_t *sptr_prev, int64_t nb_prev) {
    return 16 * (int64_t)sptr_prev[nb_prev];
}

// The decision masks of one word (see box_lists): weak and exchanged lanes,
// and with the parent option the heads of fully weak groups whose parent
// box passes the criterion (its geometry loaded only for such heads).
__device__ inline ListDecision flat_masks(bool OPT, int opt, int l, int L, double theta, bool ok, int32_t ent,
                                          double4 gb, double4 gc, const double4 *__restrict__ geomP) {
    const bool weak = ok && theta_separated(theta, theta * theta, gb, gc);
    if (!OPT) {
        ListDecision d;
        const uint64_t okm = __ballot(ok);
        const uint64_t mw = __ballot(weak);
        d.mwo = mw;
        d.mx = 0;
        d.mv = 0;
        d.ms = okm & ~mw;
        return d;
    }
    const bool exch = opt_swap(opt, l, L) && ok && !weak && exchange_separated(theta, theta * theta, gb, gc);
    bool vok = false;
    if (opt_parent(opt)) {
        const uint64_t heads = full_groups(__ballot(weak));
        if ((heads >> lane_id()) & 1) vok = theta_separated(theta, theta * theta, gb, geomP[ent]);
    }
    return decide(ok, weak, exch, vok);
}

// lvth: each level's threshold on the device (relaxed criterion), else
// nullptr and theta for every level.
template <bool OPT>
__global__ void __launch_bounds__(256) k_flat_count(int l, int L, int opt, double theta,
                                                    const double *__restrict__ lvth,
                                                    const double4 *__restrict__ geomL,
                                                    const double4 *__restrict__ geomP,
                                                    const int32_t *__restrict__ sptr_prev, int64_t nb_prev,
                                                    const int32_t *__restrict__ sidx_pool,
                                                    const int32_t *__restrict__ owner_prev,
                                                    const int64_t *__restrict__ pool_state,
                                                    uint64_t *__restrict__ bits, int64_t wcap,
                                                    int32_t *__restrict__ cnt_s, int32_t *__restrict__ cnt_w,
                                                    int32_t *__restrict__ cnt_x) {
    if (pool_state[slot_flag(L)]) return;  // uniform
    const double th = lvth ? lvth[l] : theta;
    const int64_t NC = level_candidates(sptr_prev, nb_prev);
    const int64_t nwords = (NC + 63) >> 6;
    const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
    const uint32_t lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t w0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * FB; w0 < nwords;
         w0 += nwaves * FB) {
        FlatCand fc;
        flat_decode(w0, NC, owner_prev, sptr_prev, sidx_prev, fc);
        double4 gb[FB], gc[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            gb[u] = fc.ok[u] ? geomL[fc.b[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
            gc[u] = fc.ok[u] ? geomL[fc.cbox[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
        }
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const ListDecision d = flat_masks(OPT, opt, l, L, th, fc.ok[u], fc.ent[u], gb[u], gc[u], geomP);
            if (lane == (uint32_t)u && w0 + u < nwords) {
                bits[w0 + u] = d.mwo;
                cnt_s[w0 + u] = (int32_t)__popcll(d.ms);
                cnt_w[w0 + u] = (int32_t)__popcll(d.mwo);
                if (OPT) {
                    bits[wcap + w0 + u] = d.mx;
                    bits[2 * wcap + w0 + u] = d.mv;
                    cnt_x[w0 + u] = (int32_t)__popcll(d.mx);
                }
            }
        }
    }
}

// ---- relaxed criterion (Section 4, last paragraph) ----------------------
// Every candidate of level l is binned by the least threshold t_k of the
// grid (tk, nbin entries, ascending) at which the criterion holds, and the
// bins are counted (hist, nbin counters of the level, zeroed beforehand).
// The criterion is monotone in t on the grid (neighbouring thresholds lie
// far more than rounding apart), so a bisection finds the least one.  Each
// block counts in LDS and adds its counts once.
__global__ void __launch_bounds__(256) k_relax_hist(int l, int L, int nbin, const double *__restrict__ tk,
                                                    const double4 *__restrict__ geomL,
                                                    const int32_t *__restrict__ sptr_prev, int64_t nb_prev,
                                                    const int32_t *__restrict__ sidx_pool,
                                                    const int32_t *__restrict__ owner_prev,
                                                    const int64_t *__restrict__ pool_state,
                                                    uint32_t *__restrict__ hist) {
    __shared__ uint32_t h[RELAX_MAX_BINS];
    __shared__ double t_s[RELAX_MAX_BINS];
    for (int k = threadIdx.x; k < nbin; k += blockDim.x) {
        h[k] = 0;
        t_s[k] = tk[k];
    }
    __syncthreads();
    if (!pool_state[slot_flag(L)]) {  // uniform: a flagged level is not examined
        const int64_t NC = level_candidates(sptr_prev, nb_prev);
        const int64_t nwords = (NC + 63) >> 6;
        const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
        const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
        for (int64_t w0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * FB; w0 < nwords;
             w0 += nwaves * FB) {
            FlatCand fc;
            flat_decode(w0, NC, owner_prev, sptr_prev, sidx_prev, fc);
            double4 gb[FB], gc[FB];
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                gb[u] = fc.ok[u] ? geomL[fc.b[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
                gc[u] = fc.ok[u] ? geomL[fc.cbox[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
            }
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                if (!fc.ok[u]) continue;
                int lo = 0, hi = nbin;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    const double t = t_s[mid];
                    if (theta_separated(t, t * t, gb[u], gc[u])) hi = mid;
                    else lo = mid + 1;
                }
                if (lo < nbin) atomicAdd(&h[lo], 1u);
            }
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < nbin; k += blockDim.x)
        if (h[k]) atomicAdd(&hist[k], h[k]);
}

// The level's admitted bins: the largest K >= k0 - 1 such that for every k
// from k0 - 1 to K the counts of bins 0..k satisfy
//     sum_j count_j t_j^(p+1) <= theta^(p+1) sum_j count_j
// (binary64, summed in bin order, products and sums rounded one by one);
// writes K and t_K, the threshold the count and fill passes then apply.
__global__ void k_relax_pick(int l, int L, int nbin, int k0, double etheta, const double *__restrict__ tk,
                             const double *__restrict__ ek, const uint32_t *__restrict__ hist,
                             double *__restrict__ lvth, int32_t *__restrict__ lvk,
                             const int64_t *__restrict__ pool_state) {
#pragma clang fp contract(off)
    if (threadIdx.x != 0 || pool_state[slot_flag(L)]) return;
    double sum = 0.0;
    int64_t n = 0;
    int K = k0 - 1;
    for (int k = 0; k < nbin; ++k) {
        const double term = (double)hist[k] * ek[k];
        sum = sum + term;
        n += hist[k];
        if (k < k0 - 1) continue;
        if (k > k0 - 1 && !(sum <= etheta * (double)n)) break;
        K = k;
    }
    lvk[l] = K;
    lvth[l] = tk[K];
}

// Zeroes the bin counts of all levels; level 0 (the root alone) admits the
// plain threshold.
__global__ void k_relax_init(int L, int nbin, int k0, double theta, uint32_t *__restrict__ hist,
                             double *__restrict__ lvth, int32_t *__restrict__ lvk) {
    for (int64_t i = threadIdx.x; i < (int64_t)(L + 1) * nbin; i += blockDim.x) hist[i] = 0;
    if (threadIdx.x == 0) {
        for (int l = 0; l <= L; ++l) {
            lvth[l] = theta;
            lvk[l] = k0 - 1;
        }
    }
}

// Exclusive scan of the per-word counts over the level's words (a length
// known on the device): tile sums, one block over the tile sums (which also
// writes the level totals as the last row pointers), and the tiles in place.
// NA = 2 (S, W) or 3 (S, W, X) arrays.
__device__ inline int64_t level_words(const int32_t *sptr_prev, int64_t nb_prev) {
    return (level_candidates(sptr_prev, nb_prev) + 63) >> 6;
}

template <int NA>
__global__ void __launch_bounds__(WS_T) k_wscan_tiles(int L, const int32_t *__restrict__ sptr_prev, int64_t nb_prev,
                                                      const int64_t *__restrict__ pool_state,
                                                      const int32_t *__restrict__ cnt_s,
                                                      const int32_t *__restrict__ cnt_w,
                                                      const int32_t *__restrict__ cnt_x, int32_t *__restrict__ tsum,
                                                      int ntile) {
    __shared__ int32_t tmp[WS_T / 64];
    const bool dead = pool_state[slot_flag(L)] != 0;
    const int64_t nwords = dead ? 0 : level_words(sptr_prev, nb_prev);
    const int64_t base = (int64_t)blockIdx.x * WS_TILE + threadIdx.x * WS_PER;
    const int32_t *arrs[3] = {cnt_s, cnt_w, cnt_x};
    int32_t v[NA][WS_PER], a[NA];
#pragma unroll
    for (int k = 0; k < WS_PER; ++k) {  // all loads in flight first (word 0 always exists)
        const int64_t i = base + k < nwords ? base + k : 0;
#pragma unroll
        for (int r = 0; r < NA; ++r) v[r][k] = arrs[r][i];
    }
#pragma unroll
    for (int r = 0; r < NA; ++r) {
        a[r] = 0;
#pragma unroll
        for (int k = 0; k < WS_PER; ++k)
            if (base + k < nwords) a[r] += v[r][k];
    }
#pragma unroll
    for (int r = 0; r < NA; ++r) {
        int32_t tr;
        block_excl_scan<WS_T>(a[r], tmp, tr);
        if (threadIdx.x == 0) tsum[(int64_t)r * ntile + blockIdx.x] = tr;
    }
}

// Exclusive scan of the word counts of one level in place: each tile adds
// the sum of the tile sums before it (formed by the block itself: a level has
// a few hundred tiles at most) to its own scan.  The last tile of the level
// writes the level totals as the last row pointers; tile 0 runs even when the
// level has no word, so that the totals are 0 then.
template <int NA>
__global__ void __launch_bounds__(WS_T) k_wscan_apply(int L, const int32_t *__restrict__ sptr_prev, int64_t nb_prev,
                                                      const int64_t *__restrict__ pool_state,
                                                      int32_t *__restrict__ cnt_s, int32_t *__restrict__ cnt_w,
                                                      int32_t *__restrict__ cnt_x, const int32_t *__restrict__ tsum,
                                                      int ntile, int32_t *__restrict__ sptr_cur,
                                                      int32_t *__restrict__ wptr_cur, int32_t *__restrict__ xptr_cur,
                                                      int64_t nb) {
    __shared__ int32_t tmp[WS_T / 64];
    if (pool_state[slot_flag(L)]) return;  // uniform
    const int64_t nwords = level_words(sptr_prev, nb_prev);
    const int64_t nact = (nwords + WS_TILE - 1) / WS_TILE;
    const int64_t last = nact > 1 ? nact - 1 : 0;
    if ((int64_t)blockIdx.x > last) return;  // uniform
    const int64_t base = (int64_t)blockIdx.x * WS_TILE + threadIdx.x * WS_PER;
    int32_t *arrs[3] = {cnt_s, cnt_w, cnt_x};
    int32_t *ptrs[3] = {sptr_cur, wptr_cur, xptr_cur};
    for (int arr = 0; arr < NA; ++arr) {
        const int32_t *ts = tsum + (int64_t)arr * ntile;
        int32_t s = 0;
        for (int k = threadIdx.x; k < (int)blockIdx.x; k += WS_T) s += ts[k];
        int32_t before;
        (void)block_excl_scan<WS_T>(s, tmp, before);  // the tile sums before this tile
        int32_t *cnt = arrs[arr];
        int32_t v[WS_PER], sum = 0;
#pragma unroll
        for (int k = 0; k < WS_PER; ++k) {
            v[k] = base + k < nwords ? cnt[base + k] : 0;
            sum += v[k];
        }
        int32_t total;
        int32_t run = block_excl_scan<WS_T>(sum, tmp, total) + before;
#pragma unroll
        for (int k = 0; k < WS_PER; ++k) {
            if (base + k < nwords) cnt[base + k] = run;
            run += v[k];
        }
        if ((int64_t)blockIdx.x == last && threadIdx.x == 0) ptrs[arr][nb] = before + total;
    }
}

// Fill pass: every candidate's pool position from the word prefixes and its
// bits; row pointers at each box's first candidate; owners for the next
// level; near-field records on the finest level.
template <bool OPT>
__global__ void __launch_bounds__(256) k_flat_fill(int l, int L, const double4 *__restrict__ geomL,
                                                   const int32_t *__restrict__ sptr_prev, int64_t nb_prev,
                                                   int32_t *__restrict__ sidx_pool, int32_t *__restrict__ widx_pool,
                                                   int32_t *__restrict__ xidx_pool,
                                                   const int32_t *__restrict__ owner_prev,
                                                   int32_t *__restrict__ owner_cur,
                                                   const int64_t *__restrict__ pool_state,
                                                   const uint64_t *__restrict__ bits, int64_t wcap,
                                                   const int32_t *__restrict__ pre_s, const int32_t *__restrict__ pre_w,
                                                   const int32_t *__restrict__ pre_x,
                                                   int32_t *__restrict__ sptr_cur, int32_t *__restrict__ wptr_cur,
                                                   int32_t *__restrict__ xptr_cur,
                                                   const int32_t *__restrict__ stL,
                                                   const double4 *__restrict__ rectL, int2 *__restrict__ recj,
                                                   float4 *__restrict__ recd, int32_t *__restrict__ selfpos) {
    if (pool_state[slot_flag(L)]) return;  // uniform
    const int64_t NC = level_candidates(sptr_prev, nb_prev);
    const int64_t nwords = (NC + 63) >> 6;
    const int32_t *sidx_prev = sidx_pool + pool_state[l - 1];
    int32_t *sout = sidx_pool + pool_state[l];
    int32_t *wout = widx_pool + pool_state[(L + 2) + l];
    int32_t *xout = OPT ? xidx_pool + pool_state[slot_x(L, l)] : nullptr;
    const bool records = l == L;
    const uint32_t lane = lane_id();
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t w0 = ((int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * FB; w0 < nwords;
         w0 += nwaves * FB) {
        FlatCand fc;
        flat_decode(w0, NC, owner_prev, sptr_prev, sidx_prev, fc);
        uint64_t mwo[FB], mx[FB], mv[FB];
        int32_t ps[FB], pw[FB], px[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const bool wk = w0 + u < nwords;
            mwo[u] = wk ? bits[w0 + u] : 0ull;
            ps[u] = wk ? pre_s[w0 + u] : 0;
            pw[u] = wk ? pre_w[w0 + u] : 0;
            mx[u] = (OPT && wk) ? bits[wcap + w0 + u] : 0ull;
            mv[u] = (OPT && wk) ? bits[2 * wcap + w0 + u] : 0ull;
            px[u] = (OPT && wk) ? pre_x[w0 + u] : 0;
        }
        uint64_t ms[FB];
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const uint64_t okm = __ballot(fc.ok[u]);
            // strong: neither weak (W output or a member of a parent group) nor exchanged
            ms[u] = okm & ~(mwo[u] | expand_groups(mv[u]) | mx[u]);
        }
        double4 gb[FB], gc[FB], rb[FB], rc[FB];
        int2 rr[FB];
        if (records) {
#pragma unroll
            for (int u = 0; u < FB; ++u) {
                const bool strong = (ms[u] >> lane) & 1;
                gb[u] = strong ? geomL[fc.b[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
                gc[u] = strong ? geomL[fc.cbox[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
                rb[u] = strong ? rectL[fc.b[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
                rc[u] = strong ? rectL[fc.cbox[u]] : make_double4(0.0, 0.0, 0.0, 0.0);
                rr[u] = strong ? make_int2(stL[fc.cbox[u]], stL[fc.cbox[u] + 1]) : make_int2(0, 0);
            }
        }
#pragma unroll
        for (int u = 0; u < FB; ++u) {
            const int32_t posS = ps[u] + (int32_t)popc_below(ms[u]);
            const int32_t posW = pw[u] + (int32_t)popc_below(mwo[u]);
            const int32_t posX = px[u] + (int32_t)popc_below(mx[u]);
            if (fc.ok[u]) {
                if ((mwo[u] >> lane) & 1) {
                    wout[posW] = (OPT && ((mv[u] >> lane) & 1)) ? (fc.ent[u] | VFLAG) : fc.cbox[u];
                } else if (OPT && ((mx[u] >> lane) & 1)) {
                    xout[posX] = fc.cbox[u];
                } else if ((ms[u] >> lane) & 1) {
                    sout[posS] = fc.cbox[u];
                    if (owner_cur) owner_cur[posS] = fc.b[u];
                    if (records && fc.cbox[u] == fc.b[u]) selfpos[fc.b[u]] = posS;
                    if (records) {
                        recj[posS] = rr[u];
                        near_record(recd, posS, gb[u], gc[u], rb[u], rc[u], fc.cbox[u] == fc.b[u]);
                    }
                }
                if (fc.first[u]) {
                    sptr_cur[fc.b[u]] = posS;
                    wptr_cur[fc.b[u]] = posW;
                    if (OPT) xptr_cur[fc.b[u]] = posX;
                }
            }
        }
    }
}

}  // namespace

hipError_t build_lists_device(fmm2d_ctx *c, double theta, int opt, int64_t cap_s, int64_t cap_w, int64_t cap_x,
                              int64_t limit, int *overflow, const RelaxRule *rx) {
    TreeState &t = c->tree;
    const int L = t.L;
    const int64_t nptr = ptr_offset(L + 1);
    const bool OPT = opt != 0;
    FMM2D_TRY(side_join(c));  // side-stream work still reading the previous lists
    FMM2D_TRY(t.sptr.ensure(sizeof(int32_t) * nptr));
    FMM2D_TRY(t.wptr.ensure(sizeof(int32_t) * nptr));
    FMM2D_TRY(t.xptr.ensure(sizeof(int32_t) * nptr));
    FMM2D_TRY(t.sidx.ensure(sizeof(int32_t) * cap_s));
    FMM2D_TRY(t.widx.ensure(sizeof(int32_t) * cap_w));
    FMM2D_TRY(t.xidx.ensure(sizeof(int32_t) * (cap_x > 0 ? cap_x : 1)));
    FMM2D_TRY(t.pool_state.ensure(sizeof(int64_t) * (slot_flag(L) + 1)));
    int32_t *sptr = t.sptr.as<int32_t>(), *wptr = t.wptr.as<int32_t>(), *xptr = t.xptr.as<int32_t>();
    int64_t *ps = t.pool_state.as<int64_t>();
    const double4 *geom = t.geom.as<double4>();
    // Level 1 has 16 candidates (the root's children, four per box); later
    // levels are guarded on the device, so the host never waits inside the
    // level loop.
    if (L >= 1 && 16 > limit) {
        *overflow = 2;
        return hipSuccess;
    }
    // near-field records of the finest level's strong entries (<= cap_s)
    FMM2D_TRY(t.nrec_j.ensure(sizeof(int2) * cap_s));
    FMM2D_TRY(t.nrec_d.ensure(sizeof(float4) * 2 * cap_s));
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    // owners (rows) of the S entries of a level, for the next level's
    // decoding and (finest level) the near field; two buffers by level
    // parity; the position of every leaf in its own list
    FMM2D_TRY(t.owner0.ensure(sizeof(int32_t) * cap_s));
    FMM2D_TRY(t.owner1.ensure(sizeof(int32_t) * cap_s));
    FMM2D_TRY(t.selfpos.ensure(sizeof(int32_t) * (size_t)(int64_t(1) << (2 * L))));
    int32_t *owner[2] = {t.owner0.as<int32_t>(), t.owner1.as<int32_t>()};
    int32_t *selfpos = t.selfpos.as<int32_t>();
    // (xlo, xhi, ylo, yhi) per leaf: the points' bounding boxes when the
    // balls are drawn around them (the near records' separation test)
    const double4 *rectL = (t.shrink ? t.prect : t.rects).as<double4>() + level_offset(L);
    hipLaunchKernelGGL(k_lists_init, dim3(1), dim3(1), 0, c->stream, sptr, wptr, xptr, t.sidx.as<int32_t>(), ps, L,
                       stL, geom, rectL, t.nrec_j.as<int2>(), t.nrec_d.as<float4>(), owner[0], selfpos);
    // relaxed criterion: the grid and its powers, zeroed bin counts; every
    // level then runs the flat passes (each needs its threshold first)
    const int nbin = rx ? rx->k0 + rx->k1 : 0;
    double *lvth = nullptr;
    if (rx) {
        FMM2D_TRY(t.relax_tk.ensure(sizeof(double) * 2 * nbin));
        FMM2D_TRY(t.relax_hist.ensure(sizeof(uint32_t) * (size_t)(L + 1) * nbin));
        FMM2D_TRY(t.relax_lv.ensure(sizeof(double) * (L + 1)));
        FMM2D_TRY(t.relax_k.ensure(sizeof(int32_t) * (L + 1)));
        FMM2D_TRY(hipMemcpyAsync(t.relax_tk.ptr, t.relax_host.data(), sizeof(double) * 2 * nbin,
                                 hipMemcpyHostToDevice, c->stream));
        lvth = t.relax_lv.as<double>();
        hipLaunchKernelGGL(k_relax_init, dim3(1), dim3(256), 0, c->stream, L, nbin, rx->k0, rx->theta,
                           t.relax_hist.as<uint32_t>(), lvth, t.relax_k.as<int32_t>());
    }
    // levels of at most 64 boxes: one workgroup, one launch
    int K = 0;
    while (!rx && K < L && (int64_t(1) << (2 * (K + 1))) <= SMALL_BOXES) ++K;
    if (K >= 1)
        hipLaunchKernelGGL(k_lists_small, dim3(1), dim3(SMALL_THREADS), 0, c->stream, K, L, opt, theta, geom, sptr,
                           wptr, xptr, t.sidx.as<int32_t>(), t.widx.as<int32_t>(), t.xidx.as<int32_t>(), ps, cap_s,
                           cap_w, cap_x, limit, stL, rectL, t.nrec_j.as<int2>(), t.nrec_d.as<float4>(), owner[K & 1],
                           selfpos);
    FMM2D_TRY(hipGetLastError());
    if (K < L) {
        // a level's candidates never exceed the free pool space (checked on
        // the device before the level runs), so cap_s + cap_w bounds the words
        const int64_t words = (cap_s + cap_w + 63) / 64 + 1;
        const int ntile = (int)((words + WS_TILE - 1) / WS_TILE);
        FMM2D_TRY(t.bits.ensure(sizeof(uint64_t) * (size_t)words * (OPT ? 3 : 1)));
        FMM2D_TRY(t.cnt_s.ensure(sizeof(int32_t) * (size_t)words));
        FMM2D_TRY(t.cnt_w.ensure(sizeof(int32_t) * (size_t)words));
        if (OPT) FMM2D_TRY(t.cnt_x.ensure(sizeof(int32_t) * (size_t)words));
        FMM2D_TRY(c->scr.tiles.ensure(sizeof(int32_t) * 3 * (size_t)ntile));
        uint64_t *bits = t.bits.as<uint64_t>();
        int32_t *cs = t.cnt_s.as<int32_t>(), *cw = t.cnt_w.as<int32_t>(), *tsum = c->scr.tiles.as<int32_t>();
        int32_t *cx = OPT ? t.cnt_x.as<int32_t>() : nullptr;
        const int64_t wv_needed = (words + FB - 1) / FB;
        const unsigned fgrid = (unsigned)std::min<int64_t>(FLAT_BLOCKS, (wv_needed + 3) / 4);
        for (int l = K + 1; l <= L; ++l) {
            const int64_t nb = int64_t(1) << (2 * l), nb_prev = nb >> 2;
            const int32_t *sp_prev = sptr + ptr_offset(l - 1);
            int32_t *sp_cur = sptr + ptr_offset(l), *wp_cur = wptr + ptr_offset(l);
            int32_t *xp_cur = OPT ? xptr + ptr_offset(l) : nullptr;
            const double4 *gL = geom + level_offset(l), *gP = geom + level_offset(l - 1);
            const int32_t *own_prev = owner[(l - 1) & 1];
            int32_t *own_cur = owner[l & 1];
            if (OPT) {
                hipLaunchKernelGGL(k_flat_count<true>, dim3(fgrid), dim3(256), 0, c->stream, l, L, opt, theta,
                                   (const double *)nullptr, gL, gP, sp_prev, nb_prev, t.sidx.as<int32_t>(), own_prev,
                                   ps, bits, words, cs, cw, cx);
                hipLaunchKernelGGL(k_wscan_tiles<3>, dim3(ntile), dim3(WS_T), 0, c->stream, L, sp_prev, nb_prev, ps,
                                   cs, cw, cx, tsum, ntile);
                hipLaunchKernelGGL(k_wscan_apply<3>, dim3(ntile), dim3(WS_T), 0, c->stream, L, sp_prev, nb_prev, ps,
                                   cs, cw, cx, tsum, ntile, sp_cur, wp_cur, xp_cur, nb);
            } else {
                if (rx) {
                    uint32_t *hl = t.relax_hist.as<uint32_t>() + (size_t)l * nbin;
                    const double *tk = t.relax_tk.as<double>();
                    hipLaunchKernelGGL(k_relax_hist, dim3(fgrid), dim3(256), 0, c->stream, l, L, nbin, tk, gL,
                                       sp_prev, nb_prev, t.sidx.as<int32_t>(), own_prev, ps, hl);
                    hipLaunchKernelGGL(k_relax_pick, dim3(1), dim3(64), 0, c->stream, l, L, nbin, rx->k0,
                                       rx->etheta, tk, tk + nbin, hl, lvth, t.relax_k.as<int32_t>(), ps);
                }
                hipLaunchKernelGGL(k_flat_count<false>, dim3(fgrid), dim3(256), 0, c->stream, l, L, opt, theta,
                                   (const double *)lvth, gL, gP, sp_prev, nb_prev, t.sidx.as<int32_t>(), own_prev,
                                   ps, bits, words, cs, cw, cx);
                hipLaunchKernelGGL(k_wscan_tiles<2>, dim3(ntile), dim3(WS_T), 0, c->stream, L, sp_prev, nb_prev, ps,
                                   cs, cw, cx, tsum, ntile);
                hipLaunchKernelGGL(k_wscan_apply<2>, dim3(ntile), dim3(WS_T), 0, c->stream, L, sp_prev, nb_prev, ps,
                                   cs, cw, cx, tsum, ntile, sp_cur, wp_cur, xp_cur, nb);
            }
            hipLaunchKernelGGL(k_lists_advance, dim3(1), dim3(1), 0, c->stream, l, L, nb, sp_cur, wp_cur, xp_cur, ps,
                               cap_s, cap_w, cap_x, limit);
            if (OPT)
                hipLaunchKernelGGL(k_flat_fill<true>, dim3(fgrid), dim3(256), 0, c->stream, l, L, gL, sp_prev, nb_prev,
                                   t.sidx.as<int32_t>(), t.widx.as<int32_t>(), t.xidx.as<int32_t>(), own_prev,
                                   own_cur, ps, bits, words, cs, cw, cx, sp_cur, wp_cur, xp_cur, stL, rectL,
                                   t.nrec_j.as<int2>(), t.nrec_d.as<float4>(), selfpos);
            else
                hipLaunchKernelGGL(k_flat_fill<false>, dim3(fgrid), dim3(256), 0, c->stream, l, L, gL, sp_prev,
                                   nb_prev, t.sidx.as<int32_t>(), t.widx.as<int32_t>(), t.xidx.as<int32_t>(), own_prev,
                                   own_cur, ps, bits, words, cs, cw, cx, sp_cur, wp_cur, xp_cur, stL, rectL,
                                   t.nrec_j.as<int2>(), t.nrec_d.as<float4>(), selfpos);
            FMM2D_TRY(hipGetLastError());
        }
    }
    std::vector<int64_t> h(slot_flag(L) + 1);
    FMM2D_TRY(hipMemcpyAsync(h.data(), ps, sizeof(int64_t) * h.size(), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    *overflow = (int)h[slot_flag(L)];
    t.s_off.assign(h.begin(), h.begin() + (L + 2));
    t.w_off.assign(h.begin() + (L + 2), h.begin() + 2 * (L + 2));
    t.x_off.assign(h.begin() + 2 * (L + 2), h.begin() + 3 * (L + 2));
    if (!OPT) {
        // the flat levels wrote no X row pointers: every X list is empty
        for (int l = K + 1; l <= L; ++l) t.x_off[l + 1] = t.x_off[l];
    }
    t.opt = opt;
    t.relax_nbin = nbin;
    t.relax_k0 = rx ? rx->k0 : 0;
    return hipSuccess;
}

}  // namespace fmm2d
