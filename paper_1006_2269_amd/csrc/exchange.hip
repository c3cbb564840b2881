// Exchanged roles for strongly coupled boxes of very different radii, the
// structural optimisation of Section 4: for a pair (b, c) on the exchanged
// list X_l(b), whose criterion holds once the roles of the radii are
// exchanged (r + theta R <= theta d, disjoint balls),
//
//  * target the smaller box (r_b < r_c): the sources of c become a local
//    expansion about b (P2L), added into B_b before the L2L pass carries it
//    down:  B_0 += sum q_j log|z_j - c_b|,  B_k += -(1/k) sum q_j (s_b / (z_j - c_b))^k;
//  * target the larger box (r_b > r_c): the multipole of c is evaluated at
//    every point z of b (M2P):  phi(z) += Re[A_0 log(z - c_c) + sum_k A_k (s_c / (z - c_c))^k].
//
// Both run in binary64 in every precision mode.  All boxes of a level hold
// floor or ceil of n / 4^l points, so the work per entry is known per level.
//
// P2L work items, one per P2L entry on the deepest levels (from the first
// level whose boxes hold at most LANE_PTS points, or at most LANE_PTS_MANY
// when the level has LANE_ENTRIES P2L entries or more, onwards): one lane per
// item walks the entry's source points and writes the item's partial
// expansion.  On the coarser levels an item is a chunk of one entry's points
// (at most 32 chunks of balanced size, at least PCH points each), one
// wavefront per item, one lane per point, the lanes' sums met in a
// transposing butterfly.  Items are ordered by target box and summed per box
// in item order, and the L2L pass adds that sum into B: results do not
// depend on scheduling.  M2P runs one launch per level: items of 64 points
// of one box (or a whole box of fewer points, its entries dealt to lane
// groups), the box's M2P entries staged in LDS.  Orders above 31
// (p + 1 > 32) take generic kernels with one lane per point.
#include "evaluate.h"
#include "wavesum.h"

namespace fmm2d {
namespace {

constexpr int LANE_PTS = 256;         // boxes of at most this many points: one lane per P2L entry
constexpr int LANE_PTS_MANY = 4096;   // ... or this many, on levels with LANE_ENTRIES entries or more
constexpr int64_t LANE_ENTRIES = 32768;
constexpr int PCH = 512;  // least points per chunk on the other levels
constexpr int XT = 16;    // coefficients per pass (orders above PMAX_FAST - 1)
constexpr int PMAX_FAST = 32;  // orders p + 1 up to this many take the specialised kernels
constexpr int MSPAN = 64;      // X row positions per M2P item (at most; the spans of a row are balanced)
constexpr int MPC = 16;   // leaf points per M2P pass

// Point range [a, e) of box b of level l (its leaves are b 4^(L-l) onwards).
__device__ inline void box_range(const int32_t *__restrict__ stL, int L, int l, int64_t b, int32_t &a, int32_t &e) {
    const int sh = 2 * (L - l);
    a = stL[b << sh];
    e = stL[(b + 1) << sh];
}

// Largest box of level l: ceil(n / 4^l) points.
__host__ __device__ inline int64_t level_box_max(int64_t n, int l) {
    return (n + (int64_t(1) << (2 * l)) - 1) >> (2 * l);
}

// Points per P2L chunk on a wavefront-per-item level: the largest box split
// into at most 32 chunks of at least PCH points, as even as they come.
__host__ __device__ inline int64_t level_chunk(int64_t n, int l) {
    const int64_t m = level_box_max(n, l);
    int64_t k = (m + PCH - 1) / PCH;
    k = k < 1 ? 1 : (k > 32 ? 32 : k);
    return (m + k - 1) / k;
}

// M2P passes over the boxes of level l.  Boxes of M2P_WIDE_PTS points or
// more: passes of 64 points, one per lane (WIDE).  Smaller boxes: passes of
// w points, lane = group * w + point, the entries dealt to m2p_groups(w)
// groups; w = ceil(m / passes) for the number of passes (the least possible,
// ceil(m / 64), up to three more: each pass stages the entries again) that
// fills the most lanes per entry evaluated (m points x groups / passes, m the
// level's largest box), the fewest passes on a tie.  At most 8 groups: the
// groups read different entries' coefficients at once, and 8 entries 272
// bytes apart fall in distinct LDS banks.
constexpr int M2P_WIDE_PTS = 256;
__host__ __device__ inline int m2p_groups(int w) { return 64 / w < 8 ? 64 / w : 8; }
__host__ __device__ inline bool m2p_wide(int64_t n, int l) { return level_box_max(n, l) >= M2P_WIDE_PTS; }
__host__ __device__ inline int m2p_width(int64_t n, int l) {
    const int64_t m = level_box_max(n, l);
    if (m >= M2P_WIDE_PTS) return 64;
    int best_w = 64, best_g = 0, best_np = 1;
    const int np0 = (int)((m + 63) / 64);
    for (int np = np0; np <= np0 + 3; ++np) {
        const int w = (int)((m + np - 1) / np);
        const int ng = m2p_groups(w);
        if ((int64_t)ng * best_np > (int64_t)best_g * np) {  // more lanes per pass and entry
            best_w = w;
            best_g = ng;
            best_np = np;
        }
    }
    return best_w;
}

// The pass width of every level, for the kernels (a kernel argument: no
// division in the kernels).
struct M2PWidths {
    int32_t w[FMM2D_MAX_LEVELS + 1];
};
M2PWidths m2p_widths(int64_t n, int L) {
    M2PWidths mw{};
    for (int l = 0; l <= L && l <= FMM2D_MAX_LEVELS; ++l) mw.w[l] = m2p_width(n, l);
    return mw;
}

// Work items per global box g, one wavefront per box (lanes over the X row,
// 64 entries at a time, item positions by a wave prefix sum in row order).
// P2L (the entries of X(g) whose source box is the larger): int4 (target
// box, row position, row position + 1, first point of the chunk or -1 for
// the whole entry); levels from `lane_level` on take whole entries.  M2P
// (when X(g) holds an entry whose source box is the smaller): int4 (g, first
// point, row span start, end): the points in passes of m2p_width(n, l),
// times the row in balanced spans of at most MSPAN positions (point pass
// major), so that no item holds more than MSPAN entries however long the
// row.
template <bool FILL>
__global__ void __launch_bounds__(256) k_x_items(int L, int64_t n, int64_t nbox, int lane_level,
                                                 const int32_t *__restrict__ xptr_all,
                                                 const int32_t *__restrict__ xidx, const int64_t *__restrict__ xoff,
                                                 const double4 *__restrict__ geom, const int32_t *__restrict__ stL,
                                                 int32_t *__restrict__ cnt, int32_t *__restrict__ mcnt,
                                                 const int32_t *__restrict__ itemoff,
                                                 const int32_t *__restrict__ mitemoff, int4 *__restrict__ items,
                                                 int4 *__restrict__ mitems, M2PWidths mw) {
    const int64_t g = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (g >= nbox) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int l = level_of(g);
    int32_t t0 = 0, t1 = 0;
    const int64_t b = g - level_offset(l);
    const int32_t *ptr = xptr_all + ptr_offset(l);
    if (l >= 1) {
        t0 = ptr[b];
        t1 = ptr[b + 1];
    }
    if (t0 == t1) {  // no exchanged entry (and level 0)
        if (!FILL && lane == 0) cnt[g] = mcnt[g] = 0;
        return;
    }
    const int32_t *row = xidx + xoff[l];
    const double rb = geom[g].z;
    const bool whole = l >= lane_level;
    const int32_t chunk = (int32_t)level_chunk(n, l);
    int32_t base = FILL ? itemoff[g] : 0;
    bool m2p = false;
    for (int32_t tb = t0; tb < t1; tb += 64) {
        const int32_t t = tb + lane;
        int32_t k = 0, c = 0, a = 0, e = 0;
        if (t < t1) {
            c = row[t];
            const double rc = geom[level_offset(l) + c].z;
            if (rb < rc) {  // P2L entry
                if (whole) {
                    k = 1;
                } else {
                    box_range(stL, L, l, c, a, e);
                    k = (e - a + chunk - 1) / chunk;
                }
            } else {
                m2p = m2p || rb > rc;
            }
        }
        const int32_t incl = wave_incl_scan(k);
        if (FILL && k > 0) {
            int32_t pos = base + incl - k;
            if (whole) {
                items[pos] = make_int4((int32_t)g, t, t + 1, -1);
            } else {
                for (int32_t j = a; j < e; j += chunk) items[pos++] = make_int4((int32_t)g, t, t + 1, j);
            }
        }
        base += __shfl(incl, 63, 64);
    }
    m2p = __ballot(m2p) != 0;
    int32_t km = 0;
    if (m2p) {
        int32_t a, e;
        box_range(stL, L, l, b, a, e);
        const int32_t step = mw.w[l];
        const int32_t npc = (e - a + step - 1) / step;
        const int32_t nsp = (t1 - t0 + MSPAN - 1) / MSPAN, span = (t1 - t0 + nsp - 1) / nsp;
        km = npc * nsp;
        if (FILL) {
            const int32_t m0 = mitemoff[g];
            for (int32_t q = lane; q < km; q += 64) {
                const int32_t pc = q / nsp, s0 = t0 + (q - pc * nsp) * span;
                mitems[m0 + q] = make_int4((int32_t)g, a + pc * step, s0, s0 + span < t1 ? s0 + span : t1);
            }
        }
    }
    if (!FILL && lane == 0) {
        cnt[g] = base;
        mcnt[g] = km;
    }
}

// The scaled division and hypot for |w|^2 <= 2^-960 (where |w|^2 could
// underflow), kept out of line: no input of ordinary scale reaches it.  Both
// results come back by value (a reference argument of an out-of-line call
// would keep log|w| in scratch memory on the common path too).
struct RhoLog {
    cd rho;
    double logw;
};
__device__ __attribute__((noinline)) RhoLog recip_tiny(double s, double dx, double dy) {
    return RhoLog{cdiv(cd{s, 0.0}, cd{dx, dy}), log(hypot(dx, dy))};
}

// rho = s / w for w = (dx, dy) != 0, and log|w|.
__device__ inline cd recip_scaled(double s, double dx, double dy, double &logw) {
    const double d2 = dx * dx + dy * dy;
    if (d2 > 0x1p-960) {
        logw = 0.5 * log_pos(d2);
        // 1 / d2 by the hardware reciprocal and two Newton steps (each
        // squares the relative error; within an ulp or two of the quotient)
        double r = __builtin_amdgcn_rcp(d2);
        r = fma(r, fma(-d2, r, 1.0), r);
        r = fma(r, fma(-d2, r, 1.0), r);
        const double inv = s * r;
        return cd{dx * inv, -dy * inv};
    }
    const RhoLog t = recip_tiny(s, dx, dy);
    logw = t.logw;
    return t.rho;
}

// P2L sums of one source point about the target (gb): s[0] += q log|w|,
// s[k] += q rho^k (k >= 1); the factors -1/k are applied once per item.
template <int P1>
__device__ inline void p2l_sums(double x, double y, double q, double4 gb, cd *s) {
    double lw;
    const cd rho = recip_scaled(gb.w, x - gb.x, y - gb.y, lw);
    s[0].re = fma(q, lw, s[0].re);
    cd pw = rho;
#pragma unroll
    for (int k = 1; k < P1; ++k) {
        s[k].re = fma(q, pw.re, s[k].re);
        s[k].im = fma(q, pw.im, s[k].im);
        if (k + 1 < P1) pw = cmul(pw, rho);
    }
}

// Coefficient k of a P2L partial: the sums times -1/k (k >= 1).
__device__ inline double p2l_coef(double v, int k) { return k == 0 ? v : -v / (double)k; }

// Wavefront-per-item P2L (chunks of one entry), orders p + 1 <= 32: items
// [0, *wave_end).
template <int P1>
__global__ void __launch_bounds__(256) k_p2l(int L, int64_t n, const int4 *__restrict__ items,
                                             const int32_t *__restrict__ wave_end, const int32_t *__restrict__ xidx,
                                             const int64_t *__restrict__ xoff, const double4 *__restrict__ geom,
                                             const int32_t *__restrict__ stL, const double *__restrict__ px,
                                             const double *__restrict__ py, const double *__restrict__ qs,
                                             double *__restrict__ xpart) {
    static_assert(P1 >= 2 && P1 <= PMAX_FAST, "two passes of at most 32 values");
    const int64_t it = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (it >= *wave_end) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int4 w = items[it];
    const double4 gb = geom[w.x];
    const int l = level_of(w.x);
    const int32_t *row = xidx + xoff[l];
    cd s[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) s[k] = cd{0.0, 0.0};
    int32_t a, e;
    box_range(stL, L, l, row[w.y], a, e);
    const int32_t ch = (int32_t)level_chunk(n, l);
    const int32_t j1 = e < w.w + ch ? e : w.w + ch;
    // four points per lane at a time, their loads issued together
    int32_t j = w.w + lane;
    for (; j + 192 < j1; j += 256) {
        double bx[4], by[4], bq[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            bx[u] = px[j + 64 * u];
            by[u] = py[j + 64 * u];
            bq[u] = qs[j + 64 * u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) p2l_sums<P1>(bx[u], by[u], bq[u], gb, s);
    }
    for (; j < j1; j += 64) p2l_sums<P1>(px[j], py[j], qs[j], gb, s);
    // coefficients 16 at a time: lane i receives the total of value i / 2 of
    // the pass, coefficient k0 + i / 4, part (i / 2) % 2
#pragma unroll
    for (int k0 = 0; k0 < P1; k0 += 16) {
        double v[32];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            v[2 * k] = k0 + k < P1 ? s[k0 + k].re : 0.0;
            v[2 * k + 1] = k0 + k < P1 ? s[k0 + k].im : 0.0;
        }
        const double tot = wave_transpose_sum<32>(v, lane);
        const int vi = lane / 2, k = k0 + vi / 2;
        if ((lane & 1) == 0 && k < P1) xpart[it * 2 * P1 + 2 * k0 + vi] = p2l_coef(tot, k);
    }
}

// Lane-per-item P2L (whole entries), orders p + 1 <= 32: items
// [*wave_end, *nitem).  Each lane walks its entry's source points in bursts
// of 8: the burst's loads are issued together (consecutive addresses of one
// lane, so a cache line is fetched once per burst rather than once per
// point while 64 lanes stream 64 boxes), then its points are summed.
template <int P1>
__global__ void __launch_bounds__(256) k_p2l_lane(int L, const int4 *__restrict__ items,
                                                  const int32_t *__restrict__ wave_end,
                                                  const int32_t *__restrict__ nitem, const int32_t *__restrict__ xidx,
                                                  const int64_t *__restrict__ xoff, const double4 *__restrict__ geom,
                                                  const int32_t *__restrict__ stL, const double *__restrict__ px,
                                                  const double *__restrict__ py, const double *__restrict__ qs,
                                                  double *__restrict__ xpart) {
    const int64_t it = *wave_end + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= *nitem) return;
    const int4 w = items[it];
    const double4 gb = geom[w.x];
    const int l = level_of(w.x);
    int32_t a, e;
    box_range(stL, L, l, xidx[xoff[l] + w.y], a, e);
    cd s[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) s[k] = cd{0.0, 0.0};
    constexpr int BURST = 8;
    int32_t j = a;
    for (; j + BURST <= e; j += BURST) {
        double bx[BURST], by[BURST], bq[BURST];
#pragma unroll
        for (int u = 0; u < BURST; ++u) {
            bx[u] = px[j + u];
            by[u] = py[j + u];
            bq[u] = qs[j + u];
        }
#pragma unroll
        for (int u = 0; u < BURST; ++u) p2l_sums<P1>(bx[u], by[u], bq[u], gb, s);
    }
    for (; j < e; ++j) p2l_sums<P1>(px[j], py[j], qs[j], gb, s);
    double *out = xpart + it * 2 * P1;
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        out[2 * k] = p2l_coef(s[k].re, k);
        out[2 * k + 1] = p2l_coef(s[k].im, k);
    }
}

// The same for orders p + 1 > 32: XT coefficients per pass, one lane per
// point (entries of an item taken one after the other).
__device__ inline void p2l_point(double px_, double py_, double q, double4 gb, int k0, int p, double *ar,
                                 double *ai) {
    double lw;
    const cd rho = recip_scaled(gb.w, px_ - gb.x, py_ - gb.y, lw);
    cd pw{1.0, 0.0};
    for (int k = 0; k < k0; ++k) pw = cmul(pw, rho);  // rho^k0
#pragma unroll
    for (int k = 0; k < XT; ++k) {
        const int kk = k0 + k;
        if (kk <= p) {
            if (kk == 0) {
                ar[0] = fma(q, lw, ar[0]);
            } else {
                ar[k] = fma(q, pw.re, ar[k]);
                ai[k] = fma(q, pw.im, ai[k]);
            }
        }
        pw = cmul(pw, rho);
    }
}

__global__ void __launch_bounds__(256) k_p2l_gen(int p, int L, int64_t n, const int4 *__restrict__ items,
                                                 const int32_t *__restrict__ nitem, const int32_t *__restrict__ xidx,
                                                 const int64_t *__restrict__ xoff, const double4 *__restrict__ geom,
                                                 const int32_t *__restrict__ stL, const double *__restrict__ px,
                                                 const double *__restrict__ py, const double *__restrict__ qs,
                                                 double *__restrict__ xpart) {
    const int64_t it = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (it >= *nitem) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int4 w = items[it];
    const double4 gb = geom[w.x];
    const int l = level_of(w.x);
    const int32_t *row = xidx + xoff[l];
    const int P1 = p + 1;
    for (int k0 = 0; k0 < P1; k0 += XT) {
        double ar[XT], ai[XT];
#pragma unroll
        for (int k = 0; k < XT; ++k) {
            ar[k] = 0.0;
            ai[k] = 0.0;
        }
        for (int32_t t = w.y; t < w.z; ++t) {
            const int32_t c = row[t];
            if (!(gb.z < geom[level_offset(l) + c].z)) continue;
            int32_t a, e;
            box_range(stL, L, l, c, a, e);
            if (w.w >= 0) {
                const int32_t ch = (int32_t)level_chunk(n, l);
                a = w.w;
                e = e < w.w + ch ? e : w.w + ch;
            }
            for (int32_t j = a + lane; j < e; j += 64) p2l_point(px[j], py[j], qs[j], gb, k0, p, ar, ai);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int k = 0; k < XT; ++k) {
                ar[k] += __shfl_xor(ar[k], off, 64);
                ai[k] += __shfl_xor(ai[k], off, 64);
            }
        }
#pragma unroll
        for (int k = 0; k < XT; ++k) {
            const int kk = k0 + k;
            if (lane == k && kk <= p) {
                xpart[(it * P1 + kk) * 2] = p2l_coef(ar[k], kk);
                xpart[(it * P1 + kk) * 2 + 1] = p2l_coef(ai[k], kk);
            }
        }
    }
}

// Per target box with items: the sum of its items' partial expansions, one
// wavefront per box.  Lanes are G = 64 / (p + 1) groups of one lane per
// coefficient (one group above order 32); group q takes the box's items q, q
// + G, ... in order, four loads in flight, and group 0 adds the groups' sums
// in group order.
__global__ void __launch_bounds__(256) k_x_reduce(int p, int64_t nbox, const int32_t *__restrict__ itemoff,
                                                  const cd *__restrict__ xpart, cd *__restrict__ xsum) {
    const int64_t g = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (g >= nbox) return;
    const int32_t i0 = itemoff[g], i1 = itemoff[g + 1];
    if (i0 == i1) return;  // uniform: a box without P2L entries
    const int lane = threadIdx.x % 64, P1 = p + 1;
    const int G = P1 <= 32 ? 64 / P1 : 1;
    const int grp = lane / P1, k = lane - grp * P1;  // lanes of group G and above idle
    cd acc{0.0, 0.0};
    if (grp < G) {
        int32_t it = i0 + grp;
        for (; it + 3 * G < i1; it += 4 * G) {
            const cd v0 = xpart[(int64_t)it * P1 + k], v1 = xpart[(int64_t)(it + G) * P1 + k];
            const cd v2 = xpart[(int64_t)(it + 2 * G) * P1 + k], v3 = xpart[(int64_t)(it + 3 * G) * P1 + k];
            acc = cadd(cadd(cadd(cadd(acc, v0), v1), v2), v3);
        }
        for (; it < i1; it += G) acc = cadd(acc, xpart[(int64_t)it * P1 + k]);
    }
    cd tot = acc;
    for (int q = 1; q < G; ++q) {
        const int src = lane + q * P1 < 64 ? lane + q * P1 : lane;
        tot.re += __shfl(acc.re, src, 64);
        tot.im += __shfl(acc.im, src, 64);
    }
    if (grp == 0) xsum[g * P1 + k] = tot;
}

// M2P, orders p + 1 <= 32: one wavefront per item, the items of every level
// in one launch (those of the WIDE levels, or those of the others).  The
// item's row span is taken 32 positions at a time: its M2P entries (the
// target box the larger) are compacted by ballot, their centres, scales and
// multipoles staged in the wavefront's LDS slice by coalesced loads, then
// evaluated from there (same-address reads within a group, served by
// broadcast; 16 entries at a time above order 16).  WIDE: the item's 64
// points one per lane, every lane taking the entries in row order.
// Otherwise (passes of mp points): lane = group * mp + point, the compacted
// entries dealt to the groups in turn, group 0 adding the others' sums at its
// point in group order.  Each item writes its sums at its points to its own
// row of mpart (lane = point offset); the leaf pass adds them per point.
template <int P1>
constexpr int m_stage() { return P1 <= 16 ? 32 : 16; }  // entries staged at once (LDS of 32 KB per block)
template <int P1, bool WIDE>
__global__ void __launch_bounds__(256) k_m2p(int L, int64_t n, const int4 *__restrict__ items,
                                             const int32_t *__restrict__ first, const int32_t *__restrict__ end,
                                             const int32_t *__restrict__ xidx, const int64_t *__restrict__ xoff,
                                             const double4 *__restrict__ geom, const int32_t *__restrict__ stL,
                                             const cd *__restrict__ A, const double *__restrict__ px,
                                             const double *__restrict__ py, double *__restrict__ mpart,
                                             M2PWidths mw) {
    constexpr int MSTAGE = m_stage<P1>();
    __shared__ cd s_a[4][MSTAGE * P1];
    __shared__ double s_g[4][MSTAGE][3];
    __shared__ int64_t s_c[4][MSTAGE];
    const int32_t it = __builtin_amdgcn_readfirstlane(*first + (int32_t)(blockIdx.x * 4 + threadIdx.x / 64));
    if (it >= *end) return;  // uniform per wavefront
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int4 w = items[it];
    const int l = level_of(w.x);
    const int64_t b = w.x - level_offset(l);
    int32_t a, e;
    box_range(stL, L, l, b, a, e);
    const int mp = WIDE ? 64 : mw.w[l];
    const int ng = WIDE ? 1 : m2p_groups(mp);
    const int grp = WIDE ? 0 : lane / mp;  // lanes of group ng and above idle
    const int32_t i = w.y + (WIDE ? lane : lane % mp);
    const bool act = i < e && i < w.y + mp && grp < ng;
    const int32_t ii = act ? i : a;  // lanes past the box evaluate at its first point (finite, not written)
    const double zx = px[ii], zy = py[ii];
    const double rb = geom[w.x].z;
    const int32_t *row = xidx + xoff[l];
    const int32_t t1 = w.w;
    cd *sa = s_a[wv];
    double acc = 0.0;
    int qs = WIDE ? 0 : grp;  // this group's first compacted entry of the stage
    for (int32_t tb = w.z; tb < t1; tb += MSTAGE) {
        bool ok = false;
        int64_t cg = 0;
        double4 gc = make_double4(0.0, 0.0, 0.0, 1.0);
        if (lane < MSTAGE && tb + lane < t1) {
            cg = level_offset(l) + row[tb + lane];
            gc = geom[cg];
            ok = rb > gc.z;  // M2P entry (else P2L, handled by the P2L pass)
        }
        const uint64_t m = __ballot(ok);
        const int k = (int)__popcll(m);
        if (ok) {
            const int q = (int)popc_below(m);
            s_g[wv][q][0] = gc.x;
            s_g[wv][q][1] = gc.y;
            s_g[wv][q][2] = gc.w;
            s_c[wv][q] = cg;
        }
        __builtin_amdgcn_wave_barrier();
        for (int idx = lane; idx < k * P1; idx += 64) {
            const int q = idx / P1;
            sa[idx] = A[s_c[wv][q] * P1 + (idx - q * P1)];
        }
        __builtin_amdgcn_wave_barrier();
        int q = qs;
        for (; q < k; q += ng) {
            const cd *Ac = sa + q * P1;
            double lw;
            const cd rho = recip_scaled(s_g[wv][q][2], zx - s_g[wv][q][0], zy - s_g[wv][q][1], lw);
            cd sacc = Ac[P1 - 1];
#pragma unroll
            for (int r = P1 - 2; r >= 1; --r) sacc = cfma(sacc, rho, Ac[r]);
            acc += fma(sacc.re, rho.re, fma(-sacc.im, rho.im, Ac[0].re * lw));  // Re(sacc rho) + A_0 log|w|
        }
        qs = q - k;  // the entries continue in the next stage
        __builtin_amdgcn_wave_barrier();  // the slice is rewritten by the next stage
    }
    if (!WIDE) {
        // group 0's lanes add the other groups' sums at their point, in group order
        double tot = acc;
        for (int gq = 1; gq < ng; ++gq) tot += __shfl(acc, lane + gq * mp < 64 ? lane + gq * mp : lane, 64);
        acc = tot;
    }
    if (grp == 0 && act) mpart[(int64_t)it * 64 + lane] = acc;
}

// M2P for orders p + 1 > 32: one lane per point of the leaf.
__global__ void __launch_bounds__(256) k_m2p_gen(int p, int L, int64_t nleaf, const int32_t *__restrict__ stL,
                                                 const int32_t *__restrict__ xptr_all,
                                                 const int32_t *__restrict__ xidx, const int64_t *__restrict__ xoff,
                                                 const double4 *__restrict__ geom, const cd *__restrict__ A,
                                                 const double *__restrict__ px, const double *__restrict__ py,
                                                 const int32_t *__restrict__ perm, double *__restrict__ phi) {
    const int64_t leaf = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (leaf >= nleaf) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int P1 = p + 1;
    const int32_t a = stL[leaf], e = stL[leaf + 1];
    for (int32_t base = a; base < e; base += 64) {
        const int32_t i = base + lane;
        const bool act = i < e;
        const double zx = act ? px[i] : 0.0, zy = act ? py[i] : 0.0;
        double acc = 0.0;
        for (int l = 1; l <= L; ++l) {
            const int64_t b = leaf >> (2 * (L - l));
            const double4 gb = geom[level_offset(l) + b];
            const int32_t *ptr = xptr_all + ptr_offset(l);
            const int32_t *row = xidx + xoff[l];
            for (int32_t t = ptr[b]; t < ptr[b + 1]; ++t) {
                const int64_t cg = level_offset(l) + row[t];
                const double4 gc = geom[cg];
                if (!(gb.z > gc.z)) continue;  // P2L entry
                const cd *Ac = A + cg * P1;
                // inactive lanes evaluate at a point one scale away (finite)
                double lw;
                const cd rho = recip_scaled(gc.w, act ? zx - gc.x : gc.w, act ? zy - gc.y : 0.0, lw);
                cd s = Ac[p];
                for (int k = p - 1; k >= 1; --k) s = cfma(s, rho, Ac[k]);
                acc += fma(s.re, rho.re, fma(-s.im, rho.im, Ac[0].re * lw));
            }
        }
        if (act) phi[perm[i]] += acc;
    }
}

}  // namespace

hipError_t exchange_schedule(fmm2d_ctx *c) {
    TreeState &t = c->tree;
    t.x_ready = false;
    const int L = t.L;
    if (!(t.opt & (FMM2D_OPT_SWAP_FINEST | FMM2D_OPT_SWAP_ALL)) || L < 1) return hipSuccess;
    if (t.x_off[L + 1] == t.x_off[1]) return hipSuccess;  // no exchanged pair
    const int64_t nbox = level_offset(L + 1);
    // whole entries (one lane each) from the first level of a run down to
    // the finest in which every level has small boxes, or boxes of moderate
    // size and many entries; chunks above
    int lane_level = L + 1;
    for (int l = L; l >= 1; --l) {
        const int64_t maxpts = level_box_max(t.n, l), nx = t.x_off[l + 1] - t.x_off[l];
        if (maxpts <= LANE_PTS || (maxpts <= LANE_PTS_MANY && nx / 2 >= LANE_ENTRIES))
            lane_level = l;
        else
            break;
    }
    // at most one item per entry on the lane levels, the chunks of one entry
    // on the others
    int64_t bw = 0, bl = 0;
    for (int l = 1; l <= L; ++l) {
        const int64_t maxpts = level_box_max(t.n, l), ch = level_chunk(t.n, l), nx = t.x_off[l + 1] - t.x_off[l];
        if (l >= lane_level)
            bl += nx;
        else
            bw += nx * ((maxpts + ch - 1) / ch);
    }
    const int64_t bound = bw + bl;
    FMM2D_TRY(c->scr.segcnt.ensure(sizeof(int32_t) * nbox));
    FMM2D_TRY(t.x_itemoff.ensure(sizeof(int32_t) * (nbox + 1)));
    FMM2D_TRY(t.x_items.ensure(sizeof(int4) * (bound > 0 ? bound : 1)));
    const int32_t *xptr = t.xptr.as<int32_t>(), *xidx = t.xidx.as<int32_t>();
    const int64_t *xoff = t.pool_state.as<int64_t>() + 2 * (L + 2);  // X pool offset of each level
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const double4 *geom = t.geom.as<double4>();
    t.x_bound_wave = bw;
    t.x_bound_lane = bl;
    t.x_lane_level = lane_level;
    // M2P items: at most min(4^l, X entries) boxes of level l have some, each
    // with its point passes (ceil(points / 64) on levels of width 64, one on
    // the others) times ceil(row / MSPAN) spans; the spans of a level's rows
    // number at most boxes + entries / MSPAN.  Levels of width 64 come first.
    int wl = L + 1;
    for (int l = 1; l <= L; ++l)
        if (!m2p_wide(t.n, l)) {
            wl = l;
            break;
        }
    int64_t mw = 0, mn = 0;
    for (int l = 1; l <= L; ++l) {
        const int64_t nx = t.x_off[l + 1] - t.x_off[l], nb = int64_t(1) << (2 * l);
        const int64_t boxes = nx < nb ? nx : nb;
        const int64_t w = m2p_width(t.n, l), npc = (level_box_max(t.n, l) + w - 1) / w;
        (l < wl ? mw : mn) += npc * (boxes + nx / MSPAN);
    }
    if (mw + mn > INT32_MAX) return hipErrorInvalidValue;  // item indices are int32
    t.m_wide_level = wl;
    FMM2D_TRY(c->scr.mcnt.ensure(sizeof(int32_t) * nbox));
    FMM2D_TRY(t.m_itemoff.ensure(sizeof(int32_t) * (nbox + 1)));
    int32_t *cnts[2] = {c->scr.segcnt.as<int32_t>(), c->scr.mcnt.as<int32_t>()};
    int32_t *offs[2] = {t.x_itemoff.as<int32_t>(), t.m_itemoff.as<int32_t>()};
    const M2PWidths widths = m2p_widths(t.n, L);
    hipLaunchKernelGGL(k_x_items<false>, dim3(grid_for(nbox, 4)), dim3(256), 0, c->stream, L, t.n, nbox,
                       lane_level, xptr, xidx, xoff, geom, stL, cnts[0], cnts[1], nullptr, nullptr, nullptr, nullptr,
                       widths);
    FMM2D_TRY(hipGetLastError());
    const int32_t *cin[2] = {cnts[0], cnts[1]};
    FMM2D_TRY(scan_exclusive_n(c, 2, cin, nbox, offs));
    // the M2P item counts (before the narrower levels, and in all), read back
    // so that the items and their partial sums (512 bytes each) are sized to
    // the count rather than to the bound
    int32_t hm[2] = {0, 0};
    FMM2D_TRY(hipMemcpyAsync(&hm[0], offs[1] + level_offset(wl), sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipMemcpyAsync(&hm[1], offs[1] + nbox, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    t.m_bound_wide = hm[0];
    t.m_bound_narrow = hm[1] - hm[0];
    FMM2D_TRY(t.m_items.ensure(sizeof(int4) * (hm[1] > 0 ? hm[1] : 1)));
    hipLaunchKernelGGL(k_x_items<true>, dim3(grid_for(nbox, 4)), dim3(256), 0, c->stream, L, t.n, nbox,
                       lane_level, xptr, xidx, xoff, geom, stL, nullptr, nullptr, offs[0], offs[1],
                       t.x_items.as<int4>(), t.m_items.as<int4>(), widths);
    FMM2D_TRY(hipGetLastError());
    t.x_ready = true;
    return hipSuccess;
}

const int32_t *exchange_item_offsets(fmm2d_ctx *c) {
    return c->tree.x_ready ? c->tree.x_itemoff.as<int32_t>() : nullptr;
}

hipError_t p2l_all(fmm2d_ctx *c, int p) {
    TreeState &t = c->tree;
    if (!t.x_ready) return hipSuccess;
    EvalState &e = c->ev;
    const int64_t bound = t.x_bound_wave + t.x_bound_lane > 0 ? t.x_bound_wave + t.x_bound_lane : 1;
    const int64_t nbox = level_offset(t.L + 1);
    FMM2D_TRY(e.xpart.ensure(sizeof(cd) * bound * (p + 1)));
    FMM2D_TRY(e.xsum.ensure(sizeof(cd) * nbox * (p + 1)));
    const int32_t *itemoff = t.x_itemoff.as<int32_t>();
    const int32_t *nitem = itemoff + nbox;
    // items of the levels before the lane levels come first
    const int32_t *wave_end = itemoff + level_offset(t.x_lane_level);
    const int64_t *xoff = t.pool_state.as<int64_t>() + 2 * (t.L + 2);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * t.L);
    double *xpart = reinterpret_cast<double *>(e.xpart.as<cd>());
    const int4 *items = t.x_items.as<int4>();
    const int32_t *xidx = t.xidx.as<int32_t>();
    const double4 *geom = t.geom.as<double4>();
    const double *px = t.px.as<double>(), *py = t.py.as<double>(), *qs = e.qs.as<double>();
    const dim3 block(256);
    {
    PhaseScope kernel_scope(c, PH_P2L_KERNEL);  // the P2L kernels alone
    switch (p + 1) {
#define FMM2D_P2L(P1)                                                                                             \
    case P1:                                                                                                      \
        if (t.x_bound_wave > 0)                                                                                   \
            hipLaunchKernelGGL(k_p2l<P1>, dim3(grid_for(t.x_bound_wave, 4)), block, 0, c->stream, t.L, t.n,      \
                               items, wave_end, xidx, xoff, geom, stL, px, py, qs, xpart);                        \
        if (t.x_bound_lane > 0)                                                                                   \
            hipLaunchKernelGGL(k_p2l_lane<P1>, dim3(grid_for(t.x_bound_lane, 256)), block, 0, c->stream, t.L,    \
                               items, wave_end, nitem, xidx, xoff, geom, stL, px, py, qs, xpart);                 \
        break;
        FMM2D_P2L(2) FMM2D_P2L(3) FMM2D_P2L(4) FMM2D_P2L(5) FMM2D_P2L(6) FMM2D_P2L(7) FMM2D_P2L(8) FMM2D_P2L(9)
        FMM2D_P2L(10) FMM2D_P2L(11) FMM2D_P2L(12) FMM2D_P2L(13) FMM2D_P2L(14) FMM2D_P2L(15) FMM2D_P2L(16)
        FMM2D_P2L(17) FMM2D_P2L(18) FMM2D_P2L(19) FMM2D_P2L(20) FMM2D_P2L(21) FMM2D_P2L(22) FMM2D_P2L(23)
        FMM2D_P2L(24) FMM2D_P2L(25) FMM2D_P2L(26) FMM2D_P2L(27) FMM2D_P2L(28) FMM2D_P2L(29) FMM2D_P2L(30)
        FMM2D_P2L(31) FMM2D_P2L(32)
#undef FMM2D_P2L
        default:
            hipLaunchKernelGGL(k_p2l_gen, dim3(grid_for(bound, 4)), block, 0, c->stream, p, t.L, t.n, items, nitem,
                               xidx, xoff, geom, stL, px, py, qs, xpart);
    }
    }
    FMM2D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_x_reduce, dim3(grid_for(nbox, 4)), dim3(256), 0, c->stream, p, nbox, itemoff, e.xpart.as<cd>(),
                       e.xsum.as<cd>());
    return hipGetLastError();
}

hipError_t m2p_partials(fmm2d_ctx *c, int p) {
    TreeState &t = c->tree;
    c->ev.m2p = M2PSum{};
    if (!t.x_ready || p + 1 > PMAX_FAST) return hipSuccess;
    const int L = t.L;
    const dim3 block(256);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const int64_t *xoff = t.pool_state.as<int64_t>() + 2 * (L + 2);
    const int32_t *xidx = t.xidx.as<int32_t>();
    const double4 *geom = t.geom.as<double4>();
    const cd *A = c->ev.A.as<cd>();
    const double *px = t.px.as<double>(), *py = t.py.as<double>();
    PhaseScope kernel_scope(c, PH_M2P_KERNEL);  // the M2P kernels alone
    const int4 *items = t.m_items.as<int4>();
    const int64_t nbox = level_offset(L + 1), mb = t.m_bound_wide + t.m_bound_narrow;
    FMM2D_TRY(c->ev.mpart.ensure(sizeof(double) * 64 * (mb > 0 ? mb : 1)));
    double *mpart = c->ev.mpart.as<double>();
    const int32_t *off = t.m_itemoff.as<int32_t>();
    const M2PWidths widths = m2p_widths(t.n, L);
    for (int pass = 0; pass < 2; ++pass) {
        // the items of the levels of width 64, then those of the others
        const bool wide = pass == 0;
        const int64_t bound = wide ? t.m_bound_wide : t.m_bound_narrow;
        if (bound == 0) continue;
        const int32_t *first = off + (wide ? 0 : level_offset(t.m_wide_level));
        const int32_t *end = off + (wide ? level_offset(t.m_wide_level) : nbox);
        const dim3 grid(grid_for(bound, 4));
        switch ((p + 1) * 2 + wide) {
#define FMM2D_M2P(P1)                                                                                             \
    case 2 * P1:                                                                                                  \
        hipLaunchKernelGGL((k_m2p<P1, false>), grid, block, 0, c->stream, L, t.n, items, first, end, xidx, xoff,  \
                           geom, stL, A, px, py, mpart, widths);                                                  \
        break;                                                                                                    \
    case 2 * P1 + 1:                                                                                              \
        hipLaunchKernelGGL((k_m2p<P1, true>), grid, block, 0, c->stream, L, t.n, items, first, end, xidx, xoff,   \
                           geom, stL, A, px, py, mpart, widths);                                                  \
        break;
            FMM2D_M2P(2) FMM2D_M2P(3) FMM2D_M2P(4) FMM2D_M2P(5) FMM2D_M2P(6) FMM2D_M2P(7) FMM2D_M2P(8)
            FMM2D_M2P(9) FMM2D_M2P(10) FMM2D_M2P(11) FMM2D_M2P(12) FMM2D_M2P(13) FMM2D_M2P(14) FMM2D_M2P(15)
            FMM2D_M2P(16) FMM2D_M2P(17) FMM2D_M2P(18) FMM2D_M2P(19) FMM2D_M2P(20) FMM2D_M2P(21) FMM2D_M2P(22)
            FMM2D_M2P(23) FMM2D_M2P(24) FMM2D_M2P(25) FMM2D_M2P(26) FMM2D_M2P(27) FMM2D_M2P(28) FMM2D_M2P(29)
            FMM2D_M2P(30) FMM2D_M2P(31) FMM2D_M2P(32)
#undef FMM2D_M2P
            default:
                return hipErrorInvalidValue;
        }
        FMM2D_TRY(hipGetLastError());
    }
    M2PSum ms;
    ms.itemoff = off;
    ms.mpart = mpart;
    for (int l = 0; l <= FMM2D_MAX_LEVELS; ++l) ms.w[l] = widths.w[l];
    c->ev.m2p = ms;
    return hipSuccess;
}

hipError_t m2p_direct(fmm2d_ctx *c, int p, double *phi) {
    TreeState &t = c->tree;
    if (!t.x_ready || p + 1 <= PMAX_FAST) return hipSuccess;
    const int L = t.L;
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const int64_t *xoff = t.pool_state.as<int64_t>() + 2 * (L + 2);
    const int32_t *xptr = t.xptr.as<int32_t>(), *xidx = t.xidx.as<int32_t>(), *perm = t.perm.as<int32_t>();
    PhaseScope kernel_scope(c, PH_M2P_KERNEL);
    const int64_t nleaf = int64_t(1) << (2 * L);
    hipLaunchKernelGGL(k_m2p_gen, dim3(grid_for(nleaf, 4)), dim3(256), 0, c->stream, p, L, nleaf, stL, xptr, xidx,
                       xoff, t.geom.as<double4>(), c->ev.A.as<cd>(), t.px.as<double>(), t.py.as<double>(), perm, phi);
    return hipGetLastError();
}

}  // namespace fmm2d
