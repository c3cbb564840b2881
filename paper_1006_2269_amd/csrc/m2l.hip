// M2L along the weak lists (the far-to-local shift of Section 4), done as one
// constant matrix applied to every pair's pre-scaled multipole vector, with
// pre- and post-scaling by the pair's geometry.
//
// For a weak pair (target b, source c), z0 = c_c - c_b, rho_s = s_c / z0,
// rho_t = s_b / z0, u_k = A_k rho_s^k, the local coefficients of b gain
//   B_0 += A_0 log|z0| + sum_{k>=1} M_0k u_k,   B_l += rho_t^l sum_k M_lk u_k,
// with the constant real matrix M_00 = 0, M_0k = (-1)^k, M_l0 = -1/l and
// M_lk = (-1)^k C(l+k-1, k-1) (the multipole series re-expanded in powers of
// (z - c_b)/z0).  Exact power-of-two rescaling, M^_lk = M_lk / 2^(l+k),
// u'_k = 2^k u_k, T'_l = 2^l rho_t^l, keeps every matrix entry below one.
//
// One wavefront per segment of a target box's weak list (at most M2L_SEG
// pairs, so heavy-tailed lists do not serialise; the L2L pass adds the
// segments' sums into B in order).  The segments of all levels run in one
// launch; each finds its level from its box's global id.  This kernel (p + 1
// > 16) walks a segment in chunks of 16 pairs.
// Four lanes per pair build that pair's power tables in binary64 (binary
// exponentiation to the lane's first power, then successive products) into
// LDS, while the next chunk's geometry and coefficients are being loaded.  The 16x16x4 matrix instruction multiplies a 16-row block (8 pairs x
// real/imaginary part) of u' by M^T, which every lane keeps in registers;
// each lane then post-scales its output elements by T' and accumulates its
// coefficient l.  A cross-lane reduction adds the box's total into B.
//
// Variants: the product in FP32 (f32 matrix instruction), in three BF16
// products (bf16 matrix instruction), or binary64 (f64 matrix instruction);
// power tables and accumulation of B in FP32 or binary64.
#include <type_traits>

#include "evaluate.h"
#include "wavesum.h"

namespace fmm2d {
namespace {

// log|z| for z with |z|^2 = d2 > 0: log_pos of d2, and for |z|^2 <= 2^-960
// (where d2 could underflow) the library's hypot and log, kept out of line
// (no input of ordinary scale reaches it) and returned by value.
__device__ __attribute__((noinline)) double log_abs_tiny(double x, double y) { return log(hypot(x, y)); }
__device__ inline double log_abs(cd z, double d2) { return d2 > 0x1p-960 ? 0.5 * log_pos(d2) : log_abs_tiny(z.re, z.im); }

// Global box id of a weak-list entry of level lvl: a box of that level, or,
// with FMM2D_VFLAG set, a box of the level above (interaction via the
// parent box, Section 4's structural option).
__device__ inline int64_t m2l_source(int32_t w, int lvl) {
    return (w & FMM2D_VFLAG) ? level_offset(lvl - 1) + (w & (FMM2D_VFLAG - 1)) : level_offset(lvl) + w;
}


typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v4d __attribute__((ext_vector_type(4)));

template <typename G>
struct Mfma;
// Operand A of the 16x16x4 instructions: lane i supplies A[i % 16][i / 16];
// operand B: lane i supplies B[i / 16][i % 16].  The accumulator layouts
// differ (measured on gfx950): element r of lane i holds D[4 (i/16) + r][i % 16]
// for f32 and D[i/16 + 4 r][i % 16] for f64.  Each variant therefore maps an
// operand row to (pair, real/imaginary part) so that element r of lane group
// g = i / 16 always holds pair 2g + r/2, part r % 2.
template <>
struct Mfma<float> {
    using V = v4f;
    static __device__ inline V run(float a, float b, V c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
    static __device__ inline int pair_of_row(int row) { return row >> 1; }
    static __device__ inline int part_of_row(int row) { return row & 1; }
};
template <>
struct Mfma<double> {
    using V = v4d;
    static __device__ inline V run(double a, double b, V c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
    static __device__ inline int pair_of_row(int row) { return 2 * (row & 3) + (row >> 3); }
    static __device__ inline int part_of_row(int row) { return (row >> 2) & 1; }
};

constexpr int CP = 16;   // pairs per chunk (two 16-row blocks)
constexpr int LPP = 4;   // lanes per pair for the power tables

__device__ inline cd cpow_int(cd z, int n) {
    cd r{1.0, 0.0};
    while (n) {
        if (n & 1) r = cmul(r, z);
        z = cmul(z, z);
        n >>= 1;
    }
    return r;
}

// complex arithmetic in the precision of the power tables
template <typename T>
struct cx {
    T re, im;
};
template <typename T>
__device__ inline cx<T> cxmul(cx<T> a, cx<T> b) {
    return cx<T>{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ inline cx<T> cxpow(cx<T> z, int n) {
    cx<T> r{(T)1, (T)0};
    while (n) {
        if (n & 1) r = cxmul(r, z);
        z = cxmul(z, z);
        n >>= 1;
    }
    return r;
}

// Two-way BF16 split of an FP32 value, x ~ hi + lo, each rounded to nearest
// even (the usual rounding of the upper half of the FP32 bit pattern).
typedef short v4s __attribute__((ext_vector_type(4)));
__device__ inline short bf16_rne(float x) {
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (short)(u >> 16);
}
__device__ inline float bf16_value(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }
__device__ inline void bf16_split(float x, short &hi, short &lo) {
    hi = bf16_rne(x);
    lo = bf16_rne(x - bf16_value(hi));
}

// Modes: G is the LDS / matrix-operand type, ACC the accumulation type, PT
// the power-table type (binary64 unless the mode accumulates in FP32), and
// BF3 replaces each FP32 product by three BF16 products of the split
// operands (hi hi + hi lo + lo hi; the lo lo term, ~2^-16 relative, is
// dropped), on the 16x16x16 BF16 matrix instruction: operand A lane i
// supplies A[i % 16][4 (i / 16) + j], operand B lane i supplies
// B[4 (i / 16) + j][i % 16], j = 0..3; the accumulator layout is that of
// the 16x16x4 FP32 instruction.
template <int NT, typename G, typename ACC, bool BF3>
__global__ void __launch_bounds__(64) k_m2l(int p, const double4 *__restrict__ geom,
                                            const int32_t *__restrict__ wptr_all,
                                            const int32_t *__restrict__ widx_pool, const int64_t *__restrict__ woff,
                                            const cd *__restrict__ A, const int2 *__restrict__ segtab,
                                            const int32_t *__restrict__ nseg_ptr, cd *__restrict__ part,
                                            const double *__restrict__ Mhat) {
    using MF = Mfma<G>;
    using V = typename MF::V;
    constexpr int KSMAX = 4 * NT;   // K steps when p + 1 = 16 NT
    constexpr int KP = 16 * NT;     // padded coefficient count held in LDS
    constexpr int KRMAX = KSMAX;    // powers per lane (LPP lanes per pair)
    __shared__ G Ur[CP][KP], Ui[CP][KP];
    __shared__ double Tr[CP][KP], Ti[CP][KP];
    const int64_t seg = blockIdx.x;
    if (seg >= *nseg_ptr) return;  // the block is one wavefront: uniform exit
    const int lane = threadIdx.x;
    const int2 se = segtab[seg];
    // the segment's level: its target box, lists and multipoles
    const int lvl = level_of(se.x);
    const int64_t b = se.x - level_offset(lvl);
    const double4 *geomL = geom + level_offset(lvl);
    const int32_t *wptr = wptr_all + ptr_offset(lvl);
    const int32_t *widx = widx_pool + woff[lvl];
    const int32_t t0 = se.y;
    const int32_t t1 = (t0 + M2L_SEG) < wptr[b + 1] ? (t0 + M2L_SEG) : wptr[b + 1];
    const int P1 = p + 1;
    const int ks_n = (P1 + 3) / 4;
    const int KR = (P1 + LPP - 1) / LPP;  // LPP * KR == 4 * ks_n <= KP: every padded k is written
    const double4 gb = geomL[b];
    using PT = typename std::conditional<std::is_same<ACC, float>::value, float, double>::type;
    G mreg[BF3 ? 1 : KSMAX][NT];
    v4s mbh[BF3 ? NT : 1][NT], mbl[BF3 ? NT : 1][NT];
    if constexpr (BF3) {
#pragma unroll
        for (int kb = 0; kb < NT; ++kb)
#pragma unroll
            for (int tl = 0; tl < NT; ++tl) {
                const int l = 16 * tl + lane % 16;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const int k = 16 * kb + 4 * (lane / 16) + j;
                    const float m = (k < P1 && l < P1) ? (float)Mhat[l * 64 + k] : 0.0f;
                    short h, lo;
                    bf16_split(m, h, lo);
                    mbh[kb][tl][j] = h;
                    mbl[kb][tl][j] = lo;
                }
            }
    } else {
#pragma unroll
        for (int ks = 0; ks < KSMAX; ++ks)
#pragma unroll
            for (int tl = 0; tl < NT; ++tl) {
                const int k = 4 * ks + lane / 16, l = 16 * tl + lane % 16;
                mreg[ks][tl] = (k < P1 && l < P1) ? (G)Mhat[l * 64 + k] : (G)0;
            }
    }
    ACC accr[NT], acci[NT];
#pragma unroll
    for (int tl = 0; tl < NT; ++tl) { accr[tl] = 0; acci[tl] = 0; }
    double ext0 = 0.0;
    const int q = lane / LPP, slot = lane % LPP;
    const int k0 = slot * KR;

    // Software pipeline: the source box of chunk i+2, and the geometry and
    // coefficients of chunk i+1, are loaded while chunk i is computed.
    int32_t c_n1 = 0, c_n2 = 0;
    double4 g_n1 = gb;
    cd a_n1[KRMAX];
    {
        const int np0 = (t1 - t0) < CP ? (t1 - t0) : CP;
        if (q < np0) c_n1 = widx[t0 + q];
        if (t0 + CP + q < t1) c_n2 = widx[t0 + CP + q];
        if (q < np0) {
            const int64_t cg = m2l_source(c_n1, lvl);
            g_n1 = geom[cg];
#pragma unroll
            for (int kk = 0; kk < KRMAX; ++kk) {
                const int k = k0 + kk;
                a_n1[kk] = (kk < KR && k < P1) ? A[cg * P1 + k] : cd{0.0, 0.0};
            }
        }
    }
    for (int32_t t = t0; t < t1; t += CP) {
        const int np = (t1 - t) < CP ? (t1 - t) : CP;
        const double4 gc = g_n1;
        cd a_cur[KRMAX];
#pragma unroll
        for (int kk = 0; kk < KRMAX; ++kk) a_cur[kk] = a_n1[kk];
        // prefetch for the next chunks
        {
            const int32_t tn = t + CP;
            if (tn + q < t1) {
                const int64_t cg = m2l_source(c_n2, lvl);
                g_n1 = geom[cg];
#pragma unroll
                for (int kk = 0; kk < KRMAX; ++kk) {
                    const int k = k0 + kk;
                    a_n1[kk] = (kk < KR && k < P1) ? A[cg * P1 + k] : cd{0.0, 0.0};
                }
            }
            if (tn + CP + q < t1) c_n2 = widx[tn + CP + q];
        }
        if (q < np) {
            const cd z0{gc.x - gb.x, gc.y - gb.y};
            const double d2 = z0.re * z0.re + z0.im * z0.im;  // > 0 for a weak pair
            const double inv = gc.w / d2;
            // s_c / z0 with one division; the scaled division where |z0|^2 could underflow
            const cd rs = d2 > 0x1p-960 ? cd{z0.re * inv, -z0.im * inv} : cdiv(cd{gc.w, 0.0}, z0);
            const cd rt = cscale(rs, gb.w / gc.w);            // s_b / z0
            const cx<PT> rsp{(PT)rs.re, (PT)rs.im}, rtp{(PT)rt.re, (PT)rt.im};
            cx<PT> ws = cxpow(rsp, k0), wt = cxpow(rtp, k0);
            PT sc2 = (PT)ldexp(1.0, k0);
#pragma unroll
            for (int kk = 0; kk < KRMAX; ++kk) {
                if (kk < KR) {
                    const int k = k0 + kk;
                    if (k < P1) {
                        const cx<PT> u = cxmul(cx<PT>{(PT)a_cur[kk].re, (PT)a_cur[kk].im}, ws);
                        Ur[q][k] = (G)(u.re * sc2);
                        Ui[q][k] = (G)(u.im * sc2);
                        Tr[q][k] = (double)(wt.re * sc2);
                        Ti[q][k] = (double)(wt.im * sc2);
                    } else if (k < KP) {
                        Ur[q][k] = (G)0;
                        Ui[q][k] = (G)0;
                        Tr[q][k] = 0.0;
                        Ti[q][k] = 0.0;
                    }
                    ws = cxmul(ws, rsp);
                    wt = cxmul(wt, rtp);
                    sc2 *= (PT)2;
                }
            }
            if (slot == 0) ext0 += a_cur[0].re * log_abs(z0, d2);
        } else {
#pragma unroll
            for (int kk = 0; kk < KRMAX; ++kk) {
                const int k = k0 + kk;
                if (kk < KR && k < KP) {
                    Ur[q][k] = (G)0;
                    Ui[q][k] = (G)0;
                    Tr[q][k] = 0.0;
                    Ti[q][k] = 0.0;
                }
            }
        }
        __syncthreads();
        const int row = lane % 16, g = lane / 16;
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
            if (8 * rb >= np) break;
            const int pa = 8 * rb + MF::pair_of_row(row);
            const G *urow = MF::part_of_row(row) ? Ui[pa] : Ur[pa];
#pragma unroll
            for (int tl = 0; tl < NT; ++tl) {
                V d = {0, 0, 0, 0};
                if constexpr (BF3) {
#pragma unroll
                    for (int kb = 0; kb < NT; ++kb) {
                        if (16 * kb < P1) {
                            v4s ah, al;
#pragma unroll
                            for (int j = 0; j < 4; ++j) {
                                // entries past the K steps of the FP32 path are not written
                                const int k = 16 * kb + 4 * g + j;
                                short h, lo;
                                bf16_split(k < P1 ? (float)urow[k] : 0.0f, h, lo);
                                ah[j] = h;
                                al[j] = lo;
                            }
                            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, mbh[kb][tl], d, 0, 0, 0);
                            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, mbl[kb][tl], d, 0, 0, 0);
                            d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, mbh[kb][tl], d, 0, 0, 0);
                        }
                    }
                } else {
#pragma unroll
                    for (int ks = 0; ks < KSMAX; ++ks)
                        if (ks < ks_n) d = MF::run(urow[4 * ks + g], mreg[ks][tl], d);
                }
                const int l = 16 * tl + row;
                if (l < P1) {
#pragma unroll
                    for (int pp = 0; pp < 2; ++pp) {
                        const int pr = 8 * rb + 2 * g + pp;
                        if (pr < np) {
                            const ACC wr = (ACC)d[2 * pp], wi = (ACC)d[2 * pp + 1];
                            const ACC tr = (ACC)Tr[pr][l], ti = (ACC)Ti[pr][l];
                            accr[tl] += tr * wr - ti * wi;
                            acci[tl] += tr * wi + ti * wr;
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int tl = 0; tl < NT; ++tl) {
        accr[tl] += __shfl_xor(accr[tl], 16, 64);
        acci[tl] += __shfl_xor(acci[tl], 16, 64);
        accr[tl] += __shfl_xor(accr[tl], 32, 64);
        acci[tl] += __shfl_xor(acci[tl], 32, 64);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ext0 += __shfl_xor(ext0, off, 64);
    if (lane < 16) {
#pragma unroll
        for (int tl = 0; tl < NT; ++tl) {
            const int l = 16 * tl + lane;
            if (l < P1) part[seg * P1 + l] = cd{(double)accr[tl] + (l == 0 ? ext0 : 0.0), (double)acci[tl]};
        }
    }
}

// Orders with p + 1 <= 32 (16 with split-BF16 products): one lane per pair,
// 64 pairs per chunk, one or two 16-wide output tiles.  Each lane
// computes its pair's geometry, power table and pre-scaled row u' (stored in
// LDS as two operand rows, real and imaginary part); the matrix instruction
// multiplies the 128 rows by M^T block by block, each block's result
// replacing its own rows in LDS; the lane then post-scales its pair's
// outputs by T'_l, and a transposing butterfly (each stage halves the values
// a lane carries) sums the chunk's 64 pairs in a fixed order, leaving each
// lane one running total per pass of at most 16 values.  The post-scaled
// values live only for one pass, which keeps the register count low.
template <int P1, typename G, typename ACC, bool BF3>
__global__ void __launch_bounds__(64) k_m2l_lp(const double4 *__restrict__ geom, const int32_t *__restrict__ wptr_all,
                                               const int32_t *__restrict__ widx_pool,
                                               const int64_t *__restrict__ woff, const cd *__restrict__ A,
                                               const int2 *__restrict__ segtab, const int32_t *__restrict__ nseg_ptr,
                                               cd *__restrict__ part, const double *__restrict__ Mhat) {
    static_assert(P1 >= 1 && P1 <= 32, "at most two 16-wide coefficient tiles");
    static_assert(!BF3 || P1 <= 16, "split-BF16 products: one tile");
    using MF = Mfma<G>;
    using V = typename MF::V;
    using PT = typename std::conditional<std::is_same<ACC, float>::value, float, double>::type;
    constexpr int NTL = (P1 + 15) / 16;                      // output tiles of 16 coefficients
    // row length: the products' K columns, and the outputs read back (the
    // first tile's 16, of the second only those below P1), plus one column of
    // padding against bank conflicts
    constexpr int KW = (4 * ((P1 + 3) / 4) > (NTL > 1 ? P1 : 16)) ? 4 * ((P1 + 3) / 4) : (NTL > 1 ? P1 : 16);
    constexpr int KP = KW + 1;
    constexpr int KS = (P1 + 3) / 4;                         // K steps of the FP32/FP64 instruction
    // the post-scaled values (Re, Im) are summed in passes of NV values
    // (NV / 2 coefficients each), which bounds the live registers
    constexpr int NV = P1 <= 4 ? 8 : 16;                     // values per pass, power of two
    constexpr int NH = (2 * P1 + NV - 1) / NV;               // passes
    constexpr int SPREAD = 64 / NV;                          // lanes sharing one value after the halving stages
    __shared__ G U[64][2][KP];
    const int64_t seg = blockIdx.x;
    if (seg >= *nseg_ptr) return;  // the block is one wavefront: uniform exit
    const int lane = threadIdx.x;
    const int2 se = segtab[seg];
    // the segment's level: its target box, lists and multipoles
    const int lvl = level_of(se.x);
    const int64_t b = se.x - level_offset(lvl);
    const double4 *geomL = geom + level_offset(lvl);
    const int32_t *wptr = wptr_all + ptr_offset(lvl);
    const int32_t *widx = widx_pool + woff[lvl];
    const int32_t t0 = se.y;
    const int32_t t1 = (t0 + M2L_SEG) < wptr[b + 1] ? (t0 + M2L_SEG) : wptr[b + 1];
    const int row = lane % 16, g = lane / 16;
    const double4 gb = geomL[b];
    G mreg[NTL][KS];
    v4s mbh, mbl;
    if constexpr (BF3) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            const float m = (k < P1 && row < P1) ? (float)Mhat[row * 64 + k] : 0.0f;
            short h, lo;
            bf16_split(m, h, lo);
            mbh[j] = h;
            mbl[j] = lo;
        }
    } else {
#pragma unroll
        for (int tl = 0; tl < NTL; ++tl) {
#pragma unroll
            for (int ks = 0; ks < KS; ++ks) {
                const int k = 4 * ks + g, l = 16 * tl + row;
                mreg[tl][ks] = (k < P1 && l < P1) ? (G)Mhat[l * 64 + k] : (G)0;
            }
        }
    }
    ACC tot[NH];  // running totals of value lane / SPREAD of each pass
#pragma unroll
    for (int hf = 0; hf < NH; ++hf) tot[hf] = (ACC)0;
    ACC ext0 = (ACC)0;
    for (int32_t t = t0; t < t1; t += 64) {
        const int np = (t1 - t) < 64 ? (t1 - t) : 64;
        const bool act = lane < np;
        cx<PT> rtp{(PT)0, (PT)0};
        if (act) {
            const int64_t cg = m2l_source(widx[t + lane], lvl);
            const double4 gc = geom[cg];
            const cd *Ac = A + cg * P1;
            cd a[P1];
#pragma unroll
            for (int k = 0; k < P1; ++k) a[k] = Ac[k];  // all loads in flight together
            const cd z0{gc.x - gb.x, gc.y - gb.y};
            const double d2 = z0.re * z0.re + z0.im * z0.im;  // > 0 for a weak pair
            const double inv = gc.w / d2;
            const cd rs = d2 > 0x1p-960 ? cd{z0.re * inv, -z0.im * inv} : cdiv(cd{gc.w, 0.0}, z0);
            const cd rt = cscale(rs, gb.w / gc.w);
            ext0 += (ACC)(a[0].re * log_abs(z0, d2));
            // 2 rho: the exact factors 2^k of the rescaled matrix ride on the powers
            const cx<PT> rsp{(PT)(2.0 * rs.re), (PT)(2.0 * rs.im)};
            rtp = cx<PT>{(PT)(2.0 * rt.re), (PT)(2.0 * rt.im)};
            cx<PT> w{(PT)1, (PT)0};
#pragma unroll
            for (int k = 0; k < P1; ++k) {
                const cx<PT> u = cxmul(cx<PT>{(PT)a[k].re, (PT)a[k].im}, w);
                U[lane][0][k] = (G)u.re;
                U[lane][1][k] = (G)u.im;
                w = cxmul(w, rsp);
            }
#pragma unroll
            for (int k = P1; k < 4 * KS || (BF3 && k < 16); ++k) {
                U[lane][0][k] = (G)0;  // K padding read by the products
                U[lane][1][k] = (G)0;
            }
        }
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < 8; ++rb) {
            if (8 * rb >= np) break;
            const int pa = 8 * rb + MF::pair_of_row(row);
            const G *ur = U[pa][MF::part_of_row(row)];
            V d = {0, 0, 0, 0};
            V d2 = {0, 0, 0, 0};  // second tile (coefficients 16..31)
            if constexpr (BF3) {
                v4s ah, al;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    short h, lo;
                    bf16_split((float)ur[4 * g + j], h, lo);
                    ah[j] = h;
                    al[j] = lo;
                }
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, mbh, d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, mbl, d, 0, 0, 0);
                d = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(al, mbh, d, 0, 0, 0);
            } else {
#pragma unroll
                for (int ks = 0; ks < KS; ++ks) {
                    const G a = ur[4 * ks + g];
                    d = MF::run(a, mreg[0][ks], d);
                    if constexpr (NTL > 1) d2 = MF::run(a, mreg[NTL - 1][ks], d2);
                }
            }
            // element r of lane group g is pair 8 rb + 2 g + r / 2, part r % 2,
            // coefficient l = 16 tl + row: those rows of U belong to this block
            // only (both tiles are formed before either is written)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                U[8 * rb + 2 * g + r / 2][r % 2][row] = (G)d[r];
                if constexpr (NTL > 1)
                    if (16 + row < P1) U[8 * rb + 2 * g + r / 2][r % 2][16 + row] = (G)d2[r];
            }
        }
        __syncthreads();
        cx<PT> tp{(PT)1, (PT)0};  // (2 rho_t)^l
#pragma unroll
        for (int hf = 0; hf < NH; ++hf) {
            ACC acc[NV];
#pragma unroll
            for (int j = 0; j < NV / 2; ++j) {
                const int l = hf * (NV / 2) + j;
                if (l < P1) {
                    // rows of lanes without a pair hold stale values: zero them
                    const ACC wr = act ? (ACC)U[lane][0][l] : (ACC)0, wi = act ? (ACC)U[lane][1][l] : (ACC)0;
                    const ACC tr = (ACC)tp.re, ti = (ACC)tp.im;
                    acc[2 * j] = fma(tr, wr, -ti * wi);
                    acc[2 * j + 1] = fma(tr, wi, ti * wr);
                    tp = cxmul(tp, rtp);
                } else {
                    acc[2 * j] = (ACC)0;
                    acc[2 * j + 1] = (ACC)0;
                }
            }
            tot[hf] += wave_transpose_sum<NV>(acc, lane);
        }
        __syncthreads();
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) ext0 += __shfl_xor(ext0, off, 64);
    const int idx = lane / SPREAD, comp = idx & 1;
#pragma unroll
    for (int hf = 0; hf < NH; ++hf) {
        const int l = hf * (NV / 2) + (idx >> 1);
        if (lane % SPREAD == 0 && l < P1) {
            double v = (double)tot[hf];
            if (l == 0 && comp == 0) v += (double)ext0;
            reinterpret_cast<double *>(part)[2 * (seg * P1 + l) + comp] = v;
        }
    }
}

template <int P1>
void launch_m2l_lp(fmm2d_ctx *c, int mode, dim3 grid, const double4 *geom, const int32_t *wp, const int32_t *wi,
                   const int64_t *woff, const cd *A, const int2 *tab, const int32_t *nsp, cd *part, const double *Mh) {
    const dim3 block(64);
    if (mode == FMM2D_MODE_FP64)
        hipLaunchKernelGGL((k_m2l_lp<P1, double, double, false>), grid, block, 0, c->stream, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
    else if (mode == FMM2D_MODE_FP32_ACC64)
        hipLaunchKernelGGL((k_m2l_lp<P1, float, double, false>), grid, block, 0, c->stream, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
    else if (mode == FMM2D_MODE_BF16X3) {
        if constexpr (P1 <= 16)
            hipLaunchKernelGGL((k_m2l_lp<P1, float, float, true>), grid, block, 0, c->stream, geom, wp, wi, woff, A,
                               tab, nsp, part, Mh);
    }
    else
        hipLaunchKernelGGL((k_m2l_lp<P1, float, float, false>), grid, block, 0, c->stream, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
}

// M^ table in binary64: M^[l][k] = M_lk / 2^(l+k), 64 x 64.
__global__ void k_make_mhat(double *Mhat, const double *binom) {
    const int l = blockIdx.x, k = threadIdx.x;
    double m;
    if (l == 0) m = (k == 0) ? 0.0 : ((k & 1) ? -1.0 : 1.0);
    else if (k == 0) m = -1.0 / l;
    else m = ((k & 1) ? -1.0 : 1.0) * binom[(l + k - 1) * 128 + (k - 1)];
    Mhat[l * 64 + k] = ldexp(m, -(l + k));
}

// M2L of every level in one launch (the segments of all levels' weak lists);
// the partial sums are added into B by the L2L pass.
template <int NT>
hipError_t launch_m2l_all(fmm2d_ctx *c, int p, int mode) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const Schedule &sc = t.m2l_all;
    const int64_t nbox = level_offset(t.L + 1);
    const double4 *geom = t.geom.as<double4>();
    const int32_t *wp = t.wptr.as<int32_t>();
    const int32_t *wi = t.widx.as<int32_t>();
    const int64_t *woff = t.pool_state.as<int64_t>() + (t.L + 2);  // W pool offset of each level
    const cd *A = e.A.as<cd>();
    const double *Mh = e.mhat.as<double>();
    FMM2D_TRY(e.part.ensure(sizeof(cd) * (sc.bound > 0 ? sc.bound : 1) * (p + 1)));
    cd *part = e.part.as<cd>();
    const int2 *tab = sc.table.as<int2>();
    const int32_t *nsp = sc.segoff.as<int32_t>() + nbox;
    const dim3 grid((unsigned)(sc.bound > 0 ? sc.bound : 1)), block(64);
    PhaseScope kernel_scope(c, PH_M2L_KERNEL);  // the kernel alone
    if (NT == 1) {
        switch (p + 1) {
#define FMM2D_M2L_LP(P1) \
    case P1: launch_m2l_lp<P1>(c, mode, grid, geom, wp, wi, woff, A, tab, nsp, part, Mh); break;
            FMM2D_M2L_LP(2) FMM2D_M2L_LP(3) FMM2D_M2L_LP(4) FMM2D_M2L_LP(5) FMM2D_M2L_LP(6) FMM2D_M2L_LP(7)
            FMM2D_M2L_LP(8) FMM2D_M2L_LP(9) FMM2D_M2L_LP(10) FMM2D_M2L_LP(11) FMM2D_M2L_LP(12)
            FMM2D_M2L_LP(13) FMM2D_M2L_LP(14) FMM2D_M2L_LP(15) FMM2D_M2L_LP(16)
            default: return hipErrorInvalidValue;
        }
    } else if (NT == 2 && mode != FMM2D_MODE_BF16X3) {
        switch (p + 1) {
            FMM2D_M2L_LP(17) FMM2D_M2L_LP(18) FMM2D_M2L_LP(19) FMM2D_M2L_LP(20) FMM2D_M2L_LP(21)
            FMM2D_M2L_LP(22) FMM2D_M2L_LP(23) FMM2D_M2L_LP(24) FMM2D_M2L_LP(25) FMM2D_M2L_LP(26)
            FMM2D_M2L_LP(27) FMM2D_M2L_LP(28) FMM2D_M2L_LP(29) FMM2D_M2L_LP(30) FMM2D_M2L_LP(31)
            FMM2D_M2L_LP(32)
#undef FMM2D_M2L_LP
            default: return hipErrorInvalidValue;
        }
    } else if (mode == FMM2D_MODE_FP64) {
        hipLaunchKernelGGL((k_m2l<NT, double, double, false>), grid, block, 0, c->stream, p, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
    } else if (mode == FMM2D_MODE_FP32_ACC64) {
        hipLaunchKernelGGL((k_m2l<NT, float, double, false>), grid, block, 0, c->stream, p, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
    } else if (mode == FMM2D_MODE_BF16X3) {
        hipLaunchKernelGGL((k_m2l<NT, float, float, true>), grid, block, 0, c->stream, p, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
    } else {
        hipLaunchKernelGGL((k_m2l<NT, float, float, false>), grid, block, 0, c->stream, p, geom, wp, wi, woff, A, tab,
                           nsp, part, Mh);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t ensure_mhat(fmm2d_ctx *c) {
    EvalState &e = c->ev;
    if (e.mhat_ready) return hipSuccess;
    FMM2D_TRY(ensure_binomials(c));
    FMM2D_TRY(e.mhat.ensure(sizeof(double) * 64 * 64));
    hipLaunchKernelGGL(k_make_mhat, dim3(64), dim3(64), 0, c->stream, e.mhat.as<double>(), e.binom.as<double>());
    FMM2D_TRY(hipGetLastError());
    e.mhat_ready = true;
    return hipSuccess;
}

hipError_t m2l_all(fmm2d_ctx *c, int p, int mode) {
    TreeState &t = c->tree;
    if (t.L < 1 || t.w_off[t.L + 1] == t.w_off[1]) return hipSuccess;  // no weak pairs
    const int nt = (p + 1 + 15) / 16;
    switch (nt) {
        case 1: return launch_m2l_all<1>(c, p, mode);
        case 2: return launch_m2l_all<2>(c, p, mode);
        case 3: return launch_m2l_all<3>(c, p, mode);
        default: return launch_m2l_all<4>(c, p, mode);
    }
}

}  // namespace fmm2d
