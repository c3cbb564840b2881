// Expansions and the evaluation pass (Section 4), binary64 operators.
//
// Representation (the classical complex one of Section 5), each expansion
// normalised by its box's scale s (the enclosing-ball radius, or 1 for a box
// of zero size):
//   multipole about c:  A_0 log(z - c) + sum_{k>=1} A_k (s / (z - c))^k
//   local about c:      sum_{l>=0} B_l ((z - c) / s)^l
// Coefficients are complex binary64, stored per box as p+1 consecutive
// values (box-major), boxes numbered level by level.
//
// Order of the passes: P2M at the leaves, M2M to the root; then for each
// level from the root down, M2L along that level's weak lists (m2l.hip)
// followed by L2L to the next level; finally L2P and the near-field sum over
// the finest strong lists (near.hip), and the scatter back to input order.
#include <algorithm>
#include <vector>

#include "devutil.h"
#include "internal.h"
#include "evaluate.h"
#include "wavesum.h"

namespace fmm2d {
namespace {

constexpr int BN = 128;  // binomial table is BN x BN
constexpr int REG_P1 = 24;  // M2M and L2L with coefficients in registers up to this order p + 1

// ---- P2M: one thread per leaf, coefficients in registers -------------------
template <int PB>
__global__ void __launch_bounds__(256) k_p2m(int p, const double *__restrict__ px, const double *__restrict__ py,
                                             const double *__restrict__ qs, const int32_t *__restrict__ stL,
                                             const double4 *__restrict__ geomL, int64_t nleaf, cd *__restrict__ AL) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nleaf) return;
    const double4 g = geomL[b];
    const int32_t a = stL[b], e = stL[b + 1];
    double ar[PB], ai[PB];
#pragma unroll
    for (int k = 0; k < PB; ++k) { ar[k] = 0.0; ai[k] = 0.0; }
    for (int32_t j = a; j < e; ++j) {
        const double q = qs[j];
        const double zr = (px[j] - g.x) / g.w, zi = (py[j] - g.y) / g.w;
        double wr = zr, wi = zi;
        ar[0] += q;
#pragma unroll
        for (int k = 1; k < PB; ++k) {
            if (k <= p) {
                ar[k] += q * wr;
                ai[k] += q * wi;
                const double tr = wr * zr - wi * zi;
                wi = wr * zi + wi * zr;
                wr = tr;
            }
        }
    }
    cd *out = AL + b * (p + 1);
    out[0] = cd{ar[0], 0.0};
#pragma unroll
    for (int k = 1; k < PB; ++k)
        if (k <= p) out[k] = cd{-ar[k] / k, -ai[k] / k};
}

// ---- P2M for leaves of more than 16 points, orders p + 1 <= 32: one
// wavefront per leaf, one lane per point (points lane, lane + 64, ... of a
// larger leaf), and the lanes' 2 PB partial sums (real parts, then imaginary
// parts) added by a transposing butterfly in a fixed order.  The thread per
// leaf above leaves most of the chip idle when leaves are few and long.
template <int PB>
__global__ void __launch_bounds__(256) k_p2m_wave(int p, const double *__restrict__ px,
                                                  const double *__restrict__ py, const double *__restrict__ qs,
                                                  const int32_t *__restrict__ stL, const double4 *__restrict__ geomL,
                                                  int64_t nleaf, cd *__restrict__ AL) {
    static_assert(PB == 8 || PB == 16 || PB == 32, "2 PB values per lane");
    const int lane = (int)(threadIdx.x % 64);
    const int64_t b = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (b >= nleaf) return;  // uniform per wavefront
    const double4 g = geomL[b];
    const int32_t a = stL[b], e = stL[b + 1];
    double v[2 * PB];  // v[k]: sum of q Re w^k, v[PB + k]: sum of q Im w^k
#pragma unroll
    for (int k = 0; k < 2 * PB; ++k) v[k] = 0.0;
    for (int32_t j = a + lane; j < e; j += 64) {
        const double q = qs[j];
        const double zr = (px[j] - g.x) / g.w, zi = (py[j] - g.y) / g.w;
        double wr = zr, wi = zi;
        v[0] += q;
#pragma unroll
        for (int k = 1; k < PB; ++k) {
            if (k <= p) {
                v[k] += q * wr;
                v[PB + k] += q * wi;
                const double tr = wr * zr - wi * zi;
                wi = wr * zi + wi * zr;
                wr = tr;
            }
        }
    }
    const double s = wave_transpose_sum<2 * PB>(v, lane);  // value lane / G, G lanes each
    constexpr int G = 32 / PB;  // lanes per value
    if (lane % G == 0) {
        const int vi = lane / G;
        const bool im = vi >= PB;
        const int k = im ? vi - PB : vi;
        if (k <= p) {
            double *out = reinterpret_cast<double *>(AL + b * (p + 1)) + 2 * k + (im ? 1 : 0);
            *out = k == 0 ? (im ? 0.0 : s) : -s / k;
        }
    }
}

// Powers x^lane for every lane, by an inclusive product scan across the wave.
__device__ inline cd wave_powers(cd x) {
    const uint32_t lane = lane_id();
    cd v = lane == 0 ? cd{1.0, 0.0} : x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        cd u{__shfl_up(v.re, off, 64), __shfl_up(v.im, off, 64)};
        if (lane >= (uint32_t)off) v = cmul(u, v);
    }
    return v;
}
__device__ inline double wave_powers_real(double x) {
    const uint32_t lane = lane_id();
    double v = lane == 0 ? 1.0 : x;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double u = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v = u * v;
    }
    return v;
}

// Binomials C(i, j), i, j <= p, from the table into the block's LDS copy
// (row i at s_bin + 64 i), every thread of the block taking part.
__device__ inline void stage_binomials(int p, const double *__restrict__ binom, double *s_bin) {
    for (int idx = threadIdx.x; idx < (p + 1) * 64; idx += blockDim.x) s_bin[idx] = binom[(idx >> 6) * BN + (idx & 63)];
    __syncthreads();
}

// ---- M2M: one wavefront per parent box, lane l = output coefficient; four
// parents per block sharing one LDS copy of the binomials.  The four
// children's coefficients are loaded before the first is used.
__global__ void __launch_bounds__(256) k_m2m(int l, int p, int64_t np, const double4 *__restrict__ geom,
                                             cd *__restrict__ A, const double *__restrict__ binom) {
    __shared__ double s_bin[64 * 64];
    __shared__ cd Ac[4][64];
    __shared__ cd dp[4][64];
    __shared__ double sp[4][64];
    stage_binomials(p, binom, s_bin);
    const int wv = threadIdx.x / 64;
    const int64_t P = (int64_t)blockIdx.x * 4 + wv;
    if (P >= np) return;  // uniform per wavefront (no block barrier below)
    const int lane = (int)lane_id();
    const int64_t pbox = level_offset(l) + P;
    const double4 gp = geom[pbox];
    double4 gch[4];
    cd ach[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const int64_t cbox = level_offset(l + 1) + 4 * P + c;
        gch[c] = geom[cbox];
        ach[c] = lane <= p ? A[cbox * (p + 1) + lane] : cd{0.0, 0.0};
    }
    cd acc{0.0, 0.0};
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        const double4 gc = gch[c];
        const cd delta{(gc.x - gp.x) / gp.w, (gc.y - gp.y) / gp.w};
        const double sigma = gc.w / gp.w;
        const cd dpow = wave_powers(delta);
        const double spow = wave_powers_real(sigma);
        Ac[wv][lane] = ach[c];
        dp[wv][lane] = dpow;
        sp[wv][lane] = spow;
        __builtin_amdgcn_wave_barrier();
        if (lane <= p) {
            if (lane == 0) {
                acc = cadd(acc, Ac[wv][0]);
            } else {
                cd t = cscale(cmul(Ac[wv][0], dp[wv][lane]), -1.0 / lane);
                for (int k = 1; k <= lane; ++k) {
                    const double coef = sp[wv][k] * s_bin[(lane - 1) * 64 + (k - 1)];
                    t = cadd(t, cscale(cmul(Ac[wv][k], dp[wv][lane - k]), coef));
                }
                acc = cadd(acc, t);
            }
        }
        __builtin_amdgcn_wave_barrier();  // the slices are rewritten for the next child
    }
    if (lane <= p) A[pbox * (p + 1) + lane] = acc;
}

// ---- L2L: one wavefront per child box, lane l = coefficient, four children
// per block sharing one LDS copy of the binomials ----------------------------
// B(child) = the parent's local expansion re-centred at the child, plus the
// child's M2L segment sums (segments of global box g are
// [segoff[g], segoff[g + 1]) in part), added in segment order.
__global__ void __launch_bounds__(256) k_l2l(int l, int p, int64_t nc, const double4 *__restrict__ geom,
                                             cd *__restrict__ B, const double *__restrict__ binom,
                                             const int32_t *__restrict__ segoff, const cd *__restrict__ part,
                                             const int32_t *__restrict__ xoff, const cd *__restrict__ xsum) {
    __shared__ double s_bin[64 * 64];
    __shared__ cd Bp[4][64];
    __shared__ cd dp[4][64];
    stage_binomials(p, binom, s_bin);
    const int wv = threadIdx.x / 64;
    const int64_t cidx = (int64_t)blockIdx.x * 4 + wv;  // child within level l+1
    if (cidx >= nc) return;  // uniform per wavefront (no block barrier below)
    const int lane = (int)lane_id();
    const int64_t cbox = level_offset(l + 1) + cidx;
    const int64_t pbox = level_offset(l) + (cidx >> 2);
    const double4 gc = geom[cbox], gp = geom[pbox];
    const cd delta{(gc.x - gp.x) / gp.w, (gc.y - gp.y) / gp.w};
    const double tau = gc.w / gp.w;
    const cd dpow = wave_powers(delta);
    const double tpow = wave_powers_real(tau);
    if (lane <= p) Bp[wv][lane] = B[pbox * (p + 1) + lane];
    dp[wv][lane] = dpow;
    __builtin_amdgcn_wave_barrier();
    if (lane <= p) {
        cd t{0.0, 0.0};
        for (int k = lane; k <= p; ++k)
            t = cadd(t, cscale(cmul(Bp[wv][k], dp[wv][k - lane]), s_bin[k * 64 + lane]));
        cd v = cscale(t, tpow);
        const int32_t s0 = segoff[cbox], s1 = segoff[cbox + 1];
        if (s1 > s0) {
            cd acc{0.0, 0.0};
            for (int32_t sg = s0; sg < s1; ++sg) acc = cadd(acc, part[(int64_t)sg * (p + 1) + lane]);
            v = cadd(v, acc);
        }
        // the P2L sum of the exchanged-roles pairs (boxes with P2L items)
        if (xoff && xoff[cbox + 1] > xoff[cbox]) v = cadd(v, xsum[cbox * (p + 1) + lane]);
        B[cbox * (p + 1) + lane] = v;
    }
}

// ---- M2M and L2L for p + 1 <= REG_P1: one lane per box, coefficients in registers
// With C(n, k) = n! / (k! (n - k)!) the binomial sums are convolutions:
//   M2M (parent coefficient l >= 1, from one child):
//     (l - 1)! sum_{k=0..l} a'_k e_{l-k},  a'_0 = -A_0, a'_k = A_k sigma^k / (k - 1)!,
//   L2L (child coefficient l):
//     (tau^l / l!) sum_{k=l..p} b'_k e_{k-l},  b'_k = B_k k!,
// with e_j = delta^j / j!, delta the centre offset over the parent's scale,
// sigma and tau the ratios of the scales.  P1 is a compile-time constant,
// so every factorial is a constant and the loops unroll completely.
template <int N>
struct Fact {
    double f[N], inv[N];
    constexpr Fact() : f(), inv() {
        double v = 1.0;
        for (int i = 0; i < N; ++i) {
            if (i > 0) v *= i;
            f[i] = v;
            inv[i] = 1.0 / v;
        }
    }
};

// e_j = delta^j / j!, j < P1
template <int P1>
__device__ inline void scaled_powers(cd delta, cd *e) {
    constexpr Fact<P1> F;
    e[0] = cd{1.0, 0.0};
    cd w = delta;
#pragma unroll
    for (int j = 1; j < P1; ++j) {
        e[j] = cscale(w, F.inv[j]);
        if (j + 1 < P1) w = cmul(w, delta);
    }
}

// M2M into parent P of level l from its four children.
template <int P1>
__device__ inline void m2m_one(int l, int64_t P, const double4 *__restrict__ geom, cd *__restrict__ A) {
    constexpr Fact<P1> F;
    const int64_t pbox = level_offset(l) + P;
    const double4 gp = geom[pbox];
    const double is = 1.0 / gp.w;
    cd acc[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) acc[k] = cd{0.0, 0.0};
    for (int c = 0; c < 4; ++c) {
        const int64_t cbox = level_offset(l + 1) + 4 * P + c;
        const double4 gc = geom[cbox];
        cd a[P1];
#pragma unroll
        for (int k = 0; k < P1; ++k) a[k] = A[cbox * P1 + k];
        cd e[P1];
        scaled_powers<P1>(cd{(gc.x - gp.x) * is, (gc.y - gp.y) * is}, e);
        const double sigma = gc.w * is;
        acc[0] = cadd(acc[0], a[0]);
        // a'_k in place
        a[0] = cd{-a[0].re, -a[0].im};
        double sk = 1.0;
#pragma unroll
        for (int k = 1; k < P1; ++k) {
            sk *= sigma;
            a[k] = cscale(a[k], sk * F.inv[k - 1]);
        }
#pragma unroll
        for (int lo = 1; lo < P1; ++lo) {
            cd t{0.0, 0.0};
#pragma unroll
            for (int k = 0; k <= lo; ++k) {
                t.re = fma(a[k].re, e[lo - k].re, t.re);
                t.re = fma(-a[k].im, e[lo - k].im, t.re);
                t.im = fma(a[k].re, e[lo - k].im, t.im);
                t.im = fma(a[k].im, e[lo - k].re, t.im);
            }
            acc[lo] = cadd(acc[lo], cscale(t, F.f[lo - 1]));
        }
    }
#pragma unroll
    for (int k = 0; k < P1; ++k) A[pbox * P1 + k] = acc[k];
}

// B(child) = the parent's local expansion re-centred at the child, plus the
// child's M2L segment sums in segment order.
template <int P1>
__global__ void __launch_bounds__(64) k_m2m_box(int l, int64_t nparent, const double4 *__restrict__ geom,
                                                cd *__restrict__ A) {
    const int64_t P = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (P < nparent) m2m_one<P1>(l, P, geom, A);
}

// M2M of the coarse levels lc, lc - 1, ..., 0 (at most COARSE boxes each) in
// one workgroup: these levels are too small to fill the chip, and one launch
// per level would leave the pass launch-bound.  A device-scope fence before
// each barrier makes a level's stores visible to the next level's loads.
constexpr int COARSE = 256;
template <int P1>
__global__ void __launch_bounds__(COARSE) k_m2m_coarse(int lc, const double4 *__restrict__ geom, cd *__restrict__ A) {
    for (int l = lc; l >= 0; --l) {
        if ((int64_t)threadIdx.x < (int64_t(1) << (2 * l))) m2m_one<P1>(l, threadIdx.x, geom, A);
        __threadfence();
        __syncthreads();
    }
}

// L2L into child cidx of level l + 1 from its parent, plus the child's M2L
// segment sums in segment order.
template <int P1>
__device__ inline void l2l_one(int l, int64_t cidx, const double4 *__restrict__ geom, cd *__restrict__ B,
                               const int32_t *__restrict__ segoff, const cd *__restrict__ part,
                               const int32_t *__restrict__ xoff, const cd *__restrict__ xsum) {
    constexpr Fact<P1> F;
    const int64_t cbox = level_offset(l + 1) + cidx;
    const int64_t pbox = level_offset(l) + (cidx >> 2);
    const double4 gc = geom[cbox], gp = geom[pbox];
    const double is = 1.0 / gp.w;
    cd bp[P1];
#pragma unroll
    for (int k = 0; k < P1; ++k) {
        const cd v = B[pbox * P1 + k];
        bp[k] = cscale(v, F.f[k]);
    }
    cd e[P1];
    scaled_powers<P1>(cd{(gc.x - gp.x) * is, (gc.y - gp.y) * is}, e);
    const double tau = gc.w * is;
    cd out[P1];
    double tl = 1.0;
#pragma unroll
    for (int lo = 0; lo < P1; ++lo) {
        cd t{0.0, 0.0};
#pragma unroll
        for (int k = lo; k < P1; ++k) {
            t.re = fma(bp[k].re, e[k - lo].re, t.re);
            t.re = fma(-bp[k].im, e[k - lo].im, t.re);
            t.im = fma(bp[k].re, e[k - lo].im, t.im);
            t.im = fma(bp[k].im, e[k - lo].re, t.im);
        }
        out[lo] = cscale(t, tl * F.inv[lo]);
        tl *= tau;
    }
    const int32_t s0 = segoff[cbox], s1 = segoff[cbox + 1];
    for (int32_t sg = s0; sg < s1; ++sg) {
#pragma unroll
        for (int k = 0; k < P1; ++k) out[k] = cadd(out[k], part[(int64_t)sg * P1 + k]);
    }
    // the P2L sum of the exchanged-roles pairs (boxes with P2L items)
    if (xoff && xoff[cbox + 1] > xoff[cbox]) {
#pragma unroll
        for (int k = 0; k < P1; ++k) out[k] = cadd(out[k], xsum[cbox * P1 + k]);
    }
#pragma unroll
    for (int k = 0; k < P1; ++k) B[cbox * P1 + k] = out[k];
}

template <int P1>
__global__ void __launch_bounds__(64) k_l2l_box(int l, int64_t nchild, const double4 *__restrict__ geom,
                                                cd *__restrict__ B, const int32_t *__restrict__ segoff,
                                                const cd *__restrict__ part, const int32_t *__restrict__ xoff,
                                                const cd *__restrict__ xsum) {
    const int64_t cidx = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (cidx < nchild) l2l_one<P1>(l, cidx, geom, B, segoff, part, xoff, xsum);
}

// L2L into the children of levels 1, ..., lc + 1 (at most COARSE each) in one
// workgroup, as k_m2m_coarse.
template <int P1>
__global__ void __launch_bounds__(COARSE) k_l2l_coarse(int lc, const double4 *__restrict__ geom, cd *__restrict__ B,
                                                       const int32_t *__restrict__ segoff,
                                                       const cd *__restrict__ part, const int32_t *__restrict__ xoff,
                                                       const cd *__restrict__ xsum) {
    for (int l = 0; l <= lc; ++l) {
        if ((int64_t)threadIdx.x < (int64_t(1) << (2 * (l + 1))))
            l2l_one<P1>(l, threadIdx.x, geom, B, segoff, part, xoff, xsum);
        __threadfence();
        __syncthreads();
    }
}

__global__ void k_gather_q(const double *__restrict__ q, const int32_t *__restrict__ perm, int64_t n,
                           double *__restrict__ qs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) qs[i] = q[perm[i]];
}

__global__ void k_zero_cd(cd *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = cd{0.0, 0.0};
}

template <int PB>
hipError_t launch_p2m(fmm2d_ctx *c, int p, cd *A) {
    TreeState &t = c->tree;
    const int64_t nleaf = int64_t(1) << (2 * t.L);
    if constexpr (PB <= 32) {
        const int64_t maxleaf = (t.n + nleaf - 1) >> (2 * t.L);  // ceil(n / 4^L)
        if (maxleaf > 16) {
            constexpr int PW = PB <= 8 ? 8 : (PB <= 16 ? 16 : 32);  // 2 PW values: a power of two
            hipLaunchKernelGGL(k_p2m_wave<PW>, dim3(grid_for(nleaf, 4)), dim3(256), 0, c->stream, p,
                               t.px.as<double>(), t.py.as<double>(), c->ev.qs.as<double>(),
                               t.starts.as<int32_t>() + depth_offset(2 * t.L), t.geom.as<double4>() + level_offset(t.L),
                               nleaf, A + level_offset(t.L) * (p + 1));
            return hipGetLastError();
        }
    }
    hipLaunchKernelGGL(k_p2m<PB>, dim3(grid_for(nleaf, 256)), dim3(256), 0, c->stream, p, t.px.as<double>(),
                       t.py.as<double>(), c->ev.qs.as<double>(), t.starts.as<int32_t>() + depth_offset(2 * t.L),
                       t.geom.as<double4>() + level_offset(t.L), nleaf, A + level_offset(t.L) * (p + 1));
    return hipGetLastError();
}

}  // namespace

hipError_t ensure_binomials(fmm2d_ctx *c) {
    EvalState &e = c->ev;
    if (e.binom_ready) return hipSuccess;
    std::vector<double> h(BN * BN, 0.0);
    for (int nn = 0; nn < BN; ++nn) {
        h[nn * BN + 0] = 1.0;
        for (int k = 1; k <= nn; ++k) h[nn * BN + k] = h[(nn - 1) * BN + (k - 1)] + (k <= nn - 1 ? h[(nn - 1) * BN + k] : 0.0);
    }
    FMM2D_TRY(e.binom.ensure(sizeof(double) * BN * BN));
    FMM2D_TRY(hipMemcpyAsync(e.binom.ptr, h.data(), sizeof(double) * BN * BN, hipMemcpyHostToDevice, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    e.binom_ready = true;
    return hipSuccess;
}

// Upward pass (P2M, M2M) and downward pass (M2L, L2L), binary64 operators,
// (M2L itself is in m2l.hip.)
hipError_t upward_pass(fmm2d_ctx *c, int p) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int L = t.L;
    cd *A = e.A.as<cd>();
    const double *binom = e.binom.as<double>();
    hipError_t r;
    if (p < 8) r = launch_p2m<8>(c, p, A);
    else if (p < 16) r = launch_p2m<16>(c, p, A);
    else if (p < 24) r = launch_p2m<24>(c, p, A);
    else if (p < 32) r = launch_p2m<32>(c, p, A);
    else if (p < 48) r = launch_p2m<48>(c, p, A);
    else r = launch_p2m<64>(c, p, A);
    FMM2D_TRY(r);
    const double4 *geom = t.geom.as<double4>();
    // levels of at most COARSE parents (l <= 4) in one launch, after the finer ones
    const int lc = p + 1 <= REG_P1 ? std::min(L - 1, 4) : -1;
    for (int l = L - 1; l > lc; --l) {
        const int64_t np = int64_t(1) << (2 * l);
        if (p + 1 <= REG_P1) {
            const dim3 grid(grid_for(np, 64)), block(64);
            switch (p + 1) {
#define FMM2D_M2M(P1) \
    case P1: hipLaunchKernelGGL(k_m2m_box<P1>, grid, block, 0, c->stream, l, np, geom, A); break;
                FMM2D_M2M(2) FMM2D_M2M(3) FMM2D_M2M(4) FMM2D_M2M(5) FMM2D_M2M(6) FMM2D_M2M(7) FMM2D_M2M(8)
                FMM2D_M2M(9) FMM2D_M2M(10) FMM2D_M2M(11) FMM2D_M2M(12) FMM2D_M2M(13) FMM2D_M2M(14)
                FMM2D_M2M(15) FMM2D_M2M(16) FMM2D_M2M(17) FMM2D_M2M(18) FMM2D_M2M(19) FMM2D_M2M(20)
                FMM2D_M2M(21) FMM2D_M2M(22) FMM2D_M2M(23) FMM2D_M2M(24)
#undef FMM2D_M2M
                default: return hipErrorInvalidValue;
            }
        } else {
            hipLaunchKernelGGL(k_m2m, dim3(grid_for(np, 4)), dim3(256), 0, c->stream, l, p, np, geom, A, binom);
        }
    }
    if (lc >= 0) {
        switch (p + 1) {
#define FMM2D_M2MC(P1)     case P1: hipLaunchKernelGGL(k_m2m_coarse<P1>, dim3(1), dim3(COARSE), 0, c->stream, lc, geom, A); break;
            FMM2D_M2MC(2) FMM2D_M2MC(3) FMM2D_M2MC(4) FMM2D_M2MC(5) FMM2D_M2MC(6) FMM2D_M2MC(7) FMM2D_M2MC(8)
            FMM2D_M2MC(9) FMM2D_M2MC(10) FMM2D_M2MC(11) FMM2D_M2MC(12) FMM2D_M2MC(13) FMM2D_M2MC(14)
            FMM2D_M2MC(15) FMM2D_M2MC(16) FMM2D_M2MC(17) FMM2D_M2MC(18) FMM2D_M2MC(19) FMM2D_M2MC(20)
                FMM2D_M2MC(21) FMM2D_M2MC(22) FMM2D_M2MC(23) FMM2D_M2MC(24)
#undef FMM2D_M2MC
            default: return hipErrorInvalidValue;
        }
    }
    return hipGetLastError();
}

hipError_t l2l_level(fmm2d_ctx *c, int l, int p) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t nc = int64_t(1) << (2 * (l + 1));
    const double4 *geom = t.geom.as<double4>();
    const int32_t *segoff = t.m2l_all.segoff.as<int32_t>();
    const int32_t *xoff = exchange_item_offsets(c);
    const cd *xsum = xoff ? e.xsum.as<cd>() : nullptr;
    if (p + 1 <= REG_P1) {
        const dim3 grid(grid_for(nc, 64)), block(64);
        switch (p + 1) {
#define FMM2D_L2L(P1)                                                                                            \
    case P1:                                                                                                     \
        hipLaunchKernelGGL(k_l2l_box<P1>, grid, block, 0, c->stream, l, nc, geom, e.B.as<cd>(), segoff,         \
                           e.part.as<cd>(), xoff, xsum);                                                        \
        break;
            FMM2D_L2L(2) FMM2D_L2L(3) FMM2D_L2L(4) FMM2D_L2L(5) FMM2D_L2L(6) FMM2D_L2L(7) FMM2D_L2L(8)
            FMM2D_L2L(9) FMM2D_L2L(10) FMM2D_L2L(11) FMM2D_L2L(12) FMM2D_L2L(13) FMM2D_L2L(14) FMM2D_L2L(15)
            FMM2D_L2L(16) FMM2D_L2L(17) FMM2D_L2L(18) FMM2D_L2L(19) FMM2D_L2L(20)
                FMM2D_L2L(21) FMM2D_L2L(22) FMM2D_L2L(23) FMM2D_L2L(24)
#undef FMM2D_L2L
            default: return hipErrorInvalidValue;
        }
    } else {
        hipLaunchKernelGGL(k_l2l, dim3(grid_for(nc, 4)), dim3(256), 0, c->stream, l, p, nc, geom, e.B.as<cd>(),
                           e.binom.as<double>(), segoff, e.part.as<cd>(), xoff, xsum);
    }
    return hipGetLastError();
}

// L2L of every level: children of levels 1..4 (at most COARSE each) in one
// launch, then one launch per finer level.
hipError_t l2l_pass(fmm2d_ctx *c, int p) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int L = t.L;
    int l0 = 0;
    if (p + 1 <= REG_P1 && L >= 1) {
        const int lc = std::min(L - 1, 3);
        const double4 *geom = t.geom.as<double4>();
        const int32_t *segoff = t.m2l_all.segoff.as<int32_t>();
        const int32_t *xoff = exchange_item_offsets(c);
        const cd *xsum = xoff ? e.xsum.as<cd>() : nullptr;
        switch (p + 1) {
#define FMM2D_L2LC(P1)                                                                                                  case P1:                                                                                                                hipLaunchKernelGGL(k_l2l_coarse<P1>, dim3(1), dim3(COARSE), 0, c->stream, lc, geom, e.B.as<cd>(), segoff,                            e.part.as<cd>(), xoff, xsum);                                                                                break;
            FMM2D_L2LC(2) FMM2D_L2LC(3) FMM2D_L2LC(4) FMM2D_L2LC(5) FMM2D_L2LC(6) FMM2D_L2LC(7) FMM2D_L2LC(8)
            FMM2D_L2LC(9) FMM2D_L2LC(10) FMM2D_L2LC(11) FMM2D_L2LC(12) FMM2D_L2LC(13) FMM2D_L2LC(14)
            FMM2D_L2LC(15) FMM2D_L2LC(16) FMM2D_L2LC(17) FMM2D_L2LC(18) FMM2D_L2LC(19) FMM2D_L2LC(20)
                FMM2D_L2LC(21) FMM2D_L2LC(22) FMM2D_L2LC(23) FMM2D_L2LC(24)
#undef FMM2D_L2LC
            default: return hipErrorInvalidValue;
        }
        FMM2D_TRY(hipGetLastError());
        l0 = lc + 1;
    }
    for (int l = l0; l < L; ++l) FMM2D_TRY(l2l_level(c, l, p));  // parent's expansion plus the level's M2L sums
    return hipSuccess;
}

hipError_t evaluate_device(fmm2d_ctx *c, const double *q, int p, int mode, double *phi) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t n = t.n;
    const int L = t.L;
    const int64_t nbox = level_offset(L + 1);
    FMM2D_TRY(ensure_mhat(c));
    FMM2D_TRY(e.A.ensure(sizeof(cd) * nbox * (p + 1)));
    FMM2D_TRY(e.B.ensure(sizeof(cd) * nbox * (p + 1)));
    FMM2D_TRY(e.qs.ensure(sizeof(double) * n));
    FMM2D_TRY(side_join(c));  // second-stream work of an earlier call still reading the charges or sources
    {
        PhaseScope ps(c, PH_OTHER);
        hipLaunchKernelGGL(k_gather_q, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, q, t.perm.as<int32_t>(), n,
                           e.qs.as<double>());
        hipLaunchKernelGGL(k_zero_cd, dim3(1), dim3(64), 0, c->stream, e.B.as<cd>(), (int64_t)(p + 1));
    }
    {
        PhaseScope ps(c, PH_UPWARD);
        FMM2D_TRY(upward_pass(c, p));
    }
    {
        // the near field needs no expansion: it runs on the second stream
        // while M2L and L2L run here.  It is released after the upward pass,
        // whose short per-level launches would otherwise wait for compute
        // units behind the near kernel's blocks.
        PhaseScope ps(c, PH_LEAF);
        FMM2D_TRY(leaf_pass(c, p, mode, NEAR_PREP, phi));
        FMM2D_TRY(leaf_pass(c, p, mode, NEAR_LAUNCH, phi));
    }
    {
        PhaseScope ps(c, PH_M2L);
        FMM2D_TRY(m2l_all(c, p, mode));  // every level at once, into segment sums
    }
    FMM2D_TRY(e.part.ensure(sizeof(cd)));  // a valid pointer also when there is no weak pair
    {
        // exchanged roles, target the smaller box: its P2L partials, which
        // the L2L pass adds into B; target the larger box: the M2P sums at
        // its points, which the leaf pass adds
        PhaseScope ps(c, PH_EXCHANGE);
        FMM2D_TRY(p2l_all(c, p));
        FMM2D_TRY(m2p_partials(c, p));
    }
    {
        PhaseScope ps(c, PH_L2L);
        FMM2D_TRY(l2l_pass(c, p));
    }
    {
        PhaseScope ps(c, PH_LEAF);
        FMM2D_TRY(leaf_pass(c, p, mode, NEAR_FINISH, phi));
    }
    {
        // exchanged roles above order 32: M2P added into phi at the end
        PhaseScope ps(c, PH_EXCHANGE);
        FMM2D_TRY(m2p_direct(c, p, phi));
    }
    return hipGetLastError();
}

}  // namespace fmm2d
