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
// level from the root down, M2L along that level's weak lists followed by L2L
// to the next level; finally L2P and the near-field sum over the finest
// strong lists, and the scatter back to input order.
#include <vector>

#include "devutil.h"
#include "internal.h"
#include "evaluate.h"

namespace fmm2d {
namespace {

constexpr int BN = 128;  // binomial table is BN x BN

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

// ---- M2M: one wavefront per parent box, lane l = output coefficient --------
__global__ void __launch_bounds__(64) k_m2m(int l, int p, const double4 *__restrict__ geom, cd *__restrict__ A,
                                            const double *__restrict__ binom) {
    __shared__ cd Ac[64];
    __shared__ cd dp[64];
    __shared__ double sp[64];
    const int64_t P = blockIdx.x;
    const int lane = (int)lane_id();
    const int64_t pbox = level_offset(l) + P;
    const double4 gp = geom[pbox];
    cd acc{0.0, 0.0};
    for (int c = 0; c < 4; ++c) {
        const int64_t cbox = level_offset(l + 1) + 4 * P + c;
        const double4 gc = geom[cbox];
        const cd delta{(gc.x - gp.x) / gp.w, (gc.y - gp.y) / gp.w};
        const double sigma = gc.w / gp.w;
        const cd dpow = wave_powers(delta);
        const double spow = wave_powers_real(sigma);
        if (lane <= p) Ac[lane] = A[cbox * (p + 1) + lane];
        dp[lane] = dpow;
        sp[lane] = spow;
        __syncthreads();
        if (lane <= p) {
            if (lane == 0) {
                acc = cadd(acc, Ac[0]);
            } else {
                cd t = cscale(cmul(Ac[0], dp[lane]), -1.0 / lane);
                for (int k = 1; k <= lane; ++k) {
                    const double coef = sp[k] * binom[(lane - 1) * BN + (k - 1)];
                    t = cadd(t, cscale(cmul(Ac[k], dp[lane - k]), coef));
                }
                acc = cadd(acc, t);
            }
        }
        __syncthreads();
    }
    if (lane <= p) A[pbox * (p + 1) + lane] = acc;
}

// ---- M2L in binary64: one wavefront per target box, lane l = coefficient ---
__global__ void __launch_bounds__(64) k_m2l_fp64(int l, int p, const double4 *__restrict__ geomL,
                                                 const int32_t *__restrict__ wptr, const int32_t *__restrict__ widx,
                                                 const cd *__restrict__ AL, cd *__restrict__ BL,
                                                 const double *__restrict__ binom) {
    __shared__ cd u[64];
    const int64_t b = blockIdx.x;
    const int lane = (int)lane_id();
    const double4 gb = geomL[b];
    cd acc{0.0, 0.0};
    const int32_t t0 = wptr[b], t1 = wptr[b + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const int32_t c = widx[t];
        const double4 gc = geomL[c];
        const cd z0{gc.x - gb.x, gc.y - gb.y};
        const cd rs = cdiv(cd{gc.w, 0.0}, z0);
        const cd rt = cdiv(cd{gb.w, 0.0}, z0);
        const cd ps = wave_powers(rs);
        const cd pt = wave_powers(rt);
        if (lane <= p) u[lane] = cmul(AL[(int64_t)c * (p + 1) + lane], ps);
        __syncthreads();
        if (lane <= p) {
            cd w;
            if (lane == 0) {
                w = cscale(u[0], log(hypot(z0.re, z0.im)));
                for (int k = 1; k <= p; ++k) w = (k & 1) ? csub(w, u[k]) : cadd(w, u[k]);
            } else {
                w = cscale(u[0], -1.0 / lane);
                for (int k = 1; k <= p; ++k) {
                    const double m = ((k & 1) ? -1.0 : 1.0) * binom[(lane + k - 1) * BN + (k - 1)];
                    w = cadd(w, cscale(u[k], m));
                }
            }
            acc = cadd(acc, cmul(pt, w));
        }
        __syncthreads();
    }
    if (lane <= p && t1 > t0) {
        cd *o = BL + b * (p + 1) + lane;
        *o = cadd(*o, acc);
    }
}

// ---- L2L: one wavefront per child box, lane l = coefficient ----------------
__global__ void __launch_bounds__(64) k_l2l(int l, int p, const double4 *__restrict__ geom, cd *__restrict__ B,
                                            const double *__restrict__ binom) {
    __shared__ cd Bp[64];
    __shared__ cd dp[64];
    const int64_t cidx = blockIdx.x;  // child within level l+1
    const int lane = (int)lane_id();
    const int64_t cbox = level_offset(l + 1) + cidx;
    const int64_t pbox = level_offset(l) + (cidx >> 2);
    const double4 gc = geom[cbox], gp = geom[pbox];
    const cd delta{(gc.x - gp.x) / gp.w, (gc.y - gp.y) / gp.w};
    const double tau = gc.w / gp.w;
    const cd dpow = wave_powers(delta);
    const double tpow = wave_powers_real(tau);
    if (lane <= p) Bp[lane] = B[pbox * (p + 1) + lane];
    dp[lane] = dpow;
    __syncthreads();
    if (lane <= p) {
        cd t{0.0, 0.0};
        for (int k = lane; k <= p; ++k) t = cadd(t, cscale(cmul(Bp[k], dp[k - lane]), binom[k * BN + lane]));
        B[cbox * (p + 1) + lane] = cscale(t, tpow);
    }
}

// ---- L2P + near field in binary64: one thread per point --------------------
__global__ void __launch_bounds__(256) k_leaf_fp64(int p, int64_t n, const double *__restrict__ px,
                                                   const double *__restrict__ py, const double *__restrict__ qs,
                                                   const int32_t *__restrict__ leafid, const int32_t *__restrict__ stL,
                                                   const double4 *__restrict__ geomL, const cd *__restrict__ BL,
                                                   const int32_t *__restrict__ sptr, const int32_t *__restrict__ sidx,
                                                   double *__restrict__ phi_leaf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = leafid[i];
    const double4 g = geomL[b];
    const double xi = px[i], yi = py[i];
    const cd z{(xi - g.x) / g.w, (yi - g.y) / g.w};
    const cd *Bb = BL + (int64_t)b * (p + 1);
    cd v = Bb[p];
    for (int l = p - 1; l >= 0; --l) v = cadd(cmul(v, z), Bb[l]);
    double near = 0.0;
    for (int32_t t = sptr[b]; t < sptr[b + 1]; ++t) {
        const int32_t cb = sidx[t];
        for (int32_t j = stL[cb]; j < stL[cb + 1]; ++j) {
            const double dx = xi - px[j], dy = yi - py[j];
            if (dx != 0.0 || dy != 0.0) near += qs[j] * (0.5 * log(dx * dx + dy * dy));
        }
    }
    phi_leaf[i] = v.re + near;
}

__global__ void k_gather_q(const double *__restrict__ q, const int32_t *__restrict__ perm, int64_t n,
                           double *__restrict__ qs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) qs[i] = q[perm[i]];
}

__global__ void k_unpermute(const double *__restrict__ phi_leaf, const int32_t *__restrict__ perm, int64_t n,
                            double *__restrict__ phi) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) phi[perm[i]] = phi_leaf[i];
}

__global__ void k_zero_cd(cd *p, int64_t m) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) p[i] = cd{0.0, 0.0};
}

template <int PB>
hipError_t launch_p2m(fmm2d_ctx *c, int p, cd *A) {
    TreeState &t = c->tree;
    const int64_t nleaf = int64_t(1) << (2 * t.L);
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
// with M2L done by `m2l` (the binary64 kernel or a reduced-precision one).
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
    for (int l = L - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_m2m, dim3((unsigned)(int64_t(1) << (2 * l))), dim3(64), 0, c->stream, l, p,
                           t.geom.as<double4>(), A, binom);
    }
    return hipGetLastError();
}

hipError_t m2l_fp64_level(fmm2d_ctx *c, int l, int p) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t nb = int64_t(1) << (2 * l);
    if (t.w_off[l + 1] == t.w_off[l]) return hipSuccess;
    hipLaunchKernelGGL(k_m2l_fp64, dim3((unsigned)nb), dim3(64), 0, c->stream, l, p,
                       t.geom.as<double4>() + level_offset(l), t.wptr.as<int32_t>() + ptr_offset(l),
                       t.widx.as<int32_t>() + t.w_off[l], e.A.as<cd>() + level_offset(l) * (p + 1),
                       e.B.as<cd>() + level_offset(l) * (p + 1), e.binom.as<double>());
    return hipGetLastError();
}

hipError_t l2l_level(fmm2d_ctx *c, int l, int p) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    hipLaunchKernelGGL(k_l2l, dim3((unsigned)(int64_t(1) << (2 * (l + 1)))), dim3(64), 0, c->stream, l, p,
                       t.geom.as<double4>(), e.B.as<cd>(), e.binom.as<double>());
    return hipGetLastError();
}

hipError_t evaluate_device(fmm2d_ctx *c, const double *q, int p, int mode, double *phi) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t n = t.n;
    const int L = t.L;
    const int64_t nbox = level_offset(L + 1);
    FMM2D_TRY(ensure_binomials(c));
    FMM2D_TRY(e.A.ensure(sizeof(cd) * nbox * (p + 1)));
    FMM2D_TRY(e.B.ensure(sizeof(cd) * nbox * (p + 1)));
    FMM2D_TRY(e.qs.ensure(sizeof(double) * n));
    FMM2D_TRY(e.phi_leaf.ensure(sizeof(double) * n));
    hipLaunchKernelGGL(k_gather_q, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, q, t.perm.as<int32_t>(), n,
                       e.qs.as<double>());
    FMM2D_TRY(upward_pass(c, p));
    hipLaunchKernelGGL(k_zero_cd, dim3(1), dim3(64), 0, c->stream, e.B.as<cd>(), (int64_t)(p + 1));
    for (int l = 0; l <= L; ++l) {
        if (l >= 1) {
            if (mode == FMM2D_MODE_FP64) FMM2D_TRY(m2l_fp64_level(c, l, p));
            else FMM2D_TRY(m2l_reduced_level(c, l, p, mode));
        }
        if (l < L) FMM2D_TRY(l2l_level(c, l, p));
    }
    const int64_t offL = level_offset(L);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const int32_t *sptrL = t.sptr.as<int32_t>() + ptr_offset(L);
    const int32_t *sidxL = t.sidx.as<int32_t>() + t.s_off[L];
    if (mode == FMM2D_MODE_FP64) {
        hipLaunchKernelGGL(k_leaf_fp64, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, p, n, t.px.as<double>(),
                           t.py.as<double>(), e.qs.as<double>(), t.leafid.as<int32_t>(), stL,
                           t.geom.as<double4>() + offL, e.B.as<cd>() + offL * (p + 1), sptrL, sidxL,
                           e.phi_leaf.as<double>());
    } else {
        FMM2D_TRY(leaf_reduced(c, p, mode));
    }
    hipLaunchKernelGGL(k_unpermute, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, e.phi_leaf.as<double>(),
                       t.perm.as<int32_t>(), n, phi);
    return hipGetLastError();
}

}  // namespace fmm2d
