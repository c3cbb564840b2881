// Reduced-precision hot kernels: M2L along the weak lists and the near field.
//
// Near field: points carry FP32 offsets from their own leaf's centre; for a
// pair of leaves the difference of the two centres is formed in binary64 and
// rounded once, so every FP32 distance is computed from small numbers.
#include "evaluate.h"

namespace fmm2d {
namespace {

constexpr int BN = 128;

__global__ void k_pack_sources(const float2 *__restrict__ loc, const double *__restrict__ qs, int64_t n,
                               float4 *__restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float2 l = loc[i];
        src[i] = make_float4(l.x, l.y, (float)qs[i], 0.0f);
    }
}

// L2P (binary64) plus the FP32 near field: one thread per point.
template <bool ACC64>
__global__ void __launch_bounds__(256) k_leaf_fp32(int p, int64_t n, const double *__restrict__ px,
                                                   const double *__restrict__ py, const float4 *__restrict__ src,
                                                   const int32_t *__restrict__ leafid, const int32_t *__restrict__ stL,
                                                   const double4 *__restrict__ geomL, const cd *__restrict__ BL,
                                                   const int32_t *__restrict__ sptr, const int32_t *__restrict__ sidx,
                                                   double *__restrict__ phi_leaf) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = leafid[i];
    const double4 g = geomL[b];
    const cd z{(px[i] - g.x) / g.w, (py[i] - g.y) / g.w};
    const cd *Bb = BL + (int64_t)b * (p + 1);
    cd v = Bb[p];
    for (int l = p - 1; l >= 0; --l) v = cadd(cmul(v, z), Bb[l]);
    const float4 me = src[i];
    float acc32 = 0.0f;
    double acc64 = 0.0;
    for (int32_t t = sptr[b]; t < sptr[b + 1]; ++t) {
        const int32_t cb = sidx[t];
        const double4 gc = geomL[cb];
        const float xi = me.x + (float)(g.x - gc.x);
        const float yi = me.y + (float)(g.y - gc.y);
        float part = 0.0f;
        for (int32_t j = stL[cb]; j < stL[cb + 1]; ++j) {
            const float4 s = src[j];
            const float dx = xi - s.x, dy = yi - s.y;
            const float r2 = dx * dx + dy * dy;
            part += (r2 > 0.0f) ? s.z * __log2f(r2) : 0.0f;
        }
        if (ACC64) acc64 += (double)part;
        else acc32 += part;
    }
    const double near = ACC64 ? acc64 * 0.34657359027997264 : (double)(acc32 * 0.34657359f);  // ln(2)/2
    phi_leaf[i] = v.re + near;
}

// FP32 M2L on the vector units: one wavefront per target box, lane l.
template <bool POW64>
__global__ void __launch_bounds__(64) k_m2l_fp32(int p, const double4 *__restrict__ geomL,
                                                 const int32_t *__restrict__ wptr, const int32_t *__restrict__ widx,
                                                 const cd *__restrict__ AL, cd *__restrict__ BL,
                                                 const float *__restrict__ M) {
    __shared__ float ur[64], ui[64];
    const int64_t b = blockIdx.x;
    const int lane = (int)lane_id();
    const double4 gb = geomL[b];
    float accr = 0.f, acci = 0.f;
    double accr64 = 0.0, acci64 = 0.0;
    const int32_t t0 = wptr[b], t1 = wptr[b + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const int32_t c = widx[t];
        const double4 gc = geomL[c];
        const cd z0{gc.x - gb.x, gc.y - gb.y};
        const cd rs = cdiv(cd{gc.w, 0.0}, z0);
        const cd rt = cdiv(cd{gb.w, 0.0}, z0);
        // powers rho^k for every lane k by a product scan
        cd ps, pt;
        {
            const uint32_t ln = (uint32_t)lane;
            cd vs = ln == 0 ? cd{1.0, 0.0} : rs, vt = ln == 0 ? cd{1.0, 0.0} : rt;
            if (POW64) {
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    cd us{__shfl_up(vs.re, off, 64), __shfl_up(vs.im, off, 64)};
                    cd ut{__shfl_up(vt.re, off, 64), __shfl_up(vt.im, off, 64)};
                    if (ln >= (uint32_t)off) { vs = cmul(us, vs); vt = cmul(ut, vt); }
                }
            } else {
                float sr = (float)vs.re, si = (float)vs.im, tr = (float)vt.re, ti = (float)vt.im;
#pragma unroll
                for (int off = 1; off < 64; off <<= 1) {
                    float usr = __shfl_up(sr, off, 64), usi = __shfl_up(si, off, 64);
                    float utr = __shfl_up(tr, off, 64), uti = __shfl_up(ti, off, 64);
                    if (ln >= (uint32_t)off) {
                        float a = usr * sr - usi * si; si = usr * si + usi * sr; sr = a;
                        float d = utr * tr - uti * ti; ti = utr * ti + uti * tr; tr = d;
                    }
                }
                vs = cd{sr, si};
                vt = cd{tr, ti};
            }
            ps = vs;
            pt = vt;
        }
        if (lane <= p) {
            const cd a = AL[(int64_t)c * (p + 1) + lane];
            const cd uu = cmul(a, ps);
            ur[lane] = (float)uu.re;
            ui[lane] = (float)uu.im;
        }
        __syncthreads();
        if (lane <= p) {
            float wr = 0.f, wi = 0.f;
            for (int k = 0; k <= p; ++k) {
                const float m = M[lane * 64 + k];
                wr += m * ur[k];
                wi += m * ui[k];
            }
            if (lane == 0) {
                const float lg = (float)log(hypot(z0.re, z0.im));
                wr += ur[0] * lg;
                wi += ui[0] * lg;
            }
            if (POW64) {
                accr64 += pt.re * wr - pt.im * wi;
                acci64 += pt.re * wi + pt.im * wr;
            } else {
                const float ptr = (float)pt.re, pti = (float)pt.im;
                accr += ptr * wr - pti * wi;
                acci += ptr * wi + pti * wr;
            }
        }
        __syncthreads();
    }
    if (lane <= p && t1 > t0) {
        cd *o = BL + b * (p + 1) + lane;
        if (POW64) *o = cadd(*o, cd{accr64, acci64});
        else *o = cadd(*o, cd{(double)accr, (double)acci});
    }
}

// The constant M2L matrix in FP32: M[l][k], row l, column k (64 x 64).
__global__ void k_make_M(float *M, const double *binom) {
    const int l = blockIdx.x, k = threadIdx.x;
    double m;
    if (l == 0) m = (k == 0) ? 0.0 : ((k & 1) ? -1.0 : 1.0);
    else if (k == 0) m = -1.0 / l;
    else m = ((k & 1) ? -1.0 : 1.0) * binom[(l + k - 1) * BN + (k - 1)];
    M[l * 64 + k] = (float)m;
}

}  // namespace

hipError_t m2l_reduced_level(fmm2d_ctx *c, int l, int p, int mode) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    if (t.w_off[l + 1] == t.w_off[l]) return hipSuccess;
    FMM2D_TRY(e.work.ensure(sizeof(float) * 64 * 64));
    float *M = e.work.as<float>();
    hipLaunchKernelGGL(k_make_M, dim3(64), dim3(64), 0, c->stream, M, e.binom.as<double>());
    const int64_t nb = int64_t(1) << (2 * l);
    const double4 *gL = t.geom.as<double4>() + level_offset(l);
    const int32_t *wp = t.wptr.as<int32_t>() + ptr_offset(l);
    const int32_t *wi = t.widx.as<int32_t>() + t.w_off[l];
    const cd *AL = e.A.as<cd>() + level_offset(l) * (p + 1);
    cd *BL = e.B.as<cd>() + level_offset(l) * (p + 1);
    if (mode == FMM2D_MODE_FP32_ACC64)
        hipLaunchKernelGGL(k_m2l_fp32<true>, dim3((unsigned)nb), dim3(64), 0, c->stream, p, gL, wp, wi, AL, BL, M);
    else
        hipLaunchKernelGGL(k_m2l_fp32<false>, dim3((unsigned)nb), dim3(64), 0, c->stream, p, gL, wp, wi, AL, BL, M);
    return hipGetLastError();
}

hipError_t leaf_reduced(fmm2d_ctx *c, int p, int mode) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t n = t.n;
    const int L = t.L;
    const int64_t offL = level_offset(L);
    FMM2D_TRY(e.src.ensure(sizeof(float4) * n));
    hipLaunchKernelGGL(k_pack_sources, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, t.loc.as<float2>(),
                       e.qs.as<double>(), n, e.src.as<float4>());
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const int32_t *sptrL = t.sptr.as<int32_t>() + ptr_offset(L);
    const int32_t *sidxL = t.sidx.as<int32_t>() + t.s_off[L];
    if (mode == FMM2D_MODE_FP32_ACC64)
        hipLaunchKernelGGL(k_leaf_fp32<true>, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, p, n,
                           t.px.as<double>(), t.py.as<double>(), e.src.as<float4>(), t.leafid.as<int32_t>(), stL,
                           t.geom.as<double4>() + offL, e.B.as<cd>() + offL * (p + 1), sptrL, sidxL,
                           e.phi_leaf.as<double>());
    else
        hipLaunchKernelGGL(k_leaf_fp32<false>, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, p, n,
                           t.px.as<double>(), t.py.as<double>(), e.src.as<float4>(), t.leafid.as<int32_t>(), stL,
                           t.geom.as<double4>() + offL, e.B.as<cd>() + offL * (p + 1), sptrL, sidxL,
                           e.phi_leaf.as<double>());
    return hipGetLastError();
}

}  // namespace fmm2d
