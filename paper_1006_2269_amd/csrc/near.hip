// Near field at the finest level (the direct sum over the strong lists,
// Section 4) fused with L2P, in binary64 or FP32.
//
// One wavefront per work item (target leaf b, chunk of TM consecutive points
// of b).  The targets are uniform across the wave; the lanes spread over the
// source points of S(b): GL lanes per source leaf (GL >= the largest leaf),
// 64/GL source leaves per step, so each lane loads one source and evaluates
// it against all TM targets held in registers.  A butterfly reduction then
// gives each target's sum, in a fixed order.  Every lane of a wave walks the
// same strong list, so the loop bounds are uniform.
//
// FP32 path: targets and sources are offsets from their own leaf centres;
// the centre difference c_b - c_c is formed in binary64 and rounded once per
// (lane, source leaf).  A pair whose FP32 distance is below the rounding
// error of that computation (2^-20 of the magnitudes involved) is treated as
// coincident, which makes exactly coincident points in different leaves
// contribute nothing, as in binary64.  L2P (binary64 Horner) runs on lane k
// for target k.
#include "evaluate.h"

namespace fmm2d {
namespace {

constexpr double HALF_LN2_D = 0.34657359027997264;  // ln(2)/2
constexpr int NWB = 4;                                // wavefronts per block

template <int TM, int GL, bool ACC64>
__global__ void __launch_bounds__(64 * NWB) k_near32(int p, int64_t nitems, int chunks, int maxleaf,
                                                     const int32_t *__restrict__ stL,
                                                     const double4 *__restrict__ geomL, const float4 *__restrict__ src,
                                                     const double *__restrict__ px, const double *__restrict__ py,
                                                     const cd *__restrict__ BL, const int32_t *__restrict__ sptr,
                                                     const int32_t *__restrict__ sidx, double *__restrict__ phi_leaf) {
    constexpr int LPI = 64 / GL;  // source leaves per step
    const int64_t item = (int64_t)blockIdx.x * NWB + threadIdx.x / 64;
    if (item >= nitems) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int64_t b = item / chunks;
    const int ch = (int)(item - b * chunks);
    const int32_t le = stL[b + 1];
    const int32_t a = stL[b] + ch * TM;
    if (a >= le) return;
    const int nt = (le - a) < TM ? (le - a) : TM;
    const double4 g = geomL[b];
    float tx[TM], ty[TM], acc[TM];
    double acc64[TM];
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const float4 s = src[a + (k < nt ? k : 0)];
        tx[k] = s.x;
        ty[k] = s.y;
        acc[k] = 0.f;
        acc64[k] = 0.0;
    }
    const int grp = lane / GL, jj = lane % GL;
    const int32_t t0 = sptr[b], t1 = sptr[b + 1];
    int step = 0;
    for (int32_t t = t0; t < t1; t += LPI, ++step) {
        const int32_t tt = t + grp;
        const bool leaf_ok = tt < t1;
        const int32_t c = sidx[leaf_ok ? tt : t0];
        const double4 gc = geomL[c];
        const float dxc = (float)(g.x - gc.x), dyc = (float)(g.y - gc.y);
        const float mag = fabsf(dxc) + fabsf(dyc) + (float)g.z + (float)gc.z;
        const float thr = (mag * 0x1p-20f) * (mag * 0x1p-20f);
        const int32_t j0 = stL[c], j1 = stL[c + 1];
        for (int jb = 0; jb < maxleaf; jb += GL) {
            const int32_t j = j0 + jb + jj;
            float sx = 1e18f, sy = 1e18f, q = 0.f;
            if (leaf_ok && j < j1) {
                const float4 s = src[j];
                sx = s.x - dxc;
                sy = s.y - dyc;
                q = s.z;
            }
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                const float dx = tx[k] - sx, dy = ty[k] - sy;
                const float r2 = dx * dx + dy * dy;
                const float lg = __log2f(r2);
                acc[k] += (r2 > thr) ? q * lg : 0.f;
            }
        }
        if (ACC64 && (step & 3) == 3) {
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                acc64[k] += (double)acc[k];
                acc[k] = 0.f;
            }
        }
    }
    double mine = 0.0;
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        double v;
        if (ACC64) {
            v = acc64[k] + (double)acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        } else {
            float w = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
            v = (double)w;
        }
        if (lane == k) mine = v;
    }
    if (lane < nt) {
        const int32_t i = a + lane;
        const cd z{(px[i] - g.x) / g.w, (py[i] - g.y) / g.w};
        const cd *Bb = BL + b * (p + 1);
        cd v = Bb[p];
        for (int l = p - 1; l >= 0; --l) v = cadd(cmul(v, z), Bb[l]);
        phi_leaf[i] = v.re + mine * HALF_LN2_D;
    }
}

template <int TM, int GL>
__global__ void __launch_bounds__(64 * NWB) k_near64(int p, int64_t nitems, int chunks, int maxleaf,
                                                     const int32_t *__restrict__ stL,
                                                     const double4 *__restrict__ geomL, const double *__restrict__ px,
                                                     const double *__restrict__ py, const double *__restrict__ qs,
                                                     const cd *__restrict__ BL, const int32_t *__restrict__ sptr,
                                                     const int32_t *__restrict__ sidx, double *__restrict__ phi_leaf) {
    constexpr int LPI = 64 / GL;
    const int64_t item = (int64_t)blockIdx.x * NWB + threadIdx.x / 64;
    if (item >= nitems) return;
    const int lane = threadIdx.x % 64;
    const int64_t b = item / chunks;
    const int ch = (int)(item - b * chunks);
    const int32_t le = stL[b + 1];
    const int32_t a = stL[b] + ch * TM;
    if (a >= le) return;
    const int nt = (le - a) < TM ? (le - a) : TM;
    double tx[TM], ty[TM], acc[TM];
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const int32_t i = a + (k < nt ? k : 0);
        tx[k] = px[i];
        ty[k] = py[i];
        acc[k] = 0.0;
    }
    const int grp = lane / GL, jj = lane % GL;
    const int32_t t0 = sptr[b], t1 = sptr[b + 1];
    for (int32_t t = t0; t < t1; t += LPI) {
        const int32_t tt = t + grp;
        const bool leaf_ok = tt < t1;
        const int32_t c = sidx[leaf_ok ? tt : t0];
        const int32_t j0 = stL[c], j1 = stL[c + 1];
        for (int jb = 0; jb < maxleaf; jb += GL) {
            const int32_t j = j0 + jb + jj;
            const bool ok = leaf_ok && j < j1;
            double sx = 1e300, sy = 1e300, q = 0.0;
            if (ok) {
                sx = px[j];
                sy = py[j];
                q = qs[j];
            }
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                const double dx = tx[k] - sx, dy = ty[k] - sy;
                acc[k] += (ok && (dx != 0.0 || dy != 0.0)) ? q * log(dx * dx + dy * dy) : 0.0;
            }
        }
    }
    double mine = 0.0;
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == k) mine = v;
    }
    if (lane < nt) {
        const int32_t i = a + lane;
        const double4 g = geomL[b];
        const cd z{(px[i] - g.x) / g.w, (py[i] - g.y) / g.w};
        const cd *Bb = BL + b * (p + 1);
        cd v = Bb[p];
        for (int l = p - 1; l >= 0; --l) v = cadd(cmul(v, z), Bb[l]);
        phi_leaf[i] = v.re + 0.5 * mine;
    }
}

__global__ void k_pack_sources(const float2 *__restrict__ loc, const double *__restrict__ qs, int64_t n,
                               float4 *__restrict__ src) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float2 l = loc[i];
        src[i] = make_float4(l.x, l.y, (float)qs[i], 0.0f);
    }
}

template <int TM, int GL>
hipError_t launch_near(fmm2d_ctx *c, int p, int mode, int maxleaf) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const int chunks = (maxleaf + TM - 1) / TM;
    const int64_t nitems = nleaf * chunks;
    const int64_t offL = level_offset(L);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const double4 *gL = t.geom.as<double4>() + offL;
    const cd *BL = e.B.as<cd>() + offL * (p + 1);
    const int32_t *sp = t.sptr.as<int32_t>() + ptr_offset(L);
    const int32_t *si = t.sidx.as<int32_t>() + t.s_off[L];
    const dim3 grid(grid_for(nitems, NWB)), block(64 * NWB);
    if (mode == FMM2D_MODE_FP64) {
        hipLaunchKernelGGL((k_near64<TM, GL>), grid, block, 0, c->stream, p, nitems, chunks, maxleaf, stL, gL,
                           t.px.as<double>(), t.py.as<double>(), e.qs.as<double>(), BL, sp, si,
                           e.phi_leaf.as<double>());
    } else if (mode == FMM2D_MODE_FP32_ACC64) {
        hipLaunchKernelGGL((k_near32<TM, GL, true>), grid, block, 0, c->stream, p, nitems, chunks, maxleaf, stL, gL,
                           e.src.as<float4>(), t.px.as<double>(), t.py.as<double>(), BL, sp, si,
                           e.phi_leaf.as<double>());
    } else {
        hipLaunchKernelGGL((k_near32<TM, GL, false>), grid, block, 0, c->stream, p, nitems, chunks, maxleaf, stL, gL,
                           e.src.as<float4>(), t.px.as<double>(), t.py.as<double>(), BL, sp, si,
                           e.phi_leaf.as<double>());
    }
    return hipGetLastError();
}

}  // namespace

// L2P plus the near field for every point; writes ev.phi_leaf (leaf order).
hipError_t leaf_pass(fmm2d_ctx *c, int p, int mode) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t n = t.n;
    const int64_t maxleaf = (n + (int64_t(1) << (2 * t.L)) - 1) >> (2 * t.L);  // ceil(n / 4^L)
    if (mode != FMM2D_MODE_FP64) {
        FMM2D_TRY(e.src.ensure(sizeof(float4) * n));
        hipLaunchKernelGGL(k_pack_sources, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, t.loc.as<float2>(),
                           e.qs.as<double>(), n, e.src.as<float4>());
    }
    // GL lanes per source leaf: the smallest power of two >= the largest leaf,
    // capped at 64 (larger leaves are walked GL points at a time)
    const int ml = (int)(maxleaf < (int64_t)1 << 30 ? maxleaf : (int64_t)1 << 30);
    if (ml <= 8) return launch_near<8, 8>(c, p, mode, ml);
    if (ml <= 16) return launch_near<16, 16>(c, p, mode, ml);
    if (ml <= 32) return launch_near<16, 32>(c, p, mode, ml);
    return launch_near<16, 64>(c, p, mode, ml);
}

}  // namespace fmm2d
