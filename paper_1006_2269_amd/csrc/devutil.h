// Device helpers shared by the kernels (wave64 scans, lane masks, complex math).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fmm2d {

__device__ inline uint32_t lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// number of set bits of m strictly below this lane
__device__ inline uint32_t popc_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// inclusive prefix sum over the 64 lanes of a wave
__device__ inline int32_t wave_incl_scan(int32_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        int32_t u = __shfl_up(v, off, 64);
        if (lane >= (uint32_t)off) v += u;
    }
    return v;
}

__device__ inline int32_t wave_sum(int32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Exclusive prefix sum over a block of NT threads (NT a multiple of 64);
// `total` receives the block sum.  Uses `tmp` (NT/64 ints of LDS).
template <int NT>
__device__ inline int32_t block_excl_scan(int32_t v, int32_t *tmp, int32_t &total) {
    const int w = threadIdx.x / 64;
    const uint32_t lane = lane_id();
    int32_t inc = wave_incl_scan(v);
    if (lane == 63) tmp[w] = inc;
    __syncthreads();
    int32_t before = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k) {
        int32_t s = tmp[k];
        before += (k < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + inc - v;
}

// ---- binary64 complex helpers ---------------------------------------------
struct cd {
    double re, im;
};
__device__ __host__ inline cd cmk(double r, double i) { return cd{r, i}; }
__device__ inline cd cadd(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ inline cd csub(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ inline cd cmul(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cd cscale(cd a, double s) { return cd{a.re * s, a.im * s}; }
// a b + c in four fused multiply-adds (a Horner step)
__device__ inline cd cfma(cd a, cd b, cd c) {
    return cd{fma(a.re, b.re, fma(-a.im, b.im, c.re)), fma(a.re, b.im, fma(a.im, b.re, c.im))};
}
// Natural logarithm of a finite x > 0 in binary64, within a few ulp.  With
// x = m 2^e, m in [sqrt(1/2), sqrt(2)):  log x = e log 2 + 2 atanh(s),
// s = (m - 1) / (m + 1), |s| <= 3 - 2 sqrt(2), and the series
// atanh s = s + s^3/3 + s^5/5 + ... cut after s^19 (the rest is below
// 2.5e-17 of the sum).  m - 1 is exact; 1 / (m + 1) comes from the hardware
// reciprocal and two Newton steps.  About half the instructions of the
// correctly rounded library form, the bulk of a binary64 pair interaction.
__device__ inline double log_pos(double x) {
    int e;
    double m = frexp(x, &e);  // [1/2, 1)
    if (m < 0x1.6a09e667f3bcdp-1) {
        m += m;
        --e;
    }
    const double den = m + 1.0;
    double r = __builtin_amdgcn_rcp(den);
    r = fma(r, fma(-den, r, 1.0), r);
    r = fma(r, fma(-den, r, 1.0), r);
    const double s = (m - 1.0) * r, t = s * s;
    double q = 1.0 / 19.0;
    q = fma(q, t, 1.0 / 17.0);
    q = fma(q, t, 1.0 / 15.0);
    q = fma(q, t, 1.0 / 13.0);
    q = fma(q, t, 1.0 / 11.0);
    q = fma(q, t, 1.0 / 9.0);
    q = fma(q, t, 1.0 / 7.0);
    q = fma(q, t, 1.0 / 5.0);
    q = fma(q, t, 1.0 / 3.0);
    const double s2 = s + s;
    return fma((double)e, 0x1.62e42fefa39efp-1, fma(s2 * t, q, s2));  // the double nearest log 2
}

// a / b, scaled to avoid overflow in |b|^2
__device__ inline cd cdiv(cd a, cd b) {
    double s = fmax(fabs(b.re), fabs(b.im));
    double br = b.re / s, bi = b.im / s;
    double den = br * br + bi * bi;
    double ar = a.re / s, ai = a.im / s;
    return cd{(ar * br + ai * bi) / den, (ai * br - ar * bi) / den};
}

}  // namespace fmm2d
