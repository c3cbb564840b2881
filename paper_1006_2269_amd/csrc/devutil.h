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
// a / b, scaled to avoid overflow in |b|^2
__device__ inline cd cdiv(cd a, cd b) {
    double s = fmax(fabs(b.re), fabs(b.im));
    double br = b.re / s, bi = b.im / s;
    double den = br * br + bi * bi;
    double ar = a.re / s, ai = a.im / s;
    return cd{(ar * br + ai * bi) / den, (ai * br - ar * bi) / den};
}

}  // namespace fmm2d
