// Stable LSD radix sort of binary64 values with their original indices.
//
// Sorting a coordinate with its index as the value, stably, yields the order
// by the pair (coordinate, index): the key with which every box of the tree
// is split at its median.  Keys are the usual order-preserving map of an IEEE
// double to uint64 (after -0.0 is folded onto +0.0, so that equal values tie).
// 8-bit digits, three kernels per pass (tile histogram, digit-major scan of
// the tile histograms, stable rank-and-scatter).  Digits on which all keys
// agree are found first (one AND/OR reduction) and their passes are skipped.
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 16;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;
constexpr int RADIX = 256;

__device__ inline uint64_t to_key(double v) {
    v = v + 0.0;  // -0.0 -> +0.0
    uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double from_key(uint64_t k) {
    uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
}

__device__ inline uint64_t lanemask_lt_popc(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Lanes of this wave whose 8-bit digit equals mine (restricted to `valid`).
__device__ inline uint64_t match_digit(uint32_t d, uint64_t valid) {
    uint64_t peers = valid;
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        uint64_t m = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? m : ~m;
    }
    return peers;
}

__global__ void k_make_keys(const double *__restrict__ v, int64_t n, uint64_t *__restrict__ keys,
                            int32_t *__restrict__ vals, unsigned long long *andor) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t ka = ~0ull, ko = 0ull;
    if (i < n) {
        uint64_t k = to_key(v[i]);
        keys[i] = k;
        vals[i] = (int32_t)i;
        ka = k;
        ko = k;
    }
    for (int off = 32; off > 0; off >>= 1) {
        ka &= (uint64_t)__shfl_xor((unsigned long long)ka, off);
        ko |= (uint64_t)__shfl_xor((unsigned long long)ko, off);
    }
    if ((threadIdx.x & 63) == 0) {
        atomicAnd(&andor[0], (unsigned long long)ka);
        atomicOr(&andor[1], (unsigned long long)ko);
    }
}

__global__ void k_init_andor(unsigned long long *andor) {
    andor[0] = ~0ull;
    andor[1] = 0ull;
}

__global__ void __launch_bounds__(SORT_THREADS) k_hist(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                                       int32_t *__restrict__ hist, int nblk) {
    __shared__ int32_t h[RADIX];
    h[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        int64_t i = base + (int64_t)r * SORT_THREADS + threadIdx.x;
        bool ok = i < n;
        uint32_t d = ok ? (uint32_t)((keys[i] >> shift) & 0xff) : 0u;
        uint64_t valid = __ballot(ok);
        uint64_t peers = match_digit(d, valid);
        if (ok && lanemask_lt_popc(peers) == 0) atomicAdd(&h[d], (int32_t)__popcll(peers));
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// One block per digit: total count of that digit over all tiles.
__global__ void __launch_bounds__(256) k_digit_totals(const int32_t *__restrict__ hist, int nblk,
                                                      int32_t *__restrict__ tot) {
    __shared__ int32_t red[256];
    int d = blockIdx.x;
    int32_t s = 0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += hist[(int64_t)d * nblk + b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) tot[d] = red[0];
}

// One block per digit: exclusive scan of hist[d][*] plus the digit's base.
__global__ void __launch_bounds__(256) k_digit_scan(int32_t *__restrict__ hist, int nblk,
                                                    const int32_t *__restrict__ tot) {
    __shared__ int32_t part[256];
    __shared__ int32_t base_s;
    int d = blockIdx.x;
    if (threadIdx.x == 0) {
        int32_t b = 0;
        for (int e = 0; e < d; ++e) b += tot[e];
        base_s = b;
    }
    int per = (nblk + 255) / 256;
    int b0 = threadIdx.x * per;
    int32_t s = 0;
    for (int b = b0; b < b0 + per && b < nblk; ++b) s += hist[(int64_t)d * nblk + b];
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan over the 256 partial sums
    for (int off = 1; off < 256; off <<= 1) {
        int32_t v = (threadIdx.x >= off) ? part[threadIdx.x - off] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int32_t run = base_s + ((threadIdx.x > 0) ? part[threadIdx.x - 1] : 0);
    for (int b = b0; b < b0 + per && b < nblk; ++b) {
        int32_t c = hist[(int64_t)d * nblk + b];
        hist[(int64_t)d * nblk + b] = run;
        run += c;
    }
}

__global__ void __launch_bounds__(SORT_THREADS) k_scatter(const uint64_t *__restrict__ kin, const int32_t *__restrict__ vin,
                                                          uint64_t *__restrict__ kout, int32_t *__restrict__ vout,
                                                          int64_t n, int shift, const int32_t *__restrict__ hist,
                                                          int nblk) {
    constexpr int NW = SORT_THREADS / WAVE;
    __shared__ int32_t gbase[RADIX];
    __shared__ int32_t running[RADIX];
    __shared__ int32_t wcnt[NW][RADIX];
    const int t = threadIdx.x, w = t / WAVE;
    gbase[t] = hist[(int64_t)t * nblk + blockIdx.x];
    running[t] = 0;
    for (int k = 0; k < NW; ++k) wcnt[k][t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    for (int r = 0; r < SORT_ITEMS; ++r) {
        int64_t i = base + (int64_t)r * SORT_THREADS + t;
        bool ok = i < n;
        uint64_t k = ok ? kin[i] : 0ull;
        int32_t v = ok ? vin[i] : 0;
        uint32_t d = (uint32_t)((k >> shift) & 0xff);
        uint64_t valid = __ballot(ok);
        uint64_t peers = match_digit(d, valid);
        int32_t rank = (int32_t)lanemask_lt_popc(peers);
        if (ok && rank == 0) wcnt[w][d] = (int32_t)__popcll(peers);
        __syncthreads();
        if (ok) {
            int32_t off = running[d] + rank;
            for (int q = 0; q < w; ++q) off += wcnt[q][d];
            int64_t dst = (int64_t)gbase[d] + off;
            kout[dst] = k;
            vout[dst] = v;
        }
        __syncthreads();
        int32_t add = 0;
        for (int q = 0; q < NW; ++q) { add += wcnt[q][t]; wcnt[q][t] = 0; }
        running[t] += add;
        __syncthreads();
    }
}

__global__ void k_finish(const uint64_t *__restrict__ keys, const int32_t *__restrict__ vals, int64_t n,
                         double *__restrict__ sorted, int32_t *__restrict__ order) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        sorted[i] = from_key(keys[i]);
        order[i] = vals[i];
    }
}

}  // namespace

hipError_t sort_coordinate(fmm2d_ctx *c, const double *v, int64_t n, double *sorted, int32_t *order) {
    Scratch &s = c->scr;
    const int nblk = (int)((n + SORT_TILE - 1) / SORT_TILE);
    FMM2D_TRY(s.keys0.ensure(sizeof(uint64_t) * n));
    FMM2D_TRY(s.keys1.ensure(sizeof(uint64_t) * n));
    FMM2D_TRY(s.vals0.ensure(sizeof(int32_t) * n));
    FMM2D_TRY(s.vals1.ensure(sizeof(int32_t) * n));
    FMM2D_TRY(s.hist.ensure(sizeof(int32_t) * (size_t)RADIX * nblk));
    FMM2D_TRY(s.aux.ensure(4096));
    unsigned long long *andor = s.aux.as<unsigned long long>();
    int32_t *tot = reinterpret_cast<int32_t *>(andor + 4);
    hipLaunchKernelGGL(k_init_andor, dim3(1), dim3(1), 0, c->stream, andor);
    hipLaunchKernelGGL(k_make_keys, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, v, n,
                       s.keys0.as<uint64_t>(), s.vals0.as<int32_t>(), andor);
    FMM2D_TRY(hipGetLastError());
    unsigned long long h_andor[2];
    FMM2D_TRY(hipMemcpyAsync(h_andor, andor, sizeof(h_andor), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    const uint64_t differ = (uint64_t)(h_andor[0] ^ h_andor[1]);

    uint64_t *kin = s.keys0.as<uint64_t>(), *kout = s.keys1.as<uint64_t>();
    int32_t *vin = s.vals0.as<int32_t>(), *vout = s.vals1.as<int32_t>();
    for (int shift = 0; shift < 64; shift += 8) {
        if (((differ >> shift) & 0xffull) == 0) continue;
        hipLaunchKernelGGL(k_hist, dim3(nblk), dim3(SORT_THREADS), 0, c->stream, kin, n, shift,
                           s.hist.as<int32_t>(), nblk);
        hipLaunchKernelGGL(k_digit_totals, dim3(RADIX), dim3(256), 0, c->stream, s.hist.as<int32_t>(), nblk, tot);
        hipLaunchKernelGGL(k_digit_scan, dim3(RADIX), dim3(256), 0, c->stream, s.hist.as<int32_t>(), nblk, tot);
        hipLaunchKernelGGL(k_scatter, dim3(nblk), dim3(SORT_THREADS), 0, c->stream, kin, vin, kout, vout, n, shift,
                           s.hist.as<int32_t>(), nblk);
        FMM2D_TRY(hipGetLastError());
        uint64_t *tk = kin; kin = kout; kout = tk;
        int32_t *tv = vin; vin = vout; vout = tv;
    }
    hipLaunchKernelGGL(k_finish, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, kin, vin, n, sorted, order);
    return hipGetLastError();
}

}  // namespace fmm2d
