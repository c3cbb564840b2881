// Exclusive prefix sum of an int32 array: out[i] = sum_{j<i} in[j], out[n] = total.
// Reduce-then-scan over tiles of 4096 elements.
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;

__global__ void __launch_bounds__(SC_THREADS) k_tile_sums(const int32_t *__restrict__ in, int64_t n,
                                                          int32_t *__restrict__ tsum) {
    __shared__ int32_t tmp[SC_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * SC_TILE;
    int32_t s = 0;
    for (int r = 0; r < SC_ITEMS; ++r) {
        int64_t i = base + (int64_t)r * SC_THREADS + threadIdx.x;
        if (i < n) s += in[i];
    }
    int32_t ws = wave_sum(s);
    if (lane_id() == 0) tmp[threadIdx.x / 64] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int k = 0; k < SC_THREADS / 64; ++k) t += tmp[k];
        tsum[blockIdx.x] = t;
    }
}

// Single block: exclusive scan of m values in place, total to v[m].
__global__ void __launch_bounds__(1024) k_scan_small(int32_t *__restrict__ v, int64_t m) {
    __shared__ int32_t tmp[1024 / 64];
    int64_t per = (m + 1023) / 1024;
    int64_t b0 = (int64_t)threadIdx.x * per;
    int32_t s = 0;
    for (int64_t i = b0; i < b0 + per && i < m; ++i) s += v[i];
    int32_t total;
    int32_t run = block_excl_scan<1024>(s, tmp, total);
    for (int64_t i = b0; i < b0 + per && i < m; ++i) {
        int32_t c = v[i];
        v[i] = run;
        run += c;
    }
    if (threadIdx.x == 0) v[m] = total;
}

__global__ void __launch_bounds__(SC_THREADS) k_tile_scan(const int32_t *__restrict__ in, int64_t n,
                                                          const int32_t *__restrict__ tpre, int32_t *__restrict__ out,
                                                          int nblk) {
    __shared__ int32_t tmp[SC_THREADS / 64];
    int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    int32_t vals[SC_ITEMS];
    int32_t s = 0;
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r) {
        int64_t i = base + r;
        vals[r] = (i < n) ? in[i] : 0;
        s += vals[r];
    }
    int32_t total;
    int32_t run = tpre[blockIdx.x] + block_excl_scan<SC_THREADS>(s, tmp, total);
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r) {
        int64_t i = base + r;
        if (i < n) out[i] = run;
        run += vals[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tpre[nblk];
}

}  // namespace

hipError_t scan_exclusive(fmm2d_ctx *c, const int32_t *in, int64_t n, int32_t *out) {
    const int nblk = (int)((n + SC_TILE - 1) / SC_TILE);
    FMM2D_TRY(c->scr.tiles.ensure(sizeof(int32_t) * (nblk + 1)));
    int32_t *t = c->scr.tiles.as<int32_t>();
    if (n == 0) {
        FMM2D_TRY(hipMemsetAsync(out, 0, sizeof(int32_t), c->stream));
        return hipSuccess;
    }
    hipLaunchKernelGGL(k_tile_sums, dim3(nblk), dim3(SC_THREADS), 0, c->stream, in, n, t);
    hipLaunchKernelGGL(k_scan_small, dim3(1), dim3(1024), 0, c->stream, t, (int64_t)nblk);
    hipLaunchKernelGGL(k_tile_scan, dim3(nblk), dim3(SC_THREADS), 0, c->stream, in, n, t, out, nblk);
    return hipGetLastError();
}

}  // namespace fmm2d
