// Exclusive prefix sums of int32 arrays: out[i] = sum_{j<i} in[j], out[n] =
// total.  Up to two arrays of one length are scanned by the same launches
// (blockIdx.y selects the array).  Arrays of at most 16384 elements take one
// single-block kernel; longer ones reduce-then-scan over tiles of 4096.
// In place (out == in) is allowed.
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 16;
constexpr int SC_TILE = SC_THREADS * SC_ITEMS;
constexpr int ONE_THREADS = 1024;
constexpr int ONE_ITEMS = 16;
constexpr int64_t ONE_MAX = (int64_t)ONE_THREADS * ONE_ITEMS;

struct ScanArgs {
    const int32_t *in[2];
    int32_t *out[2];
    int32_t *tiles[2];
};

// n <= ONE_MAX: each thread owns ONE_ITEMS consecutive elements, which it
// reads before any thread writes.
__global__ void __launch_bounds__(ONE_THREADS) k_scan_one_block(ScanArgs a, int64_t n) {
    __shared__ int32_t tmp[ONE_THREADS / 64];
    const int32_t *in = a.in[blockIdx.y];
    int32_t *out = a.out[blockIdx.y];
    const int64_t b0 = (int64_t)threadIdx.x * ONE_ITEMS;
    int32_t v[ONE_ITEMS], s = 0;
#pragma unroll
    for (int r = 0; r < ONE_ITEMS; ++r) {
        v[r] = (b0 + r < n) ? in[b0 + r] : 0;
        s += v[r];
    }
    int32_t total;
    int32_t run = block_excl_scan<ONE_THREADS>(s, tmp, total);
#pragma unroll
    for (int r = 0; r < ONE_ITEMS; ++r) {
        if (b0 + r < n) out[b0 + r] = run;
        run += v[r];
    }
    if (threadIdx.x == 0) out[n] = total;
}

__global__ void __launch_bounds__(SC_THREADS) k_tile_sums(ScanArgs a, int64_t n) {
    __shared__ int32_t tmp[SC_THREADS / 64];
    const int32_t *in = a.in[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    int32_t s = 0;
    for (int r = 0; r < SC_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * SC_THREADS + threadIdx.x;
        if (i < n) s += in[i];
    }
    const int32_t ws = wave_sum(s);
    if (lane_id() == 0) tmp[threadIdx.x / 64] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        int32_t t = 0;
        for (int k = 0; k < SC_THREADS / 64; ++k) t += tmp[k];
        a.tiles[blockIdx.y][blockIdx.x] = t;
    }
}

// Single block per array: exclusive scan of m tile sums in place, total to v[m].
__global__ void __launch_bounds__(1024) k_scan_small(ScanArgs a, int64_t m) {
    __shared__ int32_t tmp[1024 / 64];
    int32_t *v = a.tiles[blockIdx.y];
    const int64_t per = (m + 1023) / 1024;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    int32_t s = 0;
    for (int64_t i = b0; i < b0 + per && i < m; ++i) s += v[i];
    int32_t total;
    int32_t run = block_excl_scan<1024>(s, tmp, total);
    for (int64_t i = b0; i < b0 + per && i < m; ++i) {
        const int32_t c = v[i];
        v[i] = run;
        run += c;
    }
    if (threadIdx.x == 0) v[m] = total;
}

__global__ void __launch_bounds__(SC_THREADS) k_tile_scan(ScanArgs a, int64_t n, int nblk) {
    __shared__ int32_t tmp[SC_THREADS / 64];
    const int32_t *in = a.in[blockIdx.y];
    int32_t *out = a.out[blockIdx.y];
    const int32_t *tpre = a.tiles[blockIdx.y];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    int32_t vals[SC_ITEMS];
    int32_t s = 0;
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r) {
        const int64_t i = base + r;
        vals[r] = (i < n) ? in[i] : 0;
        s += vals[r];
    }
    int32_t total;
    int32_t run = tpre[blockIdx.x] + block_excl_scan<SC_THREADS>(s, tmp, total);
#pragma unroll
    for (int r = 0; r < SC_ITEMS; ++r) {
        const int64_t i = base + r;
        if (i < n) out[i] = run;
        run += vals[r];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tpre[nblk];
}

__global__ void k_zero_totals(ScanArgs a) { a.out[blockIdx.x][0] = 0; }

}  // namespace

hipError_t scan_exclusive_n(fmm2d_ctx *c, int k, const int32_t *const *in, int64_t n, int32_t *const *out) {
    if (k < 1 || k > 2) return hipErrorInvalidValue;
    ScanArgs a{};
    for (int j = 0; j < k; ++j) {
        a.in[j] = in[j];
        a.out[j] = out[j];
    }
    if (n == 0) {
        hipLaunchKernelGGL(k_zero_totals, dim3(k), dim3(1), 0, c->stream, a);
        return hipGetLastError();
    }
    if (n <= ONE_MAX) {
        hipLaunchKernelGGL(k_scan_one_block, dim3(1, k), dim3(ONE_THREADS), 0, c->stream, a, n);
        return hipGetLastError();
    }
    const int nblk = (int)((n + SC_TILE - 1) / SC_TILE);
    FMM2D_TRY(c->scr.tiles.ensure(sizeof(int32_t) * 2 * (nblk + 1)));
    for (int j = 0; j < k; ++j) a.tiles[j] = c->scr.tiles.as<int32_t>() + j * (nblk + 1);
    hipLaunchKernelGGL(k_tile_sums, dim3(nblk, k), dim3(SC_THREADS), 0, c->stream, a, n);
    hipLaunchKernelGGL(k_scan_small, dim3(1, k), dim3(1024), 0, c->stream, a, (int64_t)nblk);
    hipLaunchKernelGGL(k_tile_scan, dim3(nblk, k), dim3(SC_THREADS), 0, c->stream, a, n, nblk);
    return hipGetLastError();
}

hipError_t scan_exclusive(fmm2d_ctx *c, const int32_t *in, int64_t n, int32_t *out) {
    return scan_exclusive_n(c, 1, &in, n, &out);
}

}  // namespace fmm2d
