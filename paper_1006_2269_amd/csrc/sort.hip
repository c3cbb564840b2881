// Stable LSD radix sort of the two coordinates, each with its original
// indices, in the same launches (blockIdx.y selects the coordinate).
//
// Sorting a coordinate with its index as the value, stably, yields the order
// by the pair (coordinate, index): the key with which every box of the tree
// is split at its median.  Keys are the usual order-preserving map of an IEEE
// double to uint64 (after -0.0 is folded onto +0.0, so that equal values tie).
// 8-bit digits, three kernels per pass: tile histograms, a column scan per
// (coordinate, digit), and a stable rank-and-scatter that stages each tile in
// LDS in digit order so that global writes are runs of consecutive
// addresses; the last pass writes the sorted coordinates, the order and the
// ranks directly.  The key kernel also validates the input (finite, |v| <= 2^500)
// and reduces the bitwise AND and OR of all keys per block; one small kernel
// and one host read then give the digits on which all keys agree, whose
// passes are skipped.
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;
constexpr int RADIX = 256;
constexpr int NW = SORT_THREADS / WAVE;

__device__ inline uint64_t to_key(double v) {
    v = v + 0.0;  // -0.0 -> +0.0
    uint64_t u = (uint64_t)__double_as_longlong(v);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}
__device__ inline double from_key(uint64_t k) {
    uint64_t u = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    return __longlong_as_double((long long)u);
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

struct SortBufs {
    uint64_t *keys[2][2];   // [coordinate][ping/pong]
    int32_t *vals[2][2];
};

// keys, values, per-block AND / OR of the keys and a validation flag.
// part[(y * nblk + blk) * 3 + {0, 1, 2}] = AND, OR, bad
__global__ void __launch_bounds__(256) k_make_keys(const double *__restrict__ x, const double *__restrict__ y,
                                                   int64_t n, SortBufs B, unsigned long long *__restrict__ part,
                                                   int nblk) {
    __shared__ unsigned long long sa[256 / 64], so[256 / 64];
    __shared__ int sbad[256 / 64];
    const int c = blockIdx.y;
    const double *v = c ? y : x;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t ka = ~0ull, ko = 0ull;
    int bad = 0;
    if (i < n) {
        const double d = v[i];
        bad = !(fabs(d) <= 0x1p500);  // also catches NaN
        const uint64_t k = to_key(d);
        B.keys[c][0][i] = k;
        B.vals[c][0][i] = (int32_t)i;
        ka = k;
        ko = k;
    }
    for (int off = 32; off > 0; off >>= 1) {
        ka &= (uint64_t)__shfl_xor((unsigned long long)ka, off);
        ko |= (uint64_t)__shfl_xor((unsigned long long)ko, off);
        bad |= __shfl_xor(bad, off);
    }
    const int w = threadIdx.x / 64;
    if (lane_id() == 0) {
        sa[w] = ka;
        so[w] = ko;
        sbad[w] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = ~0ull, o = 0ull;
        int bb = 0;
        for (int k = 0; k < 256 / 64; ++k) {
            a &= sa[k];
            o |= so[k];
            bb |= sbad[k];
        }
        unsigned long long *pp = part + ((int64_t)c * nblk + blockIdx.x) * 3;
        pp[0] = a;
        pp[1] = o;
        pp[2] = (unsigned long long)bb;
    }
}

// One block: reduce the per-block partials to out[c * 3 + {AND, OR, bad}].
__global__ void __launch_bounds__(256) k_reduce_andor(const unsigned long long *__restrict__ part, int nblk,
                                                      unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sa[256], so[256], sb[256];
    constexpr int U = 8;  // partials per thread in flight
    for (int c = 0; c < 2; ++c) {
        unsigned long long a = ~0ull, o = 0ull, b = 0ull;
        for (int k0 = threadIdx.x; k0 < nblk; k0 += 256 * U) {
            unsigned long long pa[U], po[U], pb[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {  // clamped indices: no branch around the loads
                const int k = k0 + u * 256;
                const unsigned long long *pp = part + ((int64_t)c * nblk + (k < nblk ? k : nblk - 1)) * 3;
                pa[u] = pp[0];
                po[u] = pp[1];
                pb[u] = pp[2];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {  // a repeated partial changes neither AND nor OR
                a &= pa[u];
                o |= po[u];
                b |= pb[u];
            }
        }
        sa[threadIdx.x] = a;
        so[threadIdx.x] = o;
        sb[threadIdx.x] = b;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if (threadIdx.x < w) {
                sa[threadIdx.x] &= sa[threadIdx.x + w];
                so[threadIdx.x] |= so[threadIdx.x + w];
                sb[threadIdx.x] |= sb[threadIdx.x + w];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            out[c * 3 + 0] = sa[0];
            out[c * 3 + 1] = so[0];
            out[c * 3 + 2] = sb[0];
        }
        __syncthreads();
    }
}

// tile histograms: hist[(c * RADIX + d) * nblk + blk]
__global__ void __launch_bounds__(SORT_THREADS) k_hist(SortBufs B, int ping, int64_t n, int shift,
                                                       int32_t *__restrict__ hist, int nblk) {
    __shared__ int32_t h[RADIX];
    const int c = blockIdx.y;
    const uint64_t *keys = B.keys[c][ping];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE;
    // every load of the tile in flight before the first ranking
    // (indices clamped into the array, so the loads need no branch)
    uint64_t kk[SORT_ITEMS];
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * SORT_THREADS + threadIdx.x;
        kk[r] = keys[i < n ? i : n - 1];
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * SORT_THREADS + threadIdx.x;
        const bool ok = i < n;
        const uint32_t d = ok ? (uint32_t)((kk[r] >> shift) & 0xff) : 0u;
        const uint64_t valid = __ballot(ok);
        const uint64_t peers = match_digit(d, valid);
        if (ok && popc_below(peers) == 0) atomicAdd(&h[d], (int32_t)__popcll(peers));
    }
    __syncthreads();
    hist[((int64_t)c * RADIX + threadIdx.x) * nblk + blockIdx.x] = h[threadIdx.x];
}

// One block per (coordinate, digit): exclusive scan of the digit's column of
// tile counts in place, and the column total to tot[c * RADIX + d].
__global__ void __launch_bounds__(256) k_colscan(int32_t *__restrict__ hist, int nblk, int32_t *__restrict__ tot) {
    __shared__ int32_t tmp[256 / 64];
    const int64_t col = (int64_t)blockIdx.y * RADIX + blockIdx.x;
    int32_t *hc = hist + col * nblk;
    const int per = (nblk + 255) / 256;
    const int b0 = threadIdx.x * per;
    int32_t s = 0;
    for (int b = b0; b < b0 + per && b < nblk; ++b) s += hc[b];
    int32_t total;
    int32_t run = block_excl_scan<256>(s, tmp, total);
    for (int b = b0; b < b0 + per && b < nblk; ++b) {
        const int32_t v = hc[b];
        hc[b] = run;
        run += v;
    }
    if (threadIdx.x == 0) tot[col] = total;
}

// Stable rank within the tile, staged in LDS in digit order, then written out
// as runs: element at LDS position s with digit d goes to
// digit_base[d] + column_offset[d][tile] + (s - tile_digit_start[d]).
// Each wavefront ranks its own SORT_ITEMS x 64 consecutive keys (rounds of 64) with
// private digit counters, so the rounds need no block barrier: within a
// round, lanes of equal digit are ranked by ballot matching and the round's
// leader advances the wave's counter.  The tile order (wave, round, lane) is
// the input order, so the sort stays stable.
// FINISH (the last pass): instead of the next key / value arrays, the tile
// writes the sorted coordinate, the order (sorted position -> index) and the
// rank (its inverse) directly.
template <bool FINISH>
__global__ void __launch_bounds__(SORT_THREADS) k_scatter(SortBufs B, int ping, int64_t n, int shift,
                                                          const int32_t *__restrict__ hist, int nblk,
                                                          const int32_t *__restrict__ tot, double *__restrict__ xs,
                                                          double *__restrict__ ys, int32_t *__restrict__ xorder,
                                                          int32_t *__restrict__ yorder, int32_t *__restrict__ xrank,
                                                          int32_t *__restrict__ yrank) {
    __shared__ uint64_t lk[SORT_TILE];
    __shared__ int32_t lv[SORT_TILE];
    __shared__ int32_t gpos[RADIX];    // global first position of this tile's digit d
    __shared__ int32_t lstart[RADIX];  // first LDS position of digit d
    __shared__ int32_t wcnt[NW][RADIX];  // per-wave digit counts, then per-wave offsets
    __shared__ int32_t tmp[SORT_THREADS / 64];
    const int c = blockIdx.y;
    const uint64_t *kin = B.keys[c][ping];
    const int32_t *vin = B.vals[c][ping];
    uint64_t *kout = B.keys[c][ping ^ 1];
    int32_t *vout = B.vals[c][ping ^ 1];
    const int t = threadIdx.x, w = t / WAVE;
    const uint32_t lane = lane_id();
    // digit bases of this coordinate: exclusive scan of the 256 totals
    int32_t total;
    const int32_t dbase = block_excl_scan<SORT_THREADS>(tot[c * RADIX + t], tmp, total);
    gpos[t] = dbase + hist[((int64_t)c * RADIX + t) * nblk + blockIdx.x];
    for (int k = 0; k < NW; ++k) wcnt[k][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SORT_TILE + (int64_t)w * (SORT_ITEMS * WAVE);
    uint64_t kr[SORT_ITEMS];
    int32_t vr[SORT_ITEMS], rk[SORT_ITEMS];
    // every load of the wave's keys and values in flight before the first ranking
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * WAVE + lane;
        const bool ok = i < n;
        kr[r] = ok ? kin[i] : 0ull;
        vr[r] = ok ? vin[i] : 0;
    }
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        const int64_t i = base + (int64_t)r * WAVE + lane;
        const bool ok = i < n;
        const uint64_t k = kr[r];
        const uint32_t d = (uint32_t)((k >> shift) & 0xff);
        const uint64_t valid = __ballot(ok);
        const uint64_t peers = match_digit(d, valid);
        const int32_t before = ok ? wcnt[w][d] : 0;  // read by every lane before the leader writes
        rk[r] = ok ? before + (int32_t)popc_below(peers) : -1;
        if (ok && popc_below(peers) == 0) wcnt[w][d] = before + (int32_t)__popcll(peers);
    }
    __syncthreads();
    // per digit: wave offsets (exclusive over waves) and the tile's count
    int32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int32_t v = wcnt[k][t];
        wcnt[k][t] = cnt;
        cnt += v;
    }
    int32_t ntile;
    const int32_t ls = block_excl_scan<SORT_THREADS>(cnt, tmp, ntile);
    lstart[t] = ls;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SORT_ITEMS; ++r) {
        if (rk[r] >= 0) {
            const uint32_t d = (uint32_t)((kr[r] >> shift) & 0xff);
            const int32_t s = lstart[d] + wcnt[w][d] + rk[r];
            lk[s] = kr[r];
            lv[s] = vr[r];
        }
    }
    __syncthreads();
    for (int s = t; s < ntile; s += SORT_THREADS) {
        const uint64_t k = lk[s];
        const uint32_t d = (uint32_t)((k >> shift) & 0xff);
        const int64_t dst = (int64_t)gpos[d] + (s - lstart[d]);
        if (FINISH) {
            const int32_t v = lv[s];
            (c ? ys : xs)[dst] = from_key(k);
            (c ? yorder : xorder)[dst] = v;
            (c ? yrank : xrank)[v] = (int32_t)dst;
        } else {
            kout[dst] = k;
            vout[dst] = lv[s];
        }
    }
}

// sorted values, order (sorted position -> index) and rank (its inverse)
__global__ void k_finish(SortBufs B, int ping, int64_t n, double *__restrict__ xs, double *__restrict__ ys,
                         int32_t *__restrict__ xorder, int32_t *__restrict__ yorder, int32_t *__restrict__ xrank,
                         int32_t *__restrict__ yrank) {
    const int c = blockIdx.y;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        (c ? ys : xs)[i] = from_key(B.keys[c][ping][i]);
        const int32_t v = B.vals[c][ping][i];
        (c ? yorder : xorder)[i] = v;
        (c ? yrank : xrank)[v] = (int32_t)i;
    }
}

}  // namespace

static void sort_bufs(fmm2d_ctx *c, int64_t n, SortBufs &B) {
    Scratch &s = c->scr;
    for (int k = 0; k < 2; ++k) {
        B.keys[k][0] = s.keys0.as<uint64_t>() + k * n;
        B.keys[k][1] = s.keys1.as<uint64_t>() + k * n;
        B.vals[k][0] = s.vals0.as<int32_t>() + k * n;
        B.vals[k][1] = s.vals1.as<int32_t>() + k * n;
    }
}

// First half: keys of both coordinates into scratch memory, validation and
// the digits on which all keys agree.  Touches nothing but scratch memory, so
// a rejected input leaves the current tree intact.
hipError_t sort_prepare(fmm2d_ctx *c, const double *x, const double *y, int64_t n, bool *bad_input) {
    Scratch &s = c->scr;
    const int nkb = (int)((n + 255) / 256);
    FMM2D_TRY(s.keys0.ensure(sizeof(uint64_t) * 2 * n));
    FMM2D_TRY(s.keys1.ensure(sizeof(uint64_t) * 2 * n));
    FMM2D_TRY(s.vals0.ensure(sizeof(int32_t) * 2 * n));
    FMM2D_TRY(s.vals1.ensure(sizeof(int32_t) * 2 * n));
    FMM2D_TRY(s.flag.ensure(sizeof(unsigned long long) * 3 * 2 * (size_t)nkb + 64));
    FMM2D_TRY(s.aux.ensure(4096));
    SortBufs B;
    sort_bufs(c, n, B);
    unsigned long long *part = s.flag.as<unsigned long long>();
    unsigned long long *andor = s.aux.as<unsigned long long>();
    hipLaunchKernelGGL(k_make_keys, dim3(nkb, 2), dim3(256), 0, c->stream, x, y, n, B, part, nkb);
    hipLaunchKernelGGL(k_reduce_andor, dim3(1), dim3(256), 0, c->stream, part, nkb, andor);
    FMM2D_TRY(hipGetLastError());
    unsigned long long h[6];
    FMM2D_TRY(hipMemcpyAsync(h, andor, sizeof(h), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    *bad_input = (h[2] | h[5]) != 0;
    s.sort_n = *bad_input ? -1 : n;
    s.sort_differ = (uint64_t)((h[0] ^ h[1]) | (h[3] ^ h[4]));
    return hipSuccess;
}

hipError_t sort_prepare_async(fmm2d_ctx *c, const double *x, const double *y, int64_t n,
                              unsigned long long *h_andor, hipEvent_t ev) {
    Scratch &s = c->scr;
    const int nkb = (int)((n + 255) / 256);
    FMM2D_TRY(s.keys0.ensure(sizeof(uint64_t) * 2 * n));
    FMM2D_TRY(s.keys1.ensure(sizeof(uint64_t) * 2 * n));
    FMM2D_TRY(s.vals0.ensure(sizeof(int32_t) * 2 * n));
    FMM2D_TRY(s.vals1.ensure(sizeof(int32_t) * 2 * n));
    FMM2D_TRY(s.flag.ensure(sizeof(unsigned long long) * 3 * 2 * (size_t)nkb + 64));
    FMM2D_TRY(s.aux.ensure(4096));
    SortBufs B;
    sort_bufs(c, n, B);
    unsigned long long *part = s.flag.as<unsigned long long>();
    unsigned long long *andor = s.aux.as<unsigned long long>();
    hipLaunchKernelGGL(k_make_keys, dim3(nkb, 2), dim3(256), 0, c->stream, x, y, n, B, part, nkb);
    hipLaunchKernelGGL(k_reduce_andor, dim3(1), dim3(256), 0, c->stream, part, nkb, andor);
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(hipMemcpyAsync(h_andor, andor, sizeof(unsigned long long) * 6, hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipEventRecord(ev, c->stream));
    s.sort_n = n;
    s.sort_differ = ~0ull;  // all eight passes: the skipped digits are known only after the host reads
    return hipSuccess;
}

// Second half: the radix passes over the digits that differ, then the sorted
// coordinates, their original indices and the ranks of the points.
hipError_t sort_finish(fmm2d_ctx *c, int64_t n, double *xs, double *ys, int32_t *xorder, int32_t *yorder,
                       int32_t *xrank, int32_t *yrank) {
    Scratch &s = c->scr;
    if (s.sort_n != n) return hipErrorInvalidValue;
    const int nblk = (int)((n + SORT_TILE - 1) / SORT_TILE);
    FMM2D_TRY(s.hist.ensure(sizeof(int32_t) * (size_t)2 * RADIX * nblk + sizeof(int32_t) * 2 * RADIX));
    SortBufs B;
    sort_bufs(c, n, B);
    int32_t *hist = s.hist.as<int32_t>();
    int32_t *tot = hist + (size_t)2 * RADIX * nblk;
    int ping = 0, last = -1;
    for (int shift = 0; shift < 64; shift += 8)
        if (((s.sort_differ >> shift) & 0xffull) != 0) last = shift;
    for (int shift = 0; shift < 64; shift += 8) {
        if (((s.sort_differ >> shift) & 0xffull) == 0) continue;
        hipLaunchKernelGGL(k_hist, dim3(nblk, 2), dim3(SORT_THREADS), 0, c->stream, B, ping, n, shift, hist, nblk);
        hipLaunchKernelGGL(k_colscan, dim3(RADIX, 2), dim3(256), 0, c->stream, hist, nblk, tot);
        if (shift == last)
            hipLaunchKernelGGL(k_scatter<true>, dim3(nblk, 2), dim3(SORT_THREADS), 0, c->stream, B, ping, n, shift,
                               hist, nblk, tot, xs, ys, xorder, yorder, xrank, yrank);
        else
            hipLaunchKernelGGL(k_scatter<false>, dim3(nblk, 2), dim3(SORT_THREADS), 0, c->stream, B, ping, n, shift,
                               hist, nblk, tot, xs, ys, xorder, yorder, xrank, yrank);
        FMM2D_TRY(hipGetLastError());
        ping ^= 1;
    }
    s.sort_n = -1;
    // every key equal (no pass ran): the input order is the sorted order
    if (last < 0)
        hipLaunchKernelGGL(k_finish, dim3(grid_for(n, 256), 2), dim3(256), 0, c->stream, B, ping, n, xs, ys, xorder,
                           yorder, xrank, yrank);
    return hipGetLastError();
}

}  // namespace fmm2d
