// Parameter selection: density features of the point set, the learned
// selector's decision, and the a-priori rule it falls back to.
//
// Features (NFEAT = 2 + 9 FL floats): log10 N, log10 TOL, then for each
// level l = 1..FL of a uniform 2^l x 2^l grid over the tight bounding box:
// the fraction of occupied cells, and an 8-bin histogram of the points by the
// relative density r = count 4^l / N of their cell (bin k: the number of the
// edges 1/8, 1/4, 1/2, 1, 2, 4, 8 that are <= r), as fractions of N.  In a
// median-split tree a box's area is inversely proportional to the density
// around it, so these histograms describe the spread of box sizes at each
// level, which sets the list lengths and hence the cost of an (L, p, theta).
// Cells are counted over a fixed sample of at most 2^18 points (every
// ceil(N / 2^18)-th point; all points when N <= 2^18), and densities and
// fractions refer to the sample size; the bounding box is that of all
// points.  All counts are integers (cell counts, LDS and global integer
// atomics), so the features do not depend on scheduling.
//
// Decision (after the network, or the rule when no weights are given or the
// input lies outside the trained range): the rule is the practical choice
// at the end of Section 4, theta = 1/2 and about 20 points per leaf
// (L = round(log4(N / 20))), with the least p for which the truncation bound
// of Section 3, K theta^(p+1) / (1 - theta)^2 with K = 0.1, is <= TOL.  The
// network predicts L - log4(N / 16) (the level count's offset from 16 points
// per leaf, continuous in N), log10 C of the error model e(p) ~ C
// theta^(p+1), and theta; L is rounded, theta snapped to
// {0.35, ..., 0.75}, and p is the least order the model says meets TOL / 2
// (a safety factor of 2 on the error).
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int FL = 10;
constexpr int NFEAT = 2 + 9 * FL;
constexpr int HDR = 194;  // weight blob header floats, see fmm2d.h
constexpr int BT = 256;
constexpr int64_t SAMPLE_MAX = int64_t(1) << 18;  // points counted into cells
constexpr double SAFETY_LOG10 = 0.30102999566398120;  // log10(2): error margin of the network's p

// Per-block min / max of x and y, and whether any coordinate is invalid.
__global__ void __launch_bounds__(BT) k_bbox_part(const double *__restrict__ x, const double *__restrict__ y,
                                                  int64_t n, double *__restrict__ part) {
    __shared__ double s[4][BT];
    __shared__ int sbad[BT];
    double xl = INFINITY, xh = -INFINITY, yl = INFINITY, yh = -INFINITY;
    int bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const double a = x[i] + 0.0, b = y[i] + 0.0;
        bad |= !(fabs(a) <= 0x1p500) || !(fabs(b) <= 0x1p500);
        xl = fmin(xl, a);
        xh = fmax(xh, a);
        yl = fmin(yl, b);
        yh = fmax(yh, b);
    }
    s[0][threadIdx.x] = xl;
    s[1][threadIdx.x] = xh;
    s[2][threadIdx.x] = yl;
    s[3][threadIdx.x] = yh;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int w = BT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
            sbad[threadIdx.x] |= sbad[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double *p = part + 5 * (int64_t)blockIdx.x;
        p[0] = s[0][0];
        p[1] = s[1][0];
        p[2] = s[2][0];
        p[3] = s[3][0];
        p[4] = sbad[0] ? 1.0 : 0.0;
    }
}

// box = {xmin, xmax, ymin, ymax, sx, sy, bad}: s = 2^FL / extent (0 when the
// extent is 0, which puts every point in cell 0).
__global__ void __launch_bounds__(BT) k_bbox_final(const double *__restrict__ part, int nblk,
                                                   double *__restrict__ box) {
#pragma clang fp contract(off)
    __shared__ double s[5][BT];
    double v[5] = {INFINITY, -INFINITY, INFINITY, -INFINITY, 0.0};
    for (int k = threadIdx.x; k < nblk; k += BT) {
        const double *p = part + 5 * (int64_t)k;
        v[0] = fmin(v[0], p[0]);
        v[1] = fmax(v[1], p[1]);
        v[2] = fmin(v[2], p[2]);
        v[3] = fmax(v[3], p[3]);
        v[4] = fmax(v[4], p[4]);
    }
    for (int j = 0; j < 5; ++j) s[j][threadIdx.x] = v[j];
    __syncthreads();
    for (int w = BT / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            s[0][threadIdx.x] = fmin(s[0][threadIdx.x], s[0][threadIdx.x + w]);
            s[1][threadIdx.x] = fmax(s[1][threadIdx.x], s[1][threadIdx.x + w]);
            s[2][threadIdx.x] = fmin(s[2][threadIdx.x], s[2][threadIdx.x + w]);
            s[3][threadIdx.x] = fmax(s[3][threadIdx.x], s[3][threadIdx.x + w]);
            s[4][threadIdx.x] = fmax(s[4][threadIdx.x], s[4][threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double ex = s[1][0] - s[0][0], ey = s[3][0] - s[2][0];
        box[0] = s[0][0];
        box[1] = s[1][0];
        box[2] = s[2][0];
        box[3] = s[3][0];
        box[4] = ex > 0.0 ? (double)(1 << FL) / ex : 0.0;
        box[5] = ey > 0.0 ? (double)(1 << FL) / ey : 0.0;
        box[6] = s[4][0];
    }
}

// Histogram totals of levels 5..10 are added by 1024 blocks; to keep the
// same-address chains of those (integer, order-independent) atomics short,
// block b adds into copy b % ACC_COPIES, and the final kernel sums the copies.
constexpr int ACC_COPIES = 32;
// Likewise the finest counts: dense clusters put hundreds of sampled points
// into one cell, so block b counts into grid copy b % GRID_COPIES and the
// pooling kernel adds the copies as it loads them.
constexpr int GRID_COPIES = 4;

// zero the finest grid copies and the counter copies
__global__ void k_zero_grid(int32_t *__restrict__ fine, int64_t nfine, unsigned long long *__restrict__ acc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < GRID_COPIES * nfine) fine[i] = 0;
    else if (i - GRID_COPIES * nfine < ACC_COPIES * 9 * FL) acc[i - GRID_COPIES * nfine] = 0ull;
}

__device__ inline int cell_coord(double v, double lo, double s) {
#pragma clang fp contract(off)
    double t = (v - lo) * s;
    if (!(t >= 0.0)) t = 0.0;  // also NaN
    if (!(t < (double)(1 << FL))) t = (double)((1 << FL) - 1);
    return (int)t;
}

// counts of the finest grid over the sample (every stride-th point)
__global__ void k_cells(const double *__restrict__ x, const double *__restrict__ y, int64_t ns, int64_t stride,
                        const double *__restrict__ box, int32_t *__restrict__ cnt) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= ns) return;
    const int64_t i = j * stride;
    const int ix = cell_coord(x[i] + 0.0, box[0], box[4]);
    const int iy = cell_coord(y[i] + 0.0, box[2], box[5]);
    atomicAdd(&cnt[(int64_t)(blockIdx.x % GRID_COPIES) * (int64_t(1) << (2 * FL)) + ((int64_t)iy << FL) + ix], 1);
}

// occupied count and density class of one cell of level l into sh (the
// level's 9 counters): class = number of edges 2^(j-4), j = 1..7, with
// count 4^l / ns >= edge, compared exactly as count 4^l 16 >= ns 2^j
__device__ inline void hist_cell(int32_t c, int l, int64_t ns, unsigned long long *sh) {
    if (c <= 0) return;
    const int64_t lhs = (int64_t)c << (2 * l + 4);
    int k = 0;
#pragma unroll
    for (int j = 1; j <= 7; ++j) k += lhs >= (ns << j) ? 1 : 0;
    atomicAdd(&sh[0], 1ull);
    atomicAdd(&sh[1 + k], (unsigned long long)c);
}

// One block per 32 x 32 tile of the finest grid: the histograms of levels
// 10..5 of the tile's cells, pooling 2 x 2 in LDS; the tile's level-5 count
// goes to cnt5 (a 32 x 32 grid) and the counters to acc.
__global__ void __launch_bounds__(BT) k_pool_hist_hi(const int32_t *__restrict__ fine, int64_t ns,
                                                     unsigned long long *__restrict__ acc, int32_t *__restrict__ cnt5) {
    __shared__ int32_t ga[1024], gb[256];
    __shared__ unsigned long long sh[9 * 6];
    const int t = threadIdx.x;
    const int tx = blockIdx.x % 32, ty = blockIdx.x / 32;
    if (t < 9 * 6) sh[t] = 0ull;
    for (int k = t; k < 1024; k += BT) {
        const int64_t cell = ((int64_t)(ty * 32 + k / 32) << FL) + tx * 32 + k % 32;
        int32_t v = 0;
#pragma unroll
        for (int g = 0; g < GRID_COPIES; ++g) v += fine[g * (int64_t(1) << (2 * FL)) + cell];
        ga[k] = v;
    }
    __syncthreads();
    int32_t *cur = ga, *nxt = gb;
    int side = 32;
    for (int l = FL; l >= 5; --l) {
        for (int k = t; k < side * side; k += BT) hist_cell(cur[k], l, ns, sh + 9 * (FL - l));
        if (l > 5) {
            const int h = side / 2;
            for (int k = t; k < h * h; k += BT) {
                const int i = k % h, j = k / h;
                nxt[k] = cur[2 * j * side + 2 * i] + cur[2 * j * side + 2 * i + 1] + cur[(2 * j + 1) * side + 2 * i] +
                         cur[(2 * j + 1) * side + 2 * i + 1];
            }
            side = h;
            int32_t *tmp = cur;
            cur = nxt;
            nxt = tmp;
        } else if (t == 0) {
            cnt5[ty * 32 + tx] = cur[0];
        }
        __syncthreads();
    }
    if (t < 9 * 6) {
        const int l = FL - t / 9, j = t % 9;
        if (sh[t]) atomicAdd(&acc[(blockIdx.x % ACC_COPIES) * (9 * FL) + 9 * (l - 1) + j], sh[t]);
    }
}

// One block: levels 4..1 from the level-5 grid, then the features (and the
// standardised network input x = (f - mean) * scale when a blob is given).
__global__ void __launch_bounds__(BT) k_pool_hist_lo(const int32_t *__restrict__ cnt5, int64_t n, int64_t ns,
                                                     double tol, const unsigned long long *__restrict__ acc,
                                                     float *__restrict__ feat, const float *__restrict__ blob,
                                                     float *__restrict__ xin) {
    __shared__ int32_t ga[1024], gb[256];
    __shared__ unsigned long long sh[9 * 4];
    const int t = threadIdx.x;
    if (t < 9 * 4) sh[t] = 0ull;
    for (int k = t; k < 1024; k += BT) ga[k] = cnt5[k];
    __syncthreads();
    int32_t *cur = ga, *nxt = gb;
    int side = 32;
    for (int l = 4; l >= 1; --l) {
        const int h = side / 2;
        for (int k = t; k < h * h; k += BT) {
            const int i = k % h, j = k / h;
            nxt[k] = cur[2 * j * side + 2 * i] + cur[2 * j * side + 2 * i + 1] + cur[(2 * j + 1) * side + 2 * i] +
                     cur[(2 * j + 1) * side + 2 * i + 1];
        }
        __syncthreads();
        for (int k = t; k < h * h; k += BT) hist_cell(nxt[k], l, ns, sh + 9 * (l - 1));
        side = h;
        int32_t *tmp = cur;
        cur = nxt;
        nxt = tmp;
        __syncthreads();
    }
    if (t >= NFEAT) return;
    double f;
    if (t == 0) f = log10((double)n);
    else if (t == 1) f = log10(tol);
    else {
        const int l = (t - 2) / 9 + 1, j = (t - 2) % 9;
        unsigned long long v = 0ull;
        if (l <= 4) {
            v = sh[9 * (l - 1) + j];
        } else {
            for (int k = 0; k < ACC_COPIES; ++k) v += acc[k * (9 * FL) + t - 2];
        }
        f = j == 0 ? (double)v / (double)(int64_t(1) << (2 * l)) : (double)v / (double)ns;
    }
    feat[t] = (float)f;
    if (blob) xin[t] = ((float)f - blob[t]) * blob[NFEAT + t];
}

// the a-priori rule
__device__ inline void rule(int64_t n, double tol, int lmax, int &L, int &p, double &theta) {
    theta = 0.5;
    const double x = log((double)n / 20.0 > 1.0 ? (double)n / 20.0 : 1.0) / log(4.0);
    L = (int)floor(x + 0.5);
    if (L > lmax) L = lmax;
    if (L < 1) L = 1;
    p = 1;
    double tp = theta * theta;  // theta^(p+1), exact for theta = 1/2
    while (0.1 * tp / ((1.0 - theta) * (1.0 - theta)) > tol && p < 63) {
        ++p;
        tp *= theta;
    }
}

// out_i = {levels, p, from_network, bad input}, out_d = {theta}
__global__ void k_select_final(const float *__restrict__ y, const float *__restrict__ blob, int64_t n, double tol,
                               const double *__restrict__ box, int *__restrict__ out_i, double *__restrict__ out_d) {
#pragma clang fp contract(off)
    const double thetas[5] = {0.35, 0.45, 0.55, 0.65, 0.75};
    if (threadIdx.x != 0) return;
    int lmax = 0;
    while (lmax < FMM2D_MAX_LEVELS && (int64_t(1) << (2 * (lmax + 1))) <= n) ++lmax;
    int L, p;
    double theta;
    bool net = false;
    if (blob) {
        const double ln = log10((double)n), lt = log10(tol);
        const float *rng = blob + 2 * NFEAT + 6;
        const bool inside = ln >= rng[0] && ln <= rng[1] && lt >= rng[2] && lt <= rng[3];
        const double dl = (double)y[0] * blob[2 * NFEAT + 3] + blob[2 * NFEAT + 0];
        const double lc = (double)y[1] * blob[2 * NFEAT + 4] + blob[2 * NFEAT + 1];
        const double th = (double)y[2] * blob[2 * NFEAT + 5] + blob[2 * NFEAT + 2];
        if (inside && isfinite(dl) && isfinite(lc) && isfinite(th) && fabs(dl) < 64.0 && fabs(lc) < 1e4) {
            net = true;
            const double x0 = log((double)n / 16.0 > 1.0 ? (double)n / 16.0 : 1.0) / log(4.0);
            L = (int)floor(x0 + dl + 0.5);
            L = L > lmax ? lmax : (L < 1 ? 1 : L);
            int g = (int)floor((th - 0.35) / 0.1 + 0.5);
            g = g < 0 ? 0 : (g > 4 ? 4 : g);
            theta = thetas[g];
            // error model e(p) ~ C theta^(p+1), with a safety factor of 2 on
            // the error: the least p with C theta^(p+1) <= TOL / 2
            const double q = ceil((lt - SAFETY_LOG10 - lc) / log10(theta)) - 1.0;
            p = q > (double)FMM2D_MAX_P ? FMM2D_MAX_P : (q < 1.0 ? 1 : (int)q);
        }
    }
    if (!net) rule(n, tol, lmax, L, p, theta);
    out_i[0] = L;
    out_i[1] = p;
    out_i[2] = net ? 1 : 0;
    out_i[3] = box[6] != 0.0 ? 1 : 0;
    out_d[0] = theta;
}

}  // namespace

// feat: device float [NFEAT]; blob (nullable): weights, then xin receives the
// standardised input.  Scratch: c->scr.sel.
hipError_t features_device(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol, float *feat,
                           const float *blob, float *xin, double **box_out, hipStream_t st) {
    Scratch &s = c->scr;
    if (!st) st = c->stream;
    const int nblk = (int)std::min<int64_t>((n + BT - 1) / BT, 1024);
    const int64_t nfine = int64_t(1) << (2 * FL);
    const int64_t stride = n > SAMPLE_MAX ? (n + SAMPLE_MAX - 1) / SAMPLE_MAX : 1;
    const int64_t ns = (n + stride - 1) / stride;
    const size_t bytes = sizeof(double) * (5 * (size_t)nblk + 8) + sizeof(unsigned long long) * ACC_COPIES * 9 * FL +
                         sizeof(int32_t) * (size_t)(GRID_COPIES * nfine + 1024) + 256;
    FMM2D_TRY(s.sel.ensure(bytes));
    char *base = s.sel.as<char>();
    double *part = reinterpret_cast<double *>(base);
    double *box = part + 5 * (size_t)nblk;
    unsigned long long *acc = reinterpret_cast<unsigned long long *>(box + 8);
    int32_t *fine = reinterpret_cast<int32_t *>(acc + ACC_COPIES * 9 * FL);
    int32_t *cnt5 = fine + GRID_COPIES * nfine;
    hipLaunchKernelGGL(k_bbox_part, dim3(nblk), dim3(BT), 0, st, x, y, n, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(BT), 0, st, part, nblk, box);
    hipLaunchKernelGGL(k_zero_grid, dim3(grid_for(GRID_COPIES * nfine + ACC_COPIES * 9 * FL, 256)), dim3(256), 0,
                       st, fine, nfine, acc);
    hipLaunchKernelGGL(k_cells, dim3(grid_for(ns, 256)), dim3(256), 0, st, x, y, ns, stride, box, fine);
    hipLaunchKernelGGL(k_pool_hist_hi, dim3(1024), dim3(BT), 0, st, fine, ns, acc, cnt5);
    hipLaunchKernelGGL(k_pool_hist_lo, dim3(1), dim3(BT), 0, st, cnt5, n, ns, tol, acc, feat, blob, xin);
    if (box_out) *box_out = box;
    return hipGetLastError();
}

// Queues the features, the network and the decision on stream st, and the
// copies of the decision into host memory h_out (levels, p, from_network, bad
// input) and h_theta; nothing waits.  Host memory that is not pinned makes
// the copies wait.
hipError_t select_launch(fmm2d_ctx *c, hipStream_t st, const double *x, const double *y, int64_t n, double tol,
                         const float *blob, int *h_out, double *h_theta) {
    Scratch &s = c->scr;
    FMM2D_TRY(s.sel2.ensure(sizeof(float) * (2 * NFEAT + 8) + 64));
    float *feat = s.sel2.as<float>();
    float *xin = feat + NFEAT;
    float *yout = xin + NFEAT;
    int *oi = reinterpret_cast<int *>(yout + 4);
    double *od = reinterpret_cast<double *>(s.sel2.as<char>() + sizeof(float) * (2 * NFEAT + 8) + 32);
    double *box = nullptr;
    FMM2D_TRY(features_device(c, x, y, n, tol, feat, blob, xin, &box, st));
    if (blob) FMM2D_TRY(mlp_forward(c, blob + HDR, xin, 1, NFEAT, yout, st));
    hipLaunchKernelGGL(k_select_final, dim3(1), dim3(64), 0, st, yout, blob, n, tol, box, oi, od);
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(hipMemcpyAsync(h_out, oi, sizeof(int) * 4, hipMemcpyDeviceToHost, st));
    return hipMemcpyAsync(h_theta, od, sizeof(double), hipMemcpyDeviceToHost, st);
}

hipError_t select_device(fmm2d_ctx *c, const double *x, const double *y, int64_t n, double tol, const float *blob,
                         int out[4], double *theta) {
    FMM2D_TRY(select_launch(c, c->stream, x, y, n, tol, blob, out, theta));
    return hipStreamSynchronize(c->stream);
}

}  // namespace fmm2d
