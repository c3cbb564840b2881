// Binary64 direct sum (eq. (1.1)) at selected targets, with Neumaier
// compensated summation: the judge of every reduced-precision result.
//
// Blocks are (64 targets) x (one chunk of the sources); a chunk is streamed
// through LDS and every lane keeps a compensated (sum, correction) pair.  The
// chunk partials are combined per target by a second kernel in chunk order,
// so the result does not depend on scheduling.
#include <mutex>

#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int JT = 64;     // targets per block
constexpr int JS = 256;    // sources per LDS tile

__device__ inline void neumaier(double &s, double &c, double t) {
    const double u = s + t;
    if (fabs(s) >= fabs(t)) c += (s - u) + t;
    else c += (t - u) + s;
    s = u;
}

__global__ void __launch_bounds__(JT) k_direct_part(const double *__restrict__ x, const double *__restrict__ y,
                                                    const double *__restrict__ q, int64_t n,
                                                    const int64_t *__restrict__ targets, int64_t m, int64_t chunk,
                                                    double2 *__restrict__ part) {
    __shared__ double sx[JS], sy[JS], sq[JS];
    const int64_t t = (int64_t)blockIdx.x * JT + threadIdx.x;
    const bool ok = t < m;
    const int64_t i = ok ? targets[t] : 0;
    const double xi = x[i], yi = y[i];
    double s = 0.0, cc = 0.0;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    for (int64_t base = j0; base < j1; base += JS) {
        const int64_t cnt = (j1 - base) < JS ? (j1 - base) : JS;
        for (int k = threadIdx.x; k < cnt; k += JT) {
            sx[k] = x[base + k];
            sy[k] = y[base + k];
            sq[k] = q[base + k];
        }
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            const double dx = xi - sx[k], dy = yi - sy[k];
            if (dx != 0.0 || dy != 0.0) neumaier(s, cc, sq[k] * log(hypot(dx, dy)));
        }
        __syncthreads();
    }
    if (ok) part[(int64_t)blockIdx.y * m + t] = make_double2(s, cc);
}

__global__ void k_direct_reduce(const double2 *__restrict__ part, int64_t m, int nchunk, double *__restrict__ phi) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    double s = 0.0, c = 0.0, corr = 0.0;
    for (int k = 0; k < nchunk; ++k) {
        const double2 v = part[(int64_t)k * m + t];
        neumaier(s, c, v.x);
        corr += v.y;
    }
    phi[t] = s + (c + corr);
}

// The gradient of the same sum, (d/dx, d/dy) of q_j log|z_i - z_j| =
// q_j (z_i - z_j) / |z_i - z_j|^2 componentwise; the same blocking and
// compensated sums, two components per target.
__global__ void __launch_bounds__(JT) k_direct_grad_part(const double *__restrict__ x, const double *__restrict__ y,
                                                         const double *__restrict__ q, int64_t n,
                                                         const int64_t *__restrict__ targets, int64_t m, int64_t chunk,
                                                         double4 *__restrict__ part) {
    __shared__ double sx[JS], sy[JS], sq[JS];
    const int64_t t = (int64_t)blockIdx.x * JT + threadIdx.x;
    const bool ok = t < m;
    const int64_t i = ok ? targets[t] : 0;
    const double xi = x[i], yi = y[i];
    double s1 = 0.0, c1 = 0.0, s2 = 0.0, c2 = 0.0;
    const int64_t j0 = (int64_t)blockIdx.y * chunk;
    const int64_t j1 = j0 + chunk < n ? j0 + chunk : n;
    for (int64_t base = j0; base < j1; base += JS) {
        const int64_t cnt = (j1 - base) < JS ? (j1 - base) : JS;
        for (int k = threadIdx.x; k < cnt; k += JT) {
            sx[k] = x[base + k];
            sy[k] = y[base + k];
            sq[k] = q[base + k];
        }
        __syncthreads();
        for (int k = 0; k < cnt; ++k) {
            const double dx = xi - sx[k], dy = yi - sy[k];
            if (dx != 0.0 || dy != 0.0) {
                const double r2 = dx * dx + dy * dy;
                neumaier(s1, c1, sq[k] * dx / r2);
                neumaier(s2, c2, sq[k] * dy / r2);
            }
        }
        __syncthreads();
    }
    if (ok) part[(int64_t)blockIdx.y * m + t] = make_double4(s1, c1, s2, c2);
}

__global__ void k_direct_grad_reduce(const double4 *__restrict__ part, int64_t m, int nchunk, double *__restrict__ gx,
                                     double *__restrict__ gy) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m) return;
    double s1 = 0.0, c1 = 0.0, k1 = 0.0, s2 = 0.0, c2 = 0.0, k2 = 0.0;
    for (int k = 0; k < nchunk; ++k) {
        const double4 v = part[(int64_t)k * m + t];
        neumaier(s1, c1, v.x);
        k1 += v.y;
        neumaier(s2, c2, v.z);
        k2 += v.w;
    }
    gx[t] = s1 + (c1 + k1);
    gy[t] = s2 + (c2 + k2);
}

static int64_t judge_chunks(int64_t n, int64_t m) {
    const int64_t groups = (m + JT - 1) / JT;
    int64_t nchunk = (2048 + groups - 1) / groups;
    const int64_t maxchunk = (n + 1023) / 1024;
    if (nchunk > maxchunk) nchunk = maxchunk;
    if (nchunk < 1) nchunk = 1;
    if (nchunk > 65535) nchunk = 65535;
    return nchunk;
}

}  // namespace

hipError_t direct_grad_device(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                              const int64_t *targets, int64_t m, double *gx, double *gy) {
    const int64_t groups = (m + JT - 1) / JT;
    const int64_t nchunk = judge_chunks(n, m);
    const int64_t chunk = (n + nchunk - 1) / nchunk;
    FMM2D_TRY(c->scr.flag.ensure(sizeof(double4) * nchunk * m));
    double4 *part = c->scr.flag.as<double4>();
    hipLaunchKernelGGL(k_direct_grad_part, dim3((unsigned)groups, (unsigned)nchunk), dim3(JT), 0, c->stream, x, y, q,
                       n, targets, m, chunk, part);
    hipLaunchKernelGGL(k_direct_grad_reduce, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, part, m, (int)nchunk,
                       gx, gy);
    return hipGetLastError();
}

// The two judge launches with the chunk partials in `part` (double2
// [direct_part_count(n, m)]).
static hipError_t direct_launch(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                                const int64_t *targets, int64_t m, double *phi, double2 *part) {
    const int64_t groups = (m + JT - 1) / JT;
    const int64_t nchunk = judge_chunks(n, m);
    const int64_t chunk = (n + nchunk - 1) / nchunk;
    hipLaunchKernelGGL(k_direct_part, dim3((unsigned)groups, (unsigned)nchunk), dim3(JT), 0, c->stream, x, y, q, n,
                       targets, m, chunk, part);
    hipLaunchKernelGGL(k_direct_reduce, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, part, m, (int)nchunk, phi);
    return hipGetLastError();
}

int64_t direct_part_count(int64_t n, int64_t m) { return judge_chunks(n, m) * m; }

hipError_t direct_device(fmm2d_ctx *c, const double *x, const double *y, const double *q, int64_t n,
                         const int64_t *targets, int64_t m, double *phi) {
    FMM2D_TRY(c->scr.flag.ensure(sizeof(double2) * direct_part_count(n, m)));
    return direct_launch(c, x, y, q, n, targets, m, phi, c->scr.flag.as<double2>());
}

// ---- the judge without allocations -----------------------------------------
// A fixed device array holds the chunk partials and the target-check flags,
// so fmm2d_direct_noalloc calls no allocator.  Each device holds its own copy;
// its address is looked up once per device (with that device current) and
// only that address is passed to kernels and copies.
constexpr size_t NOALLOC_PART_BYTES = size_t(4) << 20;
constexpr size_t NOALLOC_BYTES = NOALLOC_PART_BYTES + 256;
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

__global__ void k_flags_clear(int *flags) { flags[0] = 0; }
__global__ void k_flags_targets(const int64_t *__restrict__ t, int64_t m, int64_t n, int *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && (t[i] < 0 || t[i] >= n)) flags[0] = 1;
}
}  // namespace

hipError_t noalloc_scratch(int device, void **ptr) {
    if (device < 0 || device >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        FMM2D_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[device] = p;
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

bool noalloc_fits(int64_t n, int64_t m) {
    // judge_chunks gives at most ceil(2048 / ceil(m / 64)) chunks, so the
    // partials number at most 2048 * 64 + m: every m <= 2^18 fits in 4 MiB
    return (size_t)direct_part_count(n, m) * sizeof(double2) <= NOALLOC_PART_BYTES;
}

hipError_t direct_noalloc_device(fmm2d_ctx *c, void *scr, const double *x, const double *y, const double *q,
                                 int64_t n, const int64_t *targets, int64_t m, double *phi, bool *bad_target) {
    int *flags = reinterpret_cast<int *>(static_cast<unsigned char *>(scr) + NOALLOC_PART_BYTES);
    hipLaunchKernelGGL(k_flags_clear, dim3(1), dim3(1), 0, c->stream, flags);
    hipLaunchKernelGGL(k_flags_targets, dim3(grid_for(m, 256)), dim3(256), 0, c->stream, targets, m, n, flags);
    int hf = 0;
    FMM2D_TRY(hipMemcpyAsync(&hf, flags, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    FMM2D_TRY(hipStreamSynchronize(c->stream));
    *bad_target = hf != 0;
    if (hf) return hipSuccess;
    return direct_launch(c, x, y, q, n, targets, m, phi, static_cast<double2 *>(scr));
}

}  // namespace fmm2d
