// The gradient of the potential (the field), binary64.  A binary64
// evaluation leaves the local expansions B of every leaf; then the gradient
// of the near field over the finest strong lists (one wavefront per item of
// the full near-field schedule, as the binary64 potential kernel) and, per
// point, the derivative of the local expansion (Section 5's representation:
// with F(z) = sum_l B_l ((z - c)/s)^l, d/dx Re F = Re F' and d/dy Re F =
// -Im F').  The near-field term of a pair is q_j (z_i - z_j) / |z_i - z_j|^2
// componentwise; coincident pairs contribute nothing.
#include "devutil.h"
#include "internal.h"
#include "evaluate.h"

namespace fmm2d {
namespace {

constexpr int GNWB = 4;  // wavefronts per block

template <int TM, int GL>
__global__ void __launch_bounds__(64 * GNWB) k_near64_grad(int64_t nitems, int chunks, int maxleaf,
                                                          const int32_t *__restrict__ stL,
                                                          const double *__restrict__ px,
                                                          const double *__restrict__ py,
                                                          const double *__restrict__ qs,
                                                          const int32_t *__restrict__ sptr,
                                                          const int2 *__restrict__ segtab,
                                                          const int32_t *__restrict__ nseg_ptr,
                                                          const int2 *__restrict__ recj, double *__restrict__ gpart) {
    constexpr int LPI = 64 / GL;
    const int64_t item = (int64_t)blockIdx.x * GNWB + threadIdx.x / 64;
    if (item >= nitems) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int64_t sg = item / chunks;
    if (sg >= *nseg_ptr) return;
    const int ch = (int)(item - sg * chunks);
    const int2 se = segtab[sg];
    const int64_t b = se.x;
    const int32_t le = stL[b + 1];
    const int32_t a = stL[b] + ch * TM;
    if (a >= le) return;
    const int nt = (le - a) < TM ? (le - a) : TM;
    double tx[TM], ty[TM], ax[TM], ay[TM];
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const int32_t i = a + (k < nt ? k : 0);
        tx[k] = px[i];
        ty[k] = py[i];
        ax[k] = 0.0;
        ay[k] = 0.0;
    }
    const int grp = lane / GL, jj = lane % GL;
    const int32_t t0 = se.y, t1 = (se.y + NEAR_SEG) < sptr[b + 1] ? (se.y + NEAR_SEG) : sptr[b + 1];
    for (int32_t t = t0; t < t1; t += LPI) {
        const int32_t tt = t + grp;
        int2 rj = make_int2(0, 0);
        if (tt < t1) rj = recj[tt];
        for (int jb = 0; jb < maxleaf; jb += GL) {
            const int32_t j = rj.x + jb + jj;
            const bool ok = j < rj.y;
            double sx = 0.0, sy = 0.0, q = 0.0;
            if (ok) {
                sx = px[j];
                sy = py[j];
                q = qs[j];
            }
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                const double dx = tx[k] - sx, dy = ty[k] - sy;
                const bool use = ok && (dx != 0.0 || dy != 0.0);
                const double w = use ? q / (dx * dx + dy * dy) : 0.0;
                ax[k] += w * dx;
                ay[k] += w * dy;
            }
        }
    }
    double mx = 0.0, my = 0.0;
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        double vx = ax[k], vy = ay[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            vx += __shfl_xor(vx, off, 64);
            vy += __shfl_xor(vy, off, 64);
        }
        if (lane == k) {
            mx = vx;
            my = vy;
        }
    }
    if (lane < TM) {
        gpart[2 * (item * TM + lane)] = mx;
        gpart[2 * (item * TM + lane) + 1] = my;
    }
}

// Per point (leaf order): the near-field gradient summed over its leaf's
// segments in segment order, plus the derivative of the local expansion;
// written at the point's input position.
__global__ void k_grad_reduce(int p, int64_t n, int tm, int chunks, const int32_t *__restrict__ leafid,
                              const int32_t *__restrict__ stL, const int32_t *__restrict__ segoff,
                              const double *__restrict__ gpart, const double4 *__restrict__ geomL,
                              const double *__restrict__ px, const double *__restrict__ py,
                              const cd *__restrict__ BL, const int32_t *__restrict__ perm, double *__restrict__ gx,
                              double *__restrict__ gy) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = leafid[i];
    const int32_t off = (int32_t)(i - stL[b]);
    const int ch = off / tm, k = off - ch * tm;
    double nx = 0.0, ny = 0.0;
    for (int32_t sg = segoff[b]; sg < segoff[b + 1]; ++sg) {
        const int64_t r = ((int64_t)sg * chunks + ch) * tm + k;
        nx += gpart[2 * r];
        ny += gpart[2 * r + 1];
    }
    const double4 g = geomL[b];
    const cd z{(px[i] - g.x) / g.w, (py[i] - g.y) / g.w};
    const cd *Bb = BL + (int64_t)b * (p + 1);
    cd d{0.0, 0.0};
    for (int l = p; l >= 1; --l) d = cadd(cmul(d, z), cscale(Bb[l], (double)l));
    const int32_t o = perm[i];
    gx[o] = d.re / g.w + nx;
    gy[o] = -d.im / g.w + ny;
}

template <int TM, int GL>
hipError_t launch_grad(fmm2d_ctx *c, int p, int maxleaf, double *gx, double *gy) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const Schedule &sc = t.near_seg;
    const int chunks = (maxleaf + TM - 1) / TM;
    const int64_t nitems = sc.bound * chunks;
    FMM2D_TRY(e.gpart.ensure(sizeof(double) * 2 * (size_t)(nitems > 0 ? nitems : 1) * TM));
    double *gpart = e.gpart.as<double>();
    const int64_t offL = level_offset(L);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    hipLaunchKernelGGL((k_near64_grad<TM, GL>), dim3(grid_for(nitems, GNWB)), dim3(64 * GNWB), 0, c->stream, nitems,
                       chunks, maxleaf, stL, t.px.as<double>(), t.py.as<double>(), e.qs.as<double>(),
                       t.sptr.as<int32_t>() + ptr_offset(L), sc.table.as<int2>(),
                       sc.segoff.as<int32_t>() + nleaf, t.nrec_j.as<int2>(), gpart);
    FMM2D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_grad_reduce, dim3(grid_for(t.n, 256)), dim3(256), 0, c->stream, p, t.n, TM, chunks,
                       t.leafid.as<int32_t>(), stL, sc.segoff.as<int32_t>(), gpart,
                       t.geom.as<double4>() + offL, t.px.as<double>(), t.py.as<double>(),
                       e.B.as<cd>() + offL * (p + 1), t.perm.as<int32_t>(), gx, gy);
    return hipGetLastError();
}

}  // namespace

// After evaluate_device(..., FMM2D_MODE_FP64, ...) with the same p: the
// gradient at every point, input order.
hipError_t gradient_device(fmm2d_ctx *c, int p, double *gx, double *gy) {
    TreeState &t = c->tree;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const int64_t maxleaf = (t.n + nleaf - 1) >> (2 * L);  // ceil(n / 4^L)
    const int ml = (int)(maxleaf < (int64_t)1 << 30 ? maxleaf : (int64_t)1 << 30);
    FMM2D_TRY(ensure_near_full_schedule(c));
    if (ml <= 8) return launch_grad<8, 8>(c, p, ml, gx, gy);
    if (ml <= 16) return launch_grad<16, 16>(c, p, ml, gx, gy);
    if (ml <= 32) return launch_grad<16, 32>(c, p, ml, gx, gy);
    return launch_grad<16, 64>(c, p, ml, gx, gy);
}

}  // namespace fmm2d
