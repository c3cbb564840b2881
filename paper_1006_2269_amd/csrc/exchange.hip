// Exchanged roles for strongly coupled boxes of very different radii, the
// structural optimisation of Section 4: for a pair (b, c) on the exchanged
// list X_l(b), whose criterion holds once the roles of the radii are
// exchanged (r + theta R <= theta d, disjoint balls),
//
//  * target the smaller box (r_b < r_c): the sources of c become a local
//    expansion about b (P2L), added into B_b before the L2L pass carries it
//    down:  B_0 += sum q_j log|z_j - c_b|,  B_k += -(q_j / k) (s_b / (z_j - c_b))^k;
//  * target the larger box (r_b > r_c): the multipole of c is evaluated at
//    every point z of b (M2P):  phi(z) += Re[A_0 log(z - c_c) + sum_k A_k (s_c / (z - c_c))^k].
//
// Both run in binary64 in every precision mode.
//
// P2L is cut into work items of at most PCH source points (a coarse box can
// hold millions), one wavefront each; the items of a target box are
// consecutive, and the L2L pass adds their partial expansions in item order,
// so the result does not depend on scheduling.  M2P gathers per point: one
// wavefront per leaf walks the X lists of the leaf's ancestors (the same for
// all its lanes), so every point is written once.
#include "evaluate.h"

namespace fmm2d {
namespace {

constexpr int PCH = 512;   // source points per P2L work item
constexpr int XT = 16;     // coefficients per pass of the P2L accumulators

// Point range [a, e) of box b of level l (its leaves are b 4^(L-l) onwards).
__device__ inline void box_range(const int32_t *__restrict__ stL, int L, int l, int64_t b, int32_t &a, int32_t &e) {
    const int sh = 2 * (L - l);
    a = stL[b << sh];
    e = stL[(b + 1) << sh];
}

// Work items per global box g: for each P2L entry of X(g), ceil(points / PCH).
template <bool FILL>
__global__ void k_x_items(int L, int64_t nbox, const int32_t *__restrict__ xptr_all, const int32_t *__restrict__ xidx,
                          const int64_t *__restrict__ xoff, const double4 *__restrict__ geom,
                          const int32_t *__restrict__ stL, int32_t *__restrict__ cnt,
                          const int32_t *__restrict__ itemoff, int4 *__restrict__ items) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nbox) return;
    const int l = level_of(g);
    if (l < 1) {
        if (!FILL) cnt[g] = 0;
        return;
    }
    const int64_t b = g - level_offset(l);
    const int32_t *ptr = xptr_all + ptr_offset(l);
    const int32_t *row = xidx + xoff[l];
    const double4 gb = geom[g];
    int32_t k = FILL ? itemoff[g] : 0;
    for (int32_t t = ptr[b]; t < ptr[b + 1]; ++t) {
        const int64_t cg = level_offset(l) + row[t];
        if (!(gb.z < geom[cg].z)) continue;  // M2P entry: handled per point
        int32_t a, e;
        box_range(stL, L, l, row[t], a, e);
        for (int32_t j = a; j < e; j += PCH) {
            if (FILL) items[k] = make_int4((int32_t)g, (int32_t)cg, j, e < j + PCH ? e : j + PCH);
            ++k;
        }
    }
    if (!FILL) cnt[g] = k;
}

// One wavefront per P2L item: lanes over the item's source points, each lane
// accumulating XT coefficients at a time, the lanes summed by a butterfly.
__global__ void __launch_bounds__(256) k_p2l(int p, const int4 *__restrict__ items, const int32_t *__restrict__ nitem,
                                             const double4 *__restrict__ geom, const double *__restrict__ px,
                                             const double *__restrict__ py, const double *__restrict__ qs,
                                             cd *__restrict__ xpart) {
    const int64_t it = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (it >= *nitem) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int4 w = items[it];
    const double4 gb = geom[w.x];
    const int P1 = p + 1;
    for (int k0 = 0; k0 < P1; k0 += XT) {
        double ar[XT], ai[XT];
#pragma unroll
        for (int k = 0; k < XT; ++k) {
            ar[k] = 0.0;
            ai[k] = 0.0;
        }
        for (int32_t j = w.z + lane; j < w.w; j += 64) {
            const double dx = px[j] - gb.x, dy = py[j] - gb.y, q = qs[j];
            const double d2 = dx * dx + dy * dy;  // > 0: the source lies outside the target's ball
            const double inv = gb.w / d2;
            const cd rho = d2 > 0x1p-960 ? cd{dx * inv, -dy * inv} : cdiv(cd{gb.w, 0.0}, cd{dx, dy});
            cd pw{1.0, 0.0};
            for (int k = 0; k < k0; ++k) pw = cmul(pw, rho);  // rho^k0
#pragma unroll
            for (int k = 0; k < XT; ++k) {
                const int kk = k0 + k;
                if (kk <= p) {
                    if (kk == 0) {
                        ar[0] += q * (d2 > 0x1p-960 ? 0.5 * log(d2) : log(hypot(dx, dy)));
                    } else {
                        const double f = -q / (double)kk;
                        ar[k] = fma(f, pw.re, ar[k]);
                        ai[k] = fma(f, pw.im, ai[k]);
                    }
                }
                pw = cmul(pw, rho);
            }
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int k = 0; k < XT; ++k) {
                ar[k] += __shfl_xor(ar[k], off, 64);
                ai[k] += __shfl_xor(ai[k], off, 64);
            }
        }
#pragma unroll
        for (int k = 0; k < XT; ++k)
            if (lane == k && k0 + k <= p) xpart[it * P1 + k0 + k] = cd{ar[k], ai[k]};
    }
}

// One wavefront per leaf, one lane per point: the multipoles of the smaller
// boxes on the X lists of the leaf's ancestors at every level, evaluated at
// the point and added to its potential (input order).
__global__ void __launch_bounds__(256) k_m2p(int p, int L, int64_t nleaf, const int32_t *__restrict__ stL,
                                             const int32_t *__restrict__ xptr_all, const int32_t *__restrict__ xidx,
                                             const int64_t *__restrict__ xoff, const double4 *__restrict__ geom,
                                             const cd *__restrict__ A, const double *__restrict__ px,
                                             const double *__restrict__ py, const int32_t *__restrict__ perm,
                                             double *__restrict__ phi) {
    const int64_t leaf = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (leaf >= nleaf) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64;
    const int P1 = p + 1;
    const int32_t a = stL[leaf], e = stL[leaf + 1];
    for (int32_t base = a; base < e; base += 64) {
        const int32_t i = base + lane;
        const bool act = i < e;
        const double zx = act ? px[i] : 0.0, zy = act ? py[i] : 0.0;
        double acc = 0.0;
        for (int l = 1; l <= L; ++l) {
            const int64_t b = leaf >> (2 * (L - l));
            const double4 gb = geom[level_offset(l) + b];
            const int32_t *ptr = xptr_all + ptr_offset(l);
            const int32_t *row = xidx + xoff[l];
            for (int32_t t = ptr[b]; t < ptr[b + 1]; ++t) {
                const int64_t cg = level_offset(l) + row[t];
                const double4 gc = geom[cg];
                if (!(gb.z > gc.z)) continue;  // P2L entry: handled by k_p2l
                const cd *Ac = A + cg * P1;
                // inactive lanes evaluate at a point one scale away (finite)
                const double dx = act ? zx - gc.x : gc.w, dy = act ? zy - gc.y : 0.0;
                const double d2 = dx * dx + dy * dy;
                const double inv = gc.w / d2;
                const cd rho = d2 > 0x1p-960 ? cd{dx * inv, -dy * inv} : cdiv(cd{gc.w, 0.0}, cd{dx, dy});
                cd s = Ac[p];
                for (int k = p - 1; k >= 1; --k) s = cadd(cmul(s, rho), Ac[k]);
                s = p >= 1 ? cmul(s, rho) : cd{0.0, 0.0};
                acc += Ac[0].re * (d2 > 0x1p-960 ? 0.5 * log(d2) : log(hypot(dx, dy))) + s.re;
            }
        }
        if (act) phi[perm[i]] += acc;
    }
}

}  // namespace

hipError_t exchange_schedule(fmm2d_ctx *c) {
    TreeState &t = c->tree;
    t.x_ready = false;
    const int L = t.L;
    if (!(t.opt & (FMM2D_OPT_SWAP_FINEST | FMM2D_OPT_SWAP_ALL)) || L < 1) return hipSuccess;
    if (t.x_off[L + 1] == t.x_off[1]) return hipSuccess;  // no exchanged pair
    const int64_t nbox = level_offset(L + 1);
    // every box of level l holds floor or ceil of n / 4^l points
    int64_t bound = 0;
    for (int l = 1; l <= L; ++l) {
        const int64_t maxpts = (t.n + (int64_t(1) << (2 * l)) - 1) >> (2 * l);
        bound += (t.x_off[l + 1] - t.x_off[l]) * ((maxpts + PCH - 1) / PCH);
    }
    FMM2D_TRY(c->scr.segcnt.ensure(sizeof(int32_t) * nbox));
    FMM2D_TRY(t.x_itemoff.ensure(sizeof(int32_t) * (nbox + 1)));
    FMM2D_TRY(t.x_items.ensure(sizeof(int4) * (bound > 0 ? bound : 1)));
    const int32_t *xptr = t.xptr.as<int32_t>(), *xidx = t.xidx.as<int32_t>();
    const int64_t *xoff = t.pool_state.as<int64_t>() + 2 * (L + 2);  // X pool offset of each level
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const double4 *geom = t.geom.as<double4>();
    hipLaunchKernelGGL(k_x_items<false>, dim3(grid_for(nbox, 256)), dim3(256), 0, c->stream, L, nbox, xptr, xidx,
                       xoff, geom, stL, c->scr.segcnt.as<int32_t>(), nullptr, nullptr);
    FMM2D_TRY(hipGetLastError());
    FMM2D_TRY(scan_exclusive(c, c->scr.segcnt.as<int32_t>(), nbox, t.x_itemoff.as<int32_t>()));
    hipLaunchKernelGGL(k_x_items<true>, dim3(grid_for(nbox, 256)), dim3(256), 0, c->stream, L, nbox, xptr, xidx,
                       xoff, geom, stL, nullptr, t.x_itemoff.as<int32_t>(), t.x_items.as<int4>());
    FMM2D_TRY(hipGetLastError());
    t.x_item_bound = bound;
    t.x_ready = true;
    return hipSuccess;
}

const int32_t *exchange_item_offsets(fmm2d_ctx *c) {
    return c->tree.x_ready ? c->tree.x_itemoff.as<int32_t>() : nullptr;
}

hipError_t p2l_all(fmm2d_ctx *c, int p) {
    TreeState &t = c->tree;
    if (!t.x_ready) return hipSuccess;
    EvalState &e = c->ev;
    const int64_t bound = t.x_item_bound > 0 ? t.x_item_bound : 1;
    FMM2D_TRY(e.xpart.ensure(sizeof(cd) * bound * (p + 1)));
    const int64_t nbox = level_offset(t.L + 1);
    hipLaunchKernelGGL(k_p2l, dim3(grid_for(bound, 4)), dim3(256), 0, c->stream, p, t.x_items.as<int4>(),
                       t.x_itemoff.as<int32_t>() + nbox, t.geom.as<double4>(), t.px.as<double>(), t.py.as<double>(),
                       e.qs.as<double>(), e.xpart.as<cd>());
    return hipGetLastError();
}

hipError_t m2p_all(fmm2d_ctx *c, int p, double *phi) {
    TreeState &t = c->tree;
    if (!t.x_ready) return hipSuccess;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    hipLaunchKernelGGL(k_m2p, dim3(grid_for(nleaf, 4)), dim3(256), 0, c->stream, p, L, nleaf,
                       t.starts.as<int32_t>() + depth_offset(2 * L), t.xptr.as<int32_t>(), t.xidx.as<int32_t>(),
                       t.pool_state.as<int64_t>() + 2 * (L + 2), t.geom.as<double4>(), c->ev.A.as<cd>(),
                       t.px.as<double>(), t.py.as<double>(), t.perm.as<int32_t>(), phi);
    return hipGetLastError();
}

}  // namespace fmm2d
