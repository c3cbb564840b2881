// Near field at the finest level (the direct sum over the strong lists,
// Section 4) fused with L2P, in binary64 or FP32.
//
// One wavefront per work item (target leaf b, chunk of TM consecutive points
// of b).  The targets are uniform across the wave; the lanes spread over the
// source points of S(b): GL lanes per source leaf (GL >= the largest leaf),
// 64/GL source leaves per step, so each lane loads one source and evaluates
// it against all TM targets held in registers.  A butterfly reduction then
// gives each target's sum, in a fixed order.  Every lane of a wave walks the
// same strong list, so the loop bounds are uniform.
//
// FP32 path: targets and sources are offsets from their own leaf centres;
// the centre difference c_b - c_c is formed in binary64 and rounded once per
// (lane, source leaf).  Coincident pairs contribute nothing, as in binary64:
// within a leaf they give exactly r^2 = 0, and across leaves a pair whose
// FP32 distance is below the rounding error of its own computation (a
// bound on it, carried in the record) counts as coincident.  L2P (binary64
// Horner) runs on lane k for target k.
#include "evaluate.h"
#include "wavesum.h"

namespace fmm2d {
namespace {

constexpr double HALF_LN2_D = 0.34657359027997264;  // ln(2)/2
constexpr int NWB = 4;                                // wavefronts per block

// FP32_ACC64 takes coordinate differences in two FP32 parts: every offset is
// hi + lo (lo the FP32 rounding of what hi leaves of the binary64 offset),
// and a source offset in the target leaf's frame, (sh + sl) - (dh + dl) with
// d the centre offset c_b - c_c, is formed by an exact two-term difference of
// the high parts (Knuth's TwoSum) with the low parts' difference added to
// its error term.  A pair's difference (th - h) + (tl - l) then has the
// relative accuracy of FP32 in the difference itself, not in the leaf size:
// close pairs in large leaves keep their logarithm (FP32 alone loses about
// 2^-24 R / r of it, R the leaf's radius, r the pair's distance).
__device__ inline void dd_sub(float sh, float sl, float dh, float dl, float &h, float &l) {
    h = sh - dh;
    const float bb = h - sh;
    const float err = (sh - (h - bb)) + (-dh - bb);
    l = err + (sl - dl);
}

// FP32 near field.  The segment's records (at most NEAR_SEG = 64, one per
// lane) are staged in the wavefront's LDS slice once; each step reads its
// record from LDS and the source points of the next step are loaded while the
// current step is evaluated (two steps per loop iteration, so the pipeline
// registers alternate instead of being copied).  Loads are unconditional
// (clamped to a valid point, then masked) so the loop has no branches.
// Requires the largest leaf to fit in GL lanes.
template <int TM, int GL, bool ACC64>
__global__ void __launch_bounds__(64 * NWB) k_near32(int64_t nitems, int chunks, const int32_t *__restrict__ stL,
                                                     const float4 *__restrict__ src, const float2 *__restrict__ srclo,
                                                     const int32_t *__restrict__ sptr,
                                                     const int2 *__restrict__ segtab, const int32_t *__restrict__ nseg_ptr,
                                                     const int2 *__restrict__ recj, const float4 *__restrict__ recd,
                                                     double *__restrict__ part) {
    static_assert(NEAR_SEG <= 64, "one record per lane");
    constexpr int LPI = 64 / GL;  // source leaves per step
    __shared__ int2 s_rj[NWB][64];
    __shared__ float4 s_rd[NWB][64];
    __shared__ float4 s_rl[NWB][ACC64 ? 64 : 1];
    const int64_t item = (int64_t)blockIdx.x * NWB + threadIdx.x / 64;
    if (item >= nitems) return;  // uniform per wavefront
    const int wv = threadIdx.x / 64;
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
    const int32_t t0 = se.y, t1 = (se.y + NEAR_SEG) < sptr[b + 1] ? (se.y + NEAR_SEG) : sptr[b + 1];
    // records of this segment; lanes past its end hold empty records
    {
        const bool ok = t0 + lane < t1;
        const int32_t tr = ok ? t0 + lane : t0;
        const int2 rj = recj[tr];
        const float4 rd = recd[2 * tr];
        s_rj[wv][lane] = ok ? rj : make_int2(0, 0);
        s_rd[wv][lane] = rd;
        if constexpr (ACC64) s_rl[wv][lane] = recd[2 * tr + 1];
    }
    float tx[TM], ty[TM], acc[TM];
    float txl[ACC64 ? TM : 1], tyl[ACC64 ? TM : 1];
    double tot64 = 0.0;  // ACC64: binary64 total of target lane / (64 / TM), added at each flush
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const float4 s = src[a + (k < nt ? k : 0)];
        tx[k] = s.x;
        ty[k] = s.y;
        acc[k] = 0.f;
        if constexpr (ACC64) {
            const float2 sl = srclo[a + (k < nt ? k : 0)];
            txl[k] = sl.x;
            tyl[k] = sl.y;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int grp = lane / GL, jj = lane % GL;
    const int nsteps = (t1 - t0 + LPI - 1) / LPI;
    // source point of lane jj in the record of step st; a lane past the end
    // of its source leaf loads a point of the array, moved far from every
    // target, and carries no charge, so the load needs no branch and its
    // pairs add exactly zero
    struct Src {
        float4 v;
        float2 l;
    };
    auto load_src = [&](int st) {
        const int2 rj = s_rj[wv][st * LPI + grp];
        const bool ok = jj < rj.y - rj.x;
        const int32_t j = ok ? rj.x + jj : 0;
        Src s;
        s.v = src[j];
        s.v.x = ok ? s.v.x : 0x1p60f;
        s.v.z = ok ? s.v.z : 0.f;
        s.l = ACC64 ? srclo[j] : make_float2(0.f, 0.f);
        return s;
    };
    auto eval = [&](const Src &sv, int st) {
        const float4 rd = s_rd[wv][st * LPI + grp];
        const float q = sv.v.z;
        float sx, sy, sxl = 0.f, syl = 0.f, thr;
        if constexpr (ACC64) {
            const float4 rl = s_rl[wv][st * LPI + grp];
            dd_sub(sv.v.x, sv.l.x, rd.x, rl.x, sx, sxl);
            dd_sub(sv.v.y, sv.l.y, rd.y, rl.y, sy, syl);
            thr = rl.z;
        } else {
            sx = sv.v.x - rd.x;
            sy = sv.v.y - rd.y;
            thr = rd.z;
        }
        float lg[TM], r2[ACC64 ? TM : 1];
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            if constexpr (ACC64) {
                const float dx = (tx[k] - sx) + (txl[k] - sxl), dy = (ty[k] - sy) + (tyl[k] - syl);
                r2[k] = dx * dx + dy * dy;
                lg[k] = __log2f(r2[k]);
            } else {
                const float dx = tx[k] - sx, dy = ty[k] - sy;
                lg[k] = __log2f(dx * dx + dy * dy);
            }
        }
        // every record of the step separated: the mask would change nothing
        if (!__all(rd.w != 0.f)) {
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                float rr;
                if constexpr (ACC64) {
                    rr = r2[k];
                } else {
                    const float dx = tx[k] - sx, dy = ty[k] - sy;
                    rr = dx * dx + dy * dy;
                }
                lg[k] = (rr > thr) ? lg[k] : 0.f;  // coincident: log is masked, never multiplied
            }
        }
#pragma unroll
        for (int k = 0; k < TM; ++k) acc[k] = fmaf(q, lg[k], acc[k]);
    };
    Src svA = load_src(0), svB;
    for (int st = 0; st < nsteps; st += 2) {
        const bool two = st + 1 < nsteps;
        if (two) svB = load_src(st + 1);
        eval(svA, st);
        if (two) {
            if (st + 2 < nsteps) svA = load_src(st + 2);
            eval(svB, st + 1);
        }
        if (ACC64 && (st & 15) == 14) {  // binary64 flush every 16 steps, summed over the lanes at once
            double v[TM];
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                v[k] = (double)acc[k];
                acc[k] = 0.f;
            }
            tot64 += wave_transpose_sum<TM>(v, lane);
        }
    }
    // the 64 lanes' partial sums of each target, by the transposing
    // butterfly (fixed order; binary64 with ACC64, else FP32): lane i
    // receives target i / (64 / TM)
    double tot;
    if constexpr (ACC64) {
        double v[TM];
#pragma unroll
        for (int k = 0; k < TM; ++k) v[k] = (double)acc[k];
        tot = tot64 + wave_transpose_sum<TM>(v, lane);
    } else {
        tot = (double)wave_transpose_sum<TM>(acc, lane);
    }
    constexpr int G = 64 / TM;
    if (lane % G == 0) part[item * TM + lane / G] = tot;
}

// FP32 near field taking each leaf pair once (leaves of 17 to 64 points).
// Work items cover the strong list of target leaf b from b's own entry on
// (sources c >= b; the lists are symmetric and ascending).  The log of a pair
// serves both sides: the target's sum (q_c log r, per target as below) and,
// when c != b, the source's (q_b log r, summed over the wavefront's targets
// in the source's lane and written to spart at leaf c's own entry for b, per
// lane, where leaf c's reduction reads its entries in order).  The four
// wavefronts of a block hold the four chunks of targets of one segment; their
// per-step source sums collect in an LDS ring of RING steps, added across the
// chunks once per group of steps (one barrier per group).  With ACC64 the
// FP32 partial sums go to binary64 every 16 steps, summed over the lanes by
// the transposing butterfly at once, so a lane keeps one binary64 total
// instead of TM.
//
// The segment's records (at most NEAR_SEG = 64, one per lane) are staged in
// the wavefront's LDS slice once, and their source points taken as one
// stream, 64 per step (a step may span two or three source leaves, so
// leaves of 33 to 63 points fill the lanes); the source points of the next
// step are loaded while the current step is evaluated (two steps per loop
// iteration, so the pipeline registers alternate instead of being copied).
template <int TM, int GL, int CH, bool ACC64>
__global__ void __launch_bounds__(64 * NWB) __attribute__((amdgpu_waves_per_eu(ACC64 ? 3 : 4))) k_near32s(int64_t nitems, const int32_t *__restrict__ stL,
                                                      const float4 *__restrict__ src, const float2 *__restrict__ srclo,
                                                      int32_t jfar,
                                                      const int32_t *__restrict__ sptr,
                                                      const int32_t *__restrict__ selfpos,
                                                      const int32_t *__restrict__ transU,
                                                      const int2 *__restrict__ segtab,
                                                      const int32_t *__restrict__ nseg_ptr,
                                                      const int2 *__restrict__ recj, const float4 *__restrict__ recd,
                                                      double *__restrict__ part, float *__restrict__ spart) {
    static_assert(NEAR_SEG <= 64, "one record per lane");
    static_assert(CH == NWB, "the chunks of one segment fill a block");
    static_assert(TM == 8 || TM == 10 || TM == 12 || TM == 16, "targets per wavefront");
    constexpr int NV = TM <= 8 ? 8 : 16;  // butterfly width (TM padded with zeros)
    constexpr int RING = 8;  // steps of source sums per exchange
    __shared__ int32_t s_base[NWB][64];  // source position of a record's flat index f: s_base + f
    __shared__ int32_t s_pre[NWB][64];   // first flat source index of each record
    __shared__ float4 s_rd[NWB][64];
    __shared__ float4 s_rl[NWB][ACC64 ? 64 : 1];
    __shared__ int32_t s_tu[NWB][64];
    __shared__ float s_ring[2][RING][NWB][64];
    const int wv = threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    const int64_t item = (int64_t)blockIdx.x * NWB + wv;
    if (item >= nitems) return;  // CH = 4: uniform per block (nitems is a multiple of NWB)
    const int64_t sg = item / CH;
    const int ch = (int)(item - sg * CH);
    if (sg >= *nseg_ptr) return;  // CH = 4: uniform per block
    const int2 se = segtab[sg];
    const int64_t b = se.x;
    const int32_t lb = stL[b], le = stL[b + 1];
    const int32_t a = lb + ch * TM;
    const int nt = (le - a) < 0 ? 0 : ((le - a) < TM ? (le - a) : TM);  // a chunk may be empty
    const int32_t t0 = se.y, t1 = (se.y + NEAR_SEG) < sptr[b + 1] ? (se.y + NEAR_SEG) : sptr[b + 1];
    const int32_t tself = selfpos[b];
    int32_t rend;  // lane r: one past the last flat index of record r (records past the segment: the total)
    {
        const bool ok = t0 + lane < t1;
        const int32_t tr = ok ? t0 + lane : t0;
        const int2 rj = recj[tr];
        const float4 rd = recd[2 * tr];
        s_rd[wv][lane] = rd;
        if constexpr (ACC64) s_rl[wv][lane] = recd[2 * tr + 1];
        s_tu[wv][lane] = (ok && tr != tself) ? transU[tr] : 0;
        // the records' source points as one stream, 64 per step: record r
        // holds flat indices s_pre[r] .. rend(r) - 1
        const int32_t size = ok ? rj.y - rj.x : 0;
        rend = wave_incl_scan(size);
        s_pre[wv][lane] = rend - size;
        s_base[wv][lane] = ok ? rj.x - (rend - size) : 0;
    }
    float tx[TM], ty[TM], tq[TM], acc[TM];
    float txl[ACC64 ? TM : 1], tyl[ACC64 ? TM : 1];
    double tot64 = 0.0;  // ACC64: binary64 total of target lane / (64 / TM), added at each flush
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const float4 s = src[k < nt ? a + k : lb];
        tx[k] = s.x;
        ty[k] = s.y;
        tq[k] = k < nt ? s.z : 0.f;  // absent targets send nothing to the sources
        acc[k] = 0.f;
        if constexpr (ACC64) {
            const float2 sl = srclo[k < nt ? a + k : lb];
            txl[k] = sl.x;
            tyl[k] = sl.y;
        }
    }
    __builtin_amdgcn_wave_barrier();
    const int32_t nflat = __builtin_amdgcn_readlane(rend, 63);
    const int nsteps = (nflat + 63) / 64;
    struct Src {
        float3 v;   // x, y, q (three words: no dead register left for the compiler to reuse while the load is in flight)
        float2 l;
        int r;      // the lane's record in this step
        float3 rd;  // its centre offset (x, y) and coincidence threshold (z; FP32)
        float3 rl;  // with ACC64: the offset's low part (x, y) and the two-part threshold (z)
    };
    // record of flat index f = 64 st + lane (below nflat): the number of
    // records ending at or before f.  Those ending before the step are
    // counted at once by a ballot; the few ending inside it (a step of 64
    // spans at most 64 / (smallest leaf) + 1 records) one by one, uniformly.
    auto record_of = [&](int st) {
        const int32_t f = 64 * st + lane;
        const int r_lo = __popcll(__ballot(rend <= 64 * st));
        const int r_hi = __popcll(__ballot(rend <= 64 * st + 63));
        int r = r_lo;
        for (int i = r_lo; i < r_hi; ++i) r += (f >= __builtin_amdgcn_readlane(rend, i)) ? 1 : 0;
        return r;
    };
    // loads of one step, used a step later (nothing here waits for them)
    auto load_src = [&](int st) {  // a lane past the stream loads the far point, which has no charge
        const int32_t f = 64 * st + lane;
        const bool ok = f < nflat;
        int r = record_of(st);  // with every lane active: the ballots read all records
        r = ok ? r : 0;
        const int32_t j = ok ? s_base[wv][r] + f : jfar;
        Src s;
        s.v = *reinterpret_cast<const float3 *>(src + j);
        s.l = ACC64 ? srclo[j] : make_float2(0.f, 0.f);
        s.r = r;
        s.rd = *reinterpret_cast<const float3 *>(&s_rd[wv][r]);
        if constexpr (ACC64) s.rl = *reinterpret_cast<const float3 *>(&s_rl[wv][r]);
        return s;
    };
    // The source sums of RING steps collect in one half of s_ring; at the
    // last step of the group (or of the segment) the block meets once, and
    // each wavefront adds the four chunks' sums of RING / NWB of the steps
    // (chunk order, as one block-wide sum would) and writes them to spart at
    // leaf c's own entry for b.  The other half takes the next group, so one
    // barrier per group suffices.
    auto exchange = [&](int st_last) {
        __syncthreads();
        const int base = st_last & ~(RING - 1);
        const int half = (st_last / RING) & 1;
#pragma unroll
        for (int u = 0; u < RING / NWB; ++u) {
            const int st = base + wv * (RING / NWB) + u;
            if (st > st_last) break;  // uniform per wavefront
            const int32_t f = 64 * st + lane;
            const int r = record_of(st);
            if (f < nflat && t0 + r != tself) {
                float v = 0.f;
#pragma unroll
                for (int w = 0; w < NWB; ++w) v += s_ring[half][st & (RING - 1)][w][lane];
                spart[(int64_t)s_tu[wv][r] * GL + (f - s_pre[wv][r])] = v;  // leaf c's own entry for b
            }
        }
    };
    // one step: both sides of every pair of this lane's source and the
    // wavefront's targets
    auto eval = [&](const Src &sv, int st) {
        const float3 rd = sv.rd;
        const float q = sv.v.z;
        float sx, sy, sxl = 0.f, syl = 0.f, thr;
        if constexpr (ACC64) {
            const float3 rl = sv.rl;
            dd_sub(sv.v.x, sv.l.x, rd.x, rl.x, sx, sxl);
            dd_sub(sv.v.y, sv.l.y, rd.y, rl.y, sy, syl);
            thr = rl.z;
        } else {
            sx = sv.v.x - rd.x;
            sy = sv.v.y - rd.y;
            thr = rd.z;
        }
        float sacc = 0.f, lg[TM], r2[TM];
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            if constexpr (ACC64) {
                const float dx = (tx[k] - sx) + (txl[k] - sxl), dy = (ty[k] - sy) + (tyl[k] - syl);
                r2[k] = dx * dx + dy * dy;
            } else {
                const float dx = tx[k] - sx, dy = ty[k] - sy;
                r2[k] = dx * dx + dy * dy;
            }
            lg[k] = __log2f(r2[k]);
        }
        // the coincidence mask only where some pair of the step is within its
        // threshold (a point with itself in the leaf's own record, duplicates)
        float rmin = r2[0];
#pragma unroll
        for (int k = 1; k < TM; ++k) rmin = fminf(rmin, r2[k]);
        if (!__all(rmin > thr)) {
#pragma unroll
            for (int k = 0; k < TM; ++k) lg[k] = (r2[k] > thr) ? lg[k] : 0.f;  // coincident: log is masked, never multiplied
        }
#pragma unroll
        for (int k = 0; k < TM; ++k) {
            acc[k] = fmaf(q, lg[k], acc[k]);
            sacc = fmaf(tq[k], lg[k], sacc);
        }
        s_ring[(st / RING) & 1][st & (RING - 1)][wv][lane] = sacc;
        if ((st & (RING - 1)) == RING - 1 || st == nsteps - 1) exchange(st);  // uniform per block
    };
    // the loads are not conditional (a step past the stream loads the far
    // point): on every path the same loads are in flight, so the wait before
    // an evaluation covers only the loads it uses
    Src svA = load_src(0), svB;
    for (int st = 0; st < nsteps; st += 2) {
        svB = load_src(st + 1);
        eval(svA, st);
        svA = load_src(st + 2);
        if (st + 1 < nsteps) eval(svB, st + 1);
        if (ACC64 && (st & 15) == 14) {  // binary64 flush every 16 steps, summed over the lanes at once
            double v[NV];
#pragma unroll
            for (int k = 0; k < NV; ++k) {
                v[k] = k < TM ? (double)acc[k < TM ? k : 0] : 0.0;
                if (k < TM) acc[k] = 0.f;
            }
            tot64 += wave_transpose_sum<NV>(v, lane);
        }
    }
    // the 64 lanes' partial sums of each target, by the transposing
    // butterfly (fixed order; binary64 with ACC64, else FP32): lane i
    // receives target i / (64 / NV)
    double tot;
    if constexpr (ACC64) {
        double v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = k < TM ? (double)acc[k < TM ? k : 0] : 0.0;
        tot = tot64 + wave_transpose_sum<NV>(v, lane);
    } else {
        float v[NV];
#pragma unroll
        for (int k = 0; k < NV; ++k) v[k] = k < TM ? acc[k < TM ? k : 0] : 0.f;
        tot = (double)wave_transpose_sum<NV>(v, lane);
    }
    constexpr int G = 64 / NV;
    if (lane % G == 0 && lane / G < TM) part[item * TM + lane / G] = tot;
}

// FP32 near field for leaves larger than 64 points: a lane walks its source
// leaf 64 points at a time (not pipelined).
template <int TM, bool ACC64>
__global__ void __launch_bounds__(64 * NWB) k_near32_big(int64_t nitems, int chunks, int maxleaf,
                                                         const int32_t *__restrict__ stL,
                                                         const float4 *__restrict__ src,
                                                         const float2 *__restrict__ srclo,
                                                         const int32_t *__restrict__ sptr,
                                                         const int2 *__restrict__ segtab,
                                                         const int32_t *__restrict__ nseg_ptr,
                                                         const int2 *__restrict__ recj,
                                                         const float4 *__restrict__ recd, double *__restrict__ part) {
    const int64_t item = (int64_t)blockIdx.x * NWB + threadIdx.x / 64;
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
    float tx[TM], ty[TM], acc[TM];
    float txl[ACC64 ? TM : 1], tyl[ACC64 ? TM : 1];
    double acc64[TM];
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const float4 s = src[a + (k < nt ? k : 0)];
        tx[k] = s.x;
        ty[k] = s.y;
        acc[k] = 0.f;
        acc64[k] = 0.0;
        if constexpr (ACC64) {
            const float2 sl = srclo[a + (k < nt ? k : 0)];
            txl[k] = sl.x;
            tyl[k] = sl.y;
        }
    }
    const int32_t t0 = se.y, t1 = (se.y + NEAR_SEG) < sptr[b + 1] ? (se.y + NEAR_SEG) : sptr[b + 1];
    for (int32_t t = t0; t < t1; ++t) {
        const int2 rj = recj[t];
        const float4 rd = recd[2 * t];
        const float4 rl = ACC64 ? recd[2 * t + 1] : make_float4(0.f, 0.f, 0.f, 0.f);
        const float thr = ACC64 ? rl.z : rd.z;
        for (int jb = 0; jb < maxleaf; jb += 64) {
            const int32_t j = rj.x + jb + lane;
            float sx = 1e18f, sy = 1e18f, sxl = 0.f, syl = 0.f, q = 0.f;
            if (j < rj.y) {
                const float4 s = src[j];
                if constexpr (ACC64) {
                    const float2 sl = srclo[j];
                    dd_sub(s.x, sl.x, rd.x, rl.x, sx, sxl);
                    dd_sub(s.y, sl.y, rd.y, rl.y, sy, syl);
                } else {
                    sx = s.x - rd.x;
                    sy = s.y - rd.y;
                }
                q = s.z;
            }
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                float dx, dy;
                if constexpr (ACC64) {
                    dx = (tx[k] - sx) + (txl[k] - sxl);
                    dy = (ty[k] - sy) + (tyl[k] - syl);
                } else {
                    dx = tx[k] - sx;
                    dy = ty[k] - sy;
                }
                const float r2 = dx * dx + dy * dy;
                const float lg = __log2f(r2);
                acc[k] = fmaf(q, (r2 > thr) ? lg : 0.f, acc[k]);
            }
        }
        if (ACC64) {
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                acc64[k] += (double)acc[k];
                acc[k] = 0.f;
            }
        }
    }
    double mine = 0.0;
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        double v = ACC64 ? acc64[k] + (double)acc[k] : (double)acc[k];
        if (ACC64) {
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        } else {
            float w = acc[k];
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) w += __shfl_xor(w, off, 64);
            v = (double)w;
        }
        if (lane == k) mine = v;
    }
    if (lane < TM) part[item * TM + lane] = mine;
}

// Binary64 near field, same decomposition; sources (x, y, q) in binary64.
template <int TM, int GL>
__global__ void __launch_bounds__(64 * NWB) k_near64(int64_t nitems, int chunks, int maxleaf,
                                                     const int32_t *__restrict__ stL, const double *__restrict__ px,
                                                     const double *__restrict__ py, const double *__restrict__ qs,
                                                     const int32_t *__restrict__ sptr, const int2 *__restrict__ segtab,
                                                     const int32_t *__restrict__ nseg_ptr,
                                                     const int2 *__restrict__ recj, double *__restrict__ part) {
    constexpr int LPI = 64 / GL;
    const int64_t item = (int64_t)blockIdx.x * NWB + threadIdx.x / 64;
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
    double tx[TM], ty[TM], acc[TM];
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        const int32_t i = a + (k < nt ? k : 0);
        tx[k] = px[i];
        ty[k] = py[i];
        acc[k] = 0.0;
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
            double sx = 1e300, sy = 1e300, q = 0.0;
            if (ok) {
                sx = px[j];
                sy = py[j];
                q = qs[j];
            }
#pragma unroll
            for (int k = 0; k < TM; ++k) {
                const double dx = tx[k] - sx, dy = ty[k] - sy;
                acc[k] += (ok && (dx != 0.0 || dy != 0.0)) ? q * log_pos(dx * dx + dy * dy) : 0.0;
            }
        }
    }
    double mine = 0.0;
#pragma unroll
    for (int k = 0; k < TM; ++k) {
        double v = acc[k];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
        if (lane == k) mine = v;
    }
    if (lane < TM) part[item * TM + lane] = mine;
}

// FP32 sources (offset from the leaf centre, charge); with `lo`, the low
// parts of the offsets for the two-part differences of FP32_ACC64.
__global__ void k_pack_sources(const float2 *__restrict__ loc, const double *__restrict__ qs, int64_t n,
                               float4 *__restrict__ src, const double *__restrict__ px, const double *__restrict__ py,
                               const int32_t *__restrict__ leafid, const double4 *__restrict__ geomL,
                               float2 *__restrict__ lo) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const float2 l = loc[i];
        src[i] = make_float4(l.x, l.y, (float)qs[i], 0.0f);
        if (lo) {
            const double4 g = geomL[leafid[i]];
            lo[i] = make_float2((float)((px[i] - g.x) - (double)l.x), (float)((py[i] - g.y) - (double)l.y));
        }
    } else if (i == n) {
        // entry n: a chargeless point far from every leaf (finite logs), which
        // idle lanes of the pair-once kernel load instead of masking
        src[n] = make_float4(0x1p60f, 0.f, 0.f, 0.f);
        if (lo) lo[n] = make_float2(0.f, 0.f);
    }
}

// L2P: the local expansion B[0..p] at z (scaled offset) by Horner, the
// coefficients loaded four at a time ahead of their use.
__device__ inline cd l2p_horner(const cd *__restrict__ Bb, int p, cd z) {
    cd v = Bb[p];
    int l = p - 1;
    for (; l >= 3; l -= 4) {
        const cd b0 = Bb[l], b1 = Bb[l - 1], b2 = Bb[l - 2], b3 = Bb[l - 3];
        v = cadd(cmul(v, z), b0);
        v = cadd(cmul(v, z), b1);
        v = cadd(cmul(v, z), b2);
        v = cadd(cmul(v, z), b3);
    }
    for (; l >= 0; --l) v = cadd(cmul(v, z), Bb[l]);
    return v;
}

// Per point: the partial sums of its leaf's segments in segment order, times
// `scale`, plus L2P (binary64 Horner) of the leaf's local expansion and the
// exchanged-roles M2P sums.
__global__ void k_near_reduce(int p, int64_t n, int tm, int chunks, double scale, const int32_t *__restrict__ leafid,
                              const int32_t *__restrict__ stL, const int32_t *__restrict__ segoff,
                              const double *__restrict__ part, const double4 *__restrict__ geomL,
                              const double *__restrict__ px, const double *__restrict__ py,
                              const cd *__restrict__ BL, const int32_t *__restrict__ perm,
                              double *__restrict__ phi, int L, M2PSum ms) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = leafid[i];
    const int32_t off = (int32_t)(i - stL[b]);
    const int ch = off / tm, k = off - ch * tm;
    double near = 0.0;
    for (int32_t sg = segoff[b]; sg < segoff[b + 1]; ++sg) near += part[((int64_t)sg * chunks + ch) * tm + k];
    const double4 g = geomL[b];
    const cd z{(px[i] - g.x) / g.w, (py[i] - g.y) / g.w};
    const cd v = l2p_horner(BL + (int64_t)b * (p + 1), p, z);
    const double xm = ms.itemoff ? m2p_point_sum(ms, L, i, b, stL) : 0.0;  // exchanged roles, M2P
    phi[perm[i]] = (v.re + scale * near) + xm;  // input order
}

// Source-side sums of the entries of S_L(c) before c's own (written there by
// the near field), one wavefront per segment of at most NEAR_SEG entries: lane
// group g of 64 / GL takes entries g, g + 64/GL, ..., then the groups are
// added (fixed order) and lane jj < GL writes the segment's sum for point jj.
template <int GL>
__global__ void __launch_bounds__(256) k_near_lsum(const int2 *__restrict__ segtab,
                                                   const int32_t *__restrict__ nseg_ptr,
                                                   const int32_t *__restrict__ selfpos, const float *__restrict__ spart,
                                                   const int32_t *__restrict__ stL, double *__restrict__ lsum) {
    constexpr int LPI = 64 / GL;
    const int64_t sg = (int64_t)blockIdx.x * 4 + threadIdx.x / 64;
    if (sg >= *nseg_ptr) return;  // uniform per wavefront
    const int lane = threadIdx.x % 64, grp = lane / GL, jj = lane % GL;
    const int2 se = segtab[sg];
    // lanes past the leaf's points read nothing (their sums are never used)
    const int32_t u1 = jj >= stL[se.x + 1] - stL[se.x] ? se.y
                       : ((se.y + NEAR_SEG) < selfpos[se.x] ? (se.y + NEAR_SEG) : selfpos[se.x]);
    double v = 0.0;
    int32_t u = se.y + grp;
    for (; u + 3 * LPI < u1; u += 4 * LPI) {  // four loads in flight, added in entry order
        const float f0 = spart[(int64_t)u * GL + jj], f1 = spart[(int64_t)(u + LPI) * GL + jj];
        const float f2 = spart[(int64_t)(u + 2 * LPI) * GL + jj], f3 = spart[(int64_t)(u + 3 * LPI) * GL + jj];
        v = (((v + (double)f0) + (double)f1) + (double)f2) + (double)f3;
    }
    for (; u < u1; u += LPI) v += (double)spart[(int64_t)u * GL + jj];
#pragma unroll
    for (int off = GL; off < 64; off <<= 1) v += __shfl_xor(v, off, 64);
    if (lane < GL) lsum[sg * GL + jj] = v;
}

// Per point of the pair-once path: its leaf's target-side segment sums, then
// the source-side sums of the leaves c < b (segment sums of the entries of
// S_L(b) before b's own), times `scale`, plus L2P and the exchanged-roles M2P
// sums.
__global__ void k_near_reduce_sym(int p, int64_t n, int tm, int ch_n, int gl, double scale,
                                  const int32_t *__restrict__ leafid, const int32_t *__restrict__ stL,
                                  const int32_t *__restrict__ segoff, const double *__restrict__ part,
                                  const int32_t *__restrict__ losegoff, const double *__restrict__ lsum,
                                  const double4 *__restrict__ geomL, const double *__restrict__ px,
                                  const double *__restrict__ py, const cd *__restrict__ BL,
                                  const int32_t *__restrict__ perm, double *__restrict__ phi, int L, M2PSum ms) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t b = leafid[i];
    const int32_t off = (int32_t)(i - stL[b]);
    const int ch = off / tm, k = off - ch * tm;
    double near = 0.0;
    for (int32_t sg = segoff[b]; sg < segoff[b + 1]; ++sg) near += part[((int64_t)sg * ch_n + ch) * tm + k];
    for (int32_t sg = losegoff[b]; sg < losegoff[b + 1]; ++sg) near += lsum[(int64_t)sg * gl + off];
    const double4 g = geomL[b];
    const cd z{(px[i] - g.x) / g.w, (py[i] - g.y) / g.w};
    const cd v = l2p_horner(BL + (int64_t)b * (p + 1), p, z);
    const double xm = ms.itemoff ? m2p_point_sum(ms, L, i, b, stL) : 0.0;  // exchanged roles, M2P
    phi[perm[i]] = (v.re + scale * near) + xm;  // input order
}

// FP32 paths with leaves of at most 64 points: each leaf pair once.  Stage
// NEAR_LAUNCH queues the pair kernel and the lower-segment sums on the second
// stream (after the transposed positions, queued there by the list build),
// NEAR_FINISH the reduction with L2P on the context stream.
template <int TM, int GL, int CH>
hipError_t launch_near_sym(fmm2d_ctx *c, int p, int mode, int stage, double *phi) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const Schedule &sc = t.near_up;
    const int64_t nitems = sc.bound * CH;  // CH = 4: one block per segment
    const int64_t offL = level_offset(L);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const double4 *gL = t.geom.as<double4>() + offL;
    const cd *BL = e.B.as<cd>() + offL * (p + 1);
    const int32_t *sp = t.sptr.as<int32_t>() + ptr_offset(L);
    const int64_t ns = t.s_off[L + 1] - t.s_off[L];
    const Schedule &lo = t.near_lo;
    if (stage == NEAR_PREP) {
        FMM2D_TRY(e.npart.ensure(sizeof(double) * (nitems > 0 ? nitems : 1) * TM));
        FMM2D_TRY(t.spart.ensure(sizeof(float) * (size_t)(ns > 0 ? ns : 1) * GL));
        FMM2D_TRY(t.lsum.ensure(sizeof(double) * (size_t)(lo.bound > 0 ? lo.bound : 1) * GL));
        return side_begin(c);  // the packed sources
    }
    double *part = e.npart.as<double>();
    float *spart = t.spart.as<float>();
    if (stage == NEAR_FINISH) {
        FMM2D_TRY(side_join(c));
        hipLaunchKernelGGL(k_near_reduce_sym, dim3(grid_for(t.n, 256)), dim3(256), 0, c->stream, p, t.n, TM, CH, GL,
                           HALF_LN2_D, t.leafid.as<int32_t>(), stL, sc.segoff.as<int32_t>(), part,
                           lo.segoff.as<int32_t>(), t.lsum.as<double>(), gL, t.px.as<double>(), t.py.as<double>(),
                           BL, t.perm.as<int32_t>(), phi, L, e.m2p);
        return hipGetLastError();
    }
    const dim3 grid(grid_for(nitems, NWB)), block(64 * NWB);
    {
        PhaseScope kernel_scope(c, PH_NEAR_KERNEL, c->side);  // the near-field kernel alone
        if (mode == FMM2D_MODE_FP32_ACC64)
            hipLaunchKernelGGL((k_near32s<TM, GL, CH, true>), grid, block, 0, c->side, nitems, stL,
                               e.src.as<float4>(), e.srclo.as<float2>(), (int32_t)t.n, sp, t.selfpos.as<int32_t>(),
                               t.trans.as<int32_t>(),
                               sc.table.as<int2>(),
                               sc.segoff.as<int32_t>() + nleaf, t.nrec_j.as<int2>(), t.nrec_d.as<float4>(), part,
                               spart);
        else
            hipLaunchKernelGGL((k_near32s<TM, GL, CH, false>), grid, block, 0, c->side, nitems, stL,
                               e.src.as<float4>(), nullptr, (int32_t)t.n, sp, t.selfpos.as<int32_t>(), t.trans.as<int32_t>(),
                               sc.table.as<int2>(),
                               sc.segoff.as<int32_t>() + nleaf, t.nrec_j.as<int2>(), t.nrec_d.as<float4>(), part,
                               spart);
    }
    FMM2D_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_near_lsum<GL>, dim3(grid_for(lo.bound > 0 ? lo.bound : 1, 4)), dim3(256), 0, c->side,
                       lo.table.as<int2>(), lo.segoff.as<int32_t>() + nleaf, t.selfpos.as<int32_t>(), spart, stL,
                       t.lsum.as<double>());
    FMM2D_TRY(hipGetLastError());
    return side_end(c);
}

// Every ordered leaf pair (one-sided kernels); stages as in launch_near_sym.
template <int TM, int GL>
hipError_t launch_near(fmm2d_ctx *c, int p, int mode, int maxleaf, int stage, double *phi) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const Schedule &sc = t.near_seg;
    const int chunks = (maxleaf + TM - 1) / TM;
    const int64_t nitems = sc.bound * chunks;
    const int64_t offL = level_offset(L);
    const int32_t *stL = t.starts.as<int32_t>() + depth_offset(2 * L);
    const double4 *gL = t.geom.as<double4>() + offL;
    const cd *BL = e.B.as<cd>() + offL * (p + 1);
    const int32_t *sp = t.sptr.as<int32_t>() + ptr_offset(L);
    const int2 *rj = t.nrec_j.as<int2>();
    const float4 *rd = t.nrec_d.as<float4>();
    const int2 *tab = sc.table.as<int2>();
    const int32_t *nsp = sc.segoff.as<int32_t>() + nleaf;
    if (stage == NEAR_PREP) {
        FMM2D_TRY(e.npart.ensure(sizeof(double) * (nitems > 0 ? nitems : 1) * TM));
        return side_begin(c);  // the packed sources (charges in leaf order for binary64)
    }
    double *part = e.npart.as<double>();
    const double scale = mode == FMM2D_MODE_FP64 ? 0.5 : HALF_LN2_D;
    if (stage == NEAR_FINISH) {
        FMM2D_TRY(side_join(c));
        hipLaunchKernelGGL(k_near_reduce, dim3(grid_for(t.n, 256)), dim3(256), 0, c->stream, p, t.n, TM, chunks,
                           scale, t.leafid.as<int32_t>(), stL, sc.segoff.as<int32_t>(), part, gL, t.px.as<double>(),
                           t.py.as<double>(), BL, t.perm.as<int32_t>(), phi, L, e.m2p);
        return hipGetLastError();
    }
    const dim3 grid(grid_for(nitems, NWB)), block(64 * NWB);
    {
        PhaseScope kernel_scope(c, PH_NEAR_KERNEL, c->side);  // the near-field kernel alone
        if (mode == FMM2D_MODE_FP64) {
            hipLaunchKernelGGL((k_near64<TM, GL>), grid, block, 0, c->side, nitems, chunks, maxleaf, stL,
                               t.px.as<double>(), t.py.as<double>(), e.qs.as<double>(), sp, tab, nsp, rj, part);
        } else {
            if (maxleaf > 64) {
                if (mode == FMM2D_MODE_FP32_ACC64)
                    hipLaunchKernelGGL((k_near32_big<TM, true>), grid, block, 0, c->side, nitems, chunks, maxleaf, stL,
                                       e.src.as<float4>(), e.srclo.as<float2>(), sp, tab, nsp, rj, rd, part);
                else
                    hipLaunchKernelGGL((k_near32_big<TM, false>), grid, block, 0, c->side, nitems, chunks, maxleaf, stL,
                                       e.src.as<float4>(), nullptr, sp, tab, nsp, rj, rd, part);
            } else if (mode == FMM2D_MODE_FP32_ACC64) {
                hipLaunchKernelGGL((k_near32<TM, GL, true>), grid, block, 0, c->side, nitems, chunks, stL,
                                   e.src.as<float4>(), e.srclo.as<float2>(), sp, tab, nsp, rj, rd, part);
            } else {
                hipLaunchKernelGGL((k_near32<TM, GL, false>), grid, block, 0, c->side, nitems, chunks, stL,
                                   e.src.as<float4>(), nullptr, sp, tab, nsp, rj, rd, part);
            }
        }
    }
    FMM2D_TRY(hipGetLastError());
    return side_end(c);
}

}  // namespace

// L2P plus the near field for every point; writes phi (input order).
hipError_t leaf_pass(fmm2d_ctx *c, int p, int mode, int stage, double *phi) {
    TreeState &t = c->tree;
    EvalState &e = c->ev;
    const int64_t n = t.n;
    const int L = t.L;
    const int64_t nleaf = int64_t(1) << (2 * L);
    const int64_t maxleaf = (n + nleaf - 1) >> (2 * L);  // ceil(n / 4^L)
    if (!t.nrec_valid) return hipErrorInvalidValue;  // records come with the lists
    if (stage == NEAR_PREP && mode != FMM2D_MODE_FP64) {
        FMM2D_TRY(e.src.ensure(sizeof(float4) * (n + 1)));  // and the far point
        float2 *lo = nullptr;
        if (mode == FMM2D_MODE_FP32_ACC64) {
            FMM2D_TRY(e.srclo.ensure(sizeof(float2) * (n + 1)));
            lo = e.srclo.as<float2>();
        }
        hipLaunchKernelGGL(k_pack_sources, dim3(grid_for(n + 1, 256)), dim3(256), 0, c->stream, t.loc.as<float2>(),
                           e.qs.as<double>(), n, e.src.as<float4>(), t.px.as<double>(), t.py.as<double>(),
                           t.leafid.as<int32_t>(), t.geom.as<double4>() + level_offset(L), lo);
    }
    // GL lanes per source leaf: the smallest power of two >= the largest leaf
    // (capped at 64; larger leaves take the non-pipelined kernel)
    const int ml = (int)(maxleaf < (int64_t)1 << 30 ? maxleaf : (int64_t)1 << 30);
    if (mode != FMM2D_MODE_FP64 && pair_once_leaves(ml)) {
        // each leaf pair once, the four chunks of targets of a leaf in the
        // four wavefronts of a block
        if (ml <= 32) return launch_near_sym<8, 32, 4>(c, p, mode, stage, phi);
        if (ml <= 40) return launch_near_sym<10, 64, 4>(c, p, mode, stage, phi);  // 4 chunks of 10 targets
        if (ml <= 48) return launch_near_sym<12, 64, 4>(c, p, mode, stage, phi);  // 4 chunks of 12 targets
        return launch_near_sym<16, 64, 4>(c, p, mode, stage, phi);
    }
    if (stage == NEAR_PREP) FMM2D_TRY(ensure_near_full_schedule(c));  // on the context stream, before the second stream waits
    if (ml <= 8) return launch_near<8, 8>(c, p, mode, ml, stage, phi);
    if (ml <= 16) return launch_near<16, 16>(c, p, mode, ml, stage, phi);
    if (ml <= 32) return launch_near<16, 32>(c, p, mode, ml, stage, phi);
    return launch_near<16, 64>(c, p, mode, ml, stage, phi);
}

}  // namespace fmm2d
