// Balanced median-split pyramid (Section 4, Fig. 1.1) on the GPU.
//
// Design.  Both coordinates are sorted once by (value, index).  A point is
// then represented by its two ranks (x rank, y rank); comparing ranks is
// comparing (value, index) pairs.  Two lists are kept, partitioned into the
// current boxes ("segments"): XL, each segment in x-rank order, and YL, each
// segment in y-rank order.  Splitting a segment of m points along x needs no
// selection: its low side is the first floor(m/2) entries of its XL part, so
// the median is the entry at floor(m/2) and a point is low iff its x rank is
// below that entry's.  XL is already partitioned by this split; YL is
// partitioned stably by the flag (x rank < median rank), which keeps it in
// y-rank order inside each half.  The y split of each half is the mirror
// image (YL gives the median, XL is partitioned).  Segment sizes never depend
// on the data: a segment of m points has floor(m/2) low points, so all
// segment offsets are known before a level is examined, and the stable
// partition needs only a global prefix count of the low flags.
#include "devutil.h"
#include "internal.h"

namespace fmm2d {
namespace {

constexpr int PT = 256;     // threads per partition block
constexpr int PI = 4;       // items per thread (striped)
constexpr int PTILE = PT * PI;

struct Rect {
    double xlo, xhi, ylo, yhi;
};

// Segment of depth h holding list position i, and its range [a, e): the
// split of [a, e) puts floor((e - a) / 2) positions low, so the path from the
// root follows from i alone (no table lookups).  Segment s of depth 2l is box
// s of level l.
__device__ inline int64_t seg_of(int64_t i, int64_t n, int h, int32_t &a, int32_t &e) {
    int32_t lo = 0, hi = (int32_t)n;
    const int32_t ii = (int32_t)i;
    int64_t s = 0;
    for (int d = 0; d < h; ++d) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        const bool up = ii >= mid;
        s = 2 * s + (up ? 1 : 0);
        lo = up ? mid : lo;
        hi = up ? hi : mid;
    }
    a = lo;
    e = hi;
    return s;
}

__global__ void k_root(const double *__restrict__ xs, const double *__restrict__ ys, int64_t n,
                       int32_t *__restrict__ st0, Rect *__restrict__ rects) {
    st0[0] = 0;
    st0[1] = (int32_t)n;
    rects[0] = Rect{xs[0], xs[n - 1], ys[0], ys[n - 1]};
}

__global__ void k_init_lists(const int32_t *__restrict__ xorder, const int32_t *__restrict__ yorder,
                             const int32_t *__restrict__ xrank, const int32_t *__restrict__ yrank, int64_t n,
                             int32_t *__restrict__ XLx, int32_t *__restrict__ XLy, int32_t *__restrict__ YLx,
                             int32_t *__restrict__ YLy) {
    int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) {
        XLx[r] = (int32_t)r;
        XLy[r] = yrank[xorder[r]];
        YLy[r] = (int32_t)r;
        YLx[r] = xrank[yorder[r]];
    }
}

// Per segment of depth h: split line, child offsets, and (after a y split)
// the four child rectangles.
__device__ inline void segment_record(int h, int64_t s, int64_t nseg, int64_t n, const int32_t *__restrict__ st,
                                      int32_t *__restrict__ st1, const int32_t *__restrict__ med_list,
                                      const double *__restrict__ coord, double *__restrict__ split_cur,
                                      const double *__restrict__ split_prev, Rect *__restrict__ rects) {
    const int32_t a = st[s], e = st[s + 1];
    const int32_t k = (e - a) >> 1;  // >= 1: every segment above the leaves holds >= 2 points
    const int32_t r_hi = med_list[a + k], r_lo = med_list[a + k - 1];
    const double sp = 0.5 * (coord[r_lo] + coord[r_hi]);
    split_cur[s] = sp;
    st1[2 * s] = a;
    st1[2 * s + 1] = a + k;
    if (s == nseg - 1) st1[2 * nseg] = (int32_t)n;
    if (h & 1) {
        const int l = (h - 1) >> 1;
        const int64_t b = s >> 1;
        const int xside = (int)(s & 1);
        const Rect R = rects[level_offset(l) + b];
        const double sx = split_prev[b];
        const double xlo = xside ? sx : R.xlo;
        const double xhi = xside ? R.xhi : sx;
        const int64_t c0 = level_offset(l + 1) + 4 * b + 2 * xside;
        rects[c0] = Rect{xlo, xhi, R.ylo, sp};
        rects[c0 + 1] = Rect{xlo, xhi, sp, R.yhi};
    }
}

// Tiles of PTILE consecutive list positions, read striped (position
// base + r * PT + thread), so that every load is coalesced.  Inside a tile the
// low flags are ranked in position order by per-round wave ballots: the rank
// of round r, wave w, lane j is (low flags of rounds < r) + (of waves < w in
// round r) + (of lanes < j).
struct TileRank {
    int32_t before_round[PI];  // low flags of the tile before round r
    int32_t wave_off[PI];      // low flags of round r in the waves before this one
    int32_t total;
};

__device__ inline void tile_rank(const uint64_t *bal, int32_t (*wc)[PT / WAVE], TileRank &tr) {
    const int w = threadIdx.x / WAVE;
    if (lane_id() == 0) {
#pragma unroll
        for (int r = 0; r < PI; ++r) wc[r][w] = (int32_t)__popcll(bal[r]);
    }
    __syncthreads();
    int32_t run = 0;
#pragma unroll
    for (int r = 0; r < PI; ++r) {
        tr.before_round[r] = run;
        int32_t off = 0;
#pragma unroll
        for (int q = 0; q < PT / WAVE; ++q) {
            const int32_t v = wc[r][q];
            off += (q < w) ? v : 0;
            run += v;
        }
        tr.wave_off[r] = off;
    }
    tr.total = run;
}

// Blocks [0, ntile): count the low flags of each tile, and for every segment
// that starts in the tile, the low flags of the tile before its start.
// Blocks [ntile, ...): one thread per segment, segment_record.
__global__ void __launch_bounds__(PT) k_part_count(int h, const int32_t *__restrict__ key, int64_t n, int ntile,
                                                   const int32_t *__restrict__ st, int64_t nseg,
                                                   const int32_t *__restrict__ med_list,
                                                   int32_t *__restrict__ tcount, int32_t *__restrict__ segbase_local,
                                                   int32_t *__restrict__ st1, const double *__restrict__ coord,
                                                   double *__restrict__ split_cur,
                                                   const double *__restrict__ split_prev, Rect *__restrict__ rects) {
    if ((int)blockIdx.x >= ntile) {
        const int64_t s = (int64_t)(blockIdx.x - ntile) * PT + threadIdx.x;
        if (s < nseg) segment_record(h, s, nseg, n, st, st1, med_list, coord, split_cur, split_prev, rects);
        return;
    }
    __shared__ int32_t wc[PI][PT / WAVE];
    const int64_t base = (int64_t)blockIdx.x * PTILE + threadIdx.x;
    uint64_t bal[PI];
    int32_t segs[PI];  // segment starting at this position, or -1
    int32_t kv[PI], mv[PI];
    // every load in flight first (positions clamped into the list, so the
    // loads need no branch); positions >= n are flagged low and start nothing
#pragma unroll
    for (int r = 0; r < PI; ++r) {
        const int64_t i = base + (int64_t)r * PT;
        const int64_t ic = i < n ? i : n - 1;
        int32_t a, e;
        const int64_t s = seg_of(ic, n, h, a, e);
        kv[r] = key[ic];
        mv[r] = med_list[a + ((e - a) >> 1)];
        segs[r] = (i < n && a == (int32_t)i) ? (int32_t)s : -1;
    }
#pragma unroll
    for (int r = 0; r < PI; ++r) {
        const int64_t i = base + (int64_t)r * PT;
        bal[r] = __ballot(i < n && kv[r] < mv[r]);
    }
    TileRank tr;
    tile_rank(bal, wc, tr);
    const uint64_t below_me = (1ull << lane_id()) - 1ull;
#pragma unroll
    for (int r = 0; r < PI; ++r)
        if (segs[r] >= 0)
            segbase_local[segs[r]] = tr.before_round[r] + tr.wave_off[r] + (int32_t)__popcll(bal[r] & below_me);
    if (threadIdx.x == 0) tcount[blockIdx.x] = tr.total;
}

// Stable partition of (R0, R1) by the low flag.  tpre: exclusive prefix of the
// tile counts, or (LOCAL) the raw tile counts, whose prefix every block then
// forms in LDS (ntile <= LOCAL_TILES).
constexpr int LOCAL_TILES = 1024;
template <bool LOCAL>
__global__ void __launch_bounds__(PT) k_part_scatter(int h, const int32_t *__restrict__ R0,
                                                     const int32_t *__restrict__ R1, int keysel, int64_t n, int ntile,
                                                     const int32_t *__restrict__ med_list,
                                                     const int32_t *__restrict__ tpre,
                                                     const int32_t *__restrict__ segbase_local,
                                                     int32_t *__restrict__ O0, int32_t *__restrict__ O1) {
    __shared__ int32_t wc[PI][PT / WAVE];
    __shared__ int32_t tp[LOCAL ? LOCAL_TILES : 1];
    __shared__ int32_t tmp[PT / WAVE];
    if (LOCAL) {
        constexpr int PER = LOCAL_TILES / PT;
        int32_t v[PER], sum = 0;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int k = threadIdx.x * PER + j;
            v[j] = k < ntile ? tpre[k] : 0;
            sum += v[j];
        }
        int32_t total;
        int32_t run = block_excl_scan<PT>(sum, tmp, total);
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            tp[threadIdx.x * PER + j] = run;
            run += v[j];
        }
    }
    const int64_t base = (int64_t)blockIdx.x * PTILE + threadIdx.x;
    uint64_t bal[PI];
    int32_t v0[PI], v1[PI], segs[PI], mv[PI];
    // every load in flight first (positions clamped into the list, so the
    // loads need no branch); positions >= n are flagged low and not written
#pragma unroll
    for (int r = 0; r < PI; ++r) {
        const int64_t i = base + (int64_t)r * PT;
        const int64_t ic = i < n ? i : n - 1;
        int32_t a, e;
        segs[r] = (int32_t)seg_of(ic, n, h, a, e);
        v0[r] = R0[ic];
        v1[r] = R1[ic];
        mv[r] = med_list[a + ((e - a) >> 1)];
    }
#pragma unroll
    for (int r = 0; r < PI; ++r) {
        const int64_t i = base + (int64_t)r * PT;
        bal[r] = __ballot(i < n && (keysel ? v1[r] : v0[r]) < mv[r]);
    }
    TileRank tr;
    tile_rank(bal, wc, tr);  // its barrier also publishes tp
    const uint64_t below_me = (1ull << lane_id()) - 1ull;
    const uint64_t me = 1ull << lane_id();
    const int32_t tile_base = LOCAL ? tp[blockIdx.x] : tpre[blockIdx.x];
    int32_t lowbase[PI];
#pragma unroll
    for (int r = 0; r < PI; ++r) {  // the segments' low bases, loads first
        const int64_t i = base + (int64_t)r * PT;
        const int64_t ic = i < n ? i : n - 1;
        int32_t a, e;
        seg_of(ic, n, h, a, e);
        const int32_t tile_a = (int32_t)(a / PTILE);
        lowbase[r] = (LOCAL ? tp[tile_a] : tpre[tile_a]) + segbase_local[segs[r]];
    }
#pragma unroll
    for (int r = 0; r < PI; ++r) {
        const int64_t i = base + (int64_t)r * PT;
        if (i < n) {
            int32_t a, e;
            seg_of(i, n, h, a, e);
            const int32_t k = (e - a) >> 1;
            const int32_t pos = tile_base + tr.before_round[r] + tr.wave_off[r] + (int32_t)__popcll(bal[r] & below_me);
            const int32_t below = pos - lowbase[r];  // low flags of the segment before i
            int64_t dst;
            if (bal[r] & me) dst = (int64_t)a + below;
            else dst = (int64_t)a + k + ((int32_t)(i - a) - below);
            O0[dst] = v0[r];
            O1[dst] = v1[r];
        }
    }
}

// Depths h0 .. 2L-1 of one segment of depth h0 (at most LOC_M points) in one
// workgroup, with the two lists in LDS: per depth the same median split and
// stable partition as above (flags, one block-wide scan, scatter within each
// sub-segment), and the same segment records (split lines kept in LDS, so no
// workgroup reads another's).  Replaces two launches per depth on the fine
// depths.  The final XL lists are written back in place.
constexpr int LOC_T = 1024;
constexpr int LOC_PER = 4;
constexpr int LOC_M = LOC_T * LOC_PER;
constexpr int LOC_SEGS = 256;  // sub-segments tracked per depth (2^(2L - h0) <= LOC_SEGS)

__device__ inline int32_t seg_local(int32_t i, int32_t m, int d, int32_t &a, int32_t &e) {
    int32_t lo = 0, hi = m, s = 0;
    for (int k = 0; k < d; ++k) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        const bool up = i >= mid;
        s = 2 * s + (up ? 1 : 0);
        lo = up ? mid : lo;
        hi = up ? hi : mid;
    }
    a = lo;
    e = hi;
    return s;
}

__global__ void __launch_bounds__(LOC_T) k_part_local(int h0, int L, int64_t n, int32_t *__restrict__ gXLx,
                                                      int32_t *__restrict__ gXLy, const int32_t *__restrict__ gYLx,
                                                      const int32_t *__restrict__ gYLy, int32_t *__restrict__ starts,
                                                      const double *__restrict__ xsorted,
                                                      const double *__restrict__ ysorted,
                                                      const double *__restrict__ split_x_prev,
                                                      Rect *__restrict__ rects) {
    __shared__ int32_t buf[6][LOC_M];
    __shared__ int32_t segpre[LOC_SEGS];
    __shared__ double spl[2][LOC_SEGS];  // split lines of the previous and the current depth
    __shared__ int32_t tmp[LOC_T / 64];
    const int64_t S = blockIdx.x;  // segment of depth h0
    const int t = threadIdx.x;
    // range [A, E) of segment S of depth h0: its bits from the root, first
    // split first
    int32_t A = 0, E = (int32_t)n;
    for (int d = h0 - 1; d >= 0; --d) {
        const int32_t mid = A + ((E - A) >> 1);
        if ((S >> d) & 1) A = mid;
        else E = mid;
    }
    const int32_t m = E - A;
    int32_t *XLx = buf[0], *XLy = buf[1], *YLx = buf[2], *YLy = buf[3], *T0 = buf[4], *T1 = buf[5];
    for (int i = t; i < m; i += LOC_T) {
        XLx[i] = gXLx[A + i];
        XLy[i] = gXLy[A + i];
        YLx[i] = gYLx[A + i];
        YLy[i] = gYLy[A + i];
    }
    __syncthreads();
    int cur = 0;  // spl[cur]: split lines of the previous depth
    for (int h = h0; h < 2 * L; ++h) {
        const int d = h - h0;
        const bool xsplit = (h & 1) == 0;
        const int32_t *med = xsplit ? XLx : YLy;
        int32_t *R0 = xsplit ? YLx : XLx, *R1 = xsplit ? YLy : XLy;
        const int32_t *key = xsplit ? R0 : R1;
        // flags of this thread's positions 4t .. 4t+3 and their prefix
        bool f[LOC_PER];
        int32_t sa[LOC_PER], sk[LOC_PER], ss[LOC_PER], cnt = 0;
#pragma unroll
        for (int r = 0; r < LOC_PER; ++r) {
            const int32_t i = LOC_PER * t + r;
            f[r] = false;
            sa[r] = 0;
            sk[r] = 0;
            ss[r] = 0;
            if (i < m) {
                int32_t a, e;
                ss[r] = seg_local(i, m, d, a, e);
                sa[r] = a;
                sk[r] = (e - a) >> 1;
                f[r] = key[i] < med[a + sk[r]];
                cnt += f[r] ? 1 : 0;
            }
        }
        int32_t total;
        int32_t run = block_excl_scan<LOC_T>(cnt, tmp, total);
        int32_t pre[LOC_PER];
#pragma unroll
        for (int r = 0; r < LOC_PER; ++r) {
            pre[r] = run;
            run += f[r] ? 1 : 0;
            const int32_t i = LOC_PER * t + r;
            if (i < m && i == sa[r]) segpre[ss[r]] = pre[r];
        }
        // segment records of this depth (one thread per sub-segment)
        const int64_t nseg = int64_t(1) << h;
        const int32_t nsub = 1 << d;
        int32_t *st1 = starts + depth_offset(h + 1);
        if (t < nsub) {
            // range of sub-segment t: its bits from the segment's root
            int32_t a = 0, e = m;
            for (int q = d - 1; q >= 0; --q) {
                const int32_t mid = a + ((e - a) >> 1);
                if ((t >> q) & 1) a = mid;
                else e = mid;
            }
            const int32_t k = (e - a) >> 1;
            const double *coord = xsplit ? xsorted : ysorted;
            const double sp = 0.5 * (coord[med[a + k - 1]] + coord[med[a + k]]);
            spl[cur ^ 1][t] = sp;
            const int64_t g = (S << d) + t;
            st1[2 * g] = A + a;
            st1[2 * g + 1] = A + a + k;
            if (g == nseg - 1) st1[2 * nseg] = (int32_t)n;
            if (h & 1) {
                const int l = (h - 1) >> 1;
                const int64_t b = g >> 1;
                const int xside = (int)(g & 1);
                const Rect Rb = rects[level_offset(l) + b];
                const double sx = d >= 1 ? spl[cur][t >> 1] : split_x_prev[b];
                const double xlo = xside ? sx : Rb.xlo;
                const double xhi = xside ? Rb.xhi : sx;
                const int64_t c0 = level_offset(l + 1) + 4 * b + 2 * xside;
                rects[c0] = Rect{xlo, xhi, Rb.ylo, sp};
                rects[c0 + 1] = Rect{xlo, xhi, sp, Rb.yhi};
            }
        }
        __syncthreads();  // segpre, spl and the rectangles of this depth
        // stable partition of (R0, R1) within each sub-segment
#pragma unroll
        for (int r = 0; r < LOC_PER; ++r) {
            const int32_t i = LOC_PER * t + r;
            if (i < m) {
                const int32_t below = pre[r] - segpre[ss[r]];
                const int32_t dst = f[r] ? sa[r] + below : sa[r] + sk[r] + ((i - sa[r]) - below);
                T0[dst] = R0[i];
                T1[dst] = R1[i];
            }
        }
        __syncthreads();
        if (xsplit) {
            YLx = T0; YLy = T1; T0 = R0; T1 = R1;
        } else {
            XLx = T0; XLy = T1; T0 = R0; T1 = R1;
        }
        cur ^= 1;
    }
    for (int i = t; i < m; i += LOC_T) {
        gXLx[A + i] = XLx[i];
        gXLy[A + i] = XLy[i];
    }
}

// Centre and radius (half diagonal) of every box, each expression one
// correctly rounded binary64 operation, no contraction.
__global__ void k_geometry(const Rect *__restrict__ rects, int64_t nbox, double4 *__restrict__ geom) {
#pragma clang fp contract(off)
    int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbox) return;
    const Rect R = rects[b];
    const double cx = 0.5 * (R.xlo + R.xhi);
    const double cy = 0.5 * (R.ylo + R.yhi);
    const double w = R.xhi - R.xlo;
    const double h = R.yhi - R.ylo;
    const double w2 = w * w;
    const double h2 = h * h;
    const double r = 0.5 * sqrt(w2 + h2);
    geom[b] = make_double4(cx, cy, r, r > 0.0 ? r : 1.0);
}

__global__ void k_gather(const int32_t *__restrict__ XLx, const int32_t *__restrict__ XLy,
                         const int32_t *__restrict__ xorder, const double *__restrict__ xs,
                         const double *__restrict__ ys, int L, int64_t n, const double4 *__restrict__ geomL, int32_t *__restrict__ perm, double *__restrict__ px,
                         double *__restrict__ py, float2 *__restrict__ loc, int32_t *__restrict__ leafid) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t xr = XLx[i], yr = XLy[i];
    perm[i] = xorder[xr];
    const double x = xs[xr], y = ys[yr];
    px[i] = x;
    py[i] = y;
    int32_t a, e;
    const int64_t leaf = seg_of(i, n, 2 * L, a, e);
    leafid[i] = (int32_t)leaf;
    const double4 g = geomL[leaf];
    loc[i] = make_float2((float)(x - g.x), (float)(y - g.y));
}

// Balls drawn around the points (tree option FMM2D_TREE_SHRINK): the
// bounding box of each leaf's points, then of each box's four children
// level by level upwards (min / max: exact), and each leaf point's FP32
// offset from its leaf's new centre.
__global__ void k_leaf_bbox(const int32_t *__restrict__ stL, const double *__restrict__ px,
                            const double *__restrict__ py, int64_t nleaf, Rect *__restrict__ prL) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nleaf) return;
    const int32_t a = stL[b], e = stL[b + 1];  // every leaf holds a point
    Rect r{px[a], px[a], py[a], py[a]};
    for (int32_t i = a + 1; i < e; ++i) {
        r.xlo = fmin(r.xlo, px[i]);
        r.xhi = fmax(r.xhi, px[i]);
        r.ylo = fmin(r.ylo, py[i]);
        r.yhi = fmax(r.yhi, py[i]);
    }
    prL[b] = r;
}

__global__ void k_merge_bbox(int64_t nb, const Rect *__restrict__ child, Rect *__restrict__ parent) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    Rect r = child[4 * b];
    for (int k = 1; k < 4; ++k) {
        const Rect c = child[4 * b + k];
        r.xlo = fmin(r.xlo, c.xlo);
        r.xhi = fmax(r.xhi, c.xhi);
        r.ylo = fmin(r.ylo, c.ylo);
        r.yhi = fmax(r.yhi, c.yhi);
    }
    parent[b] = r;
}

__global__ void k_leaf_offsets(const double *__restrict__ px, const double *__restrict__ py,
                               const int32_t *__restrict__ leafid, const double4 *__restrict__ geomL, int64_t n,
                               float2 *__restrict__ loc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 g = geomL[leafid[i]];
    loc[i] = make_float2((float)(px[i] - g.x), (float)(py[i] - g.y));
}

}  // namespace

// The tree's arrays of n entries (the sort writes into some of them).
static hipError_t tree_point_buffers(TreeState &t, int64_t n) {
    FMM2D_TRY(t.xsorted.ensure(sizeof(double) * n));
    FMM2D_TRY(t.ysorted.ensure(sizeof(double) * n));
    FMM2D_TRY(t.xorder.ensure(sizeof(int32_t) * n));
    for (DevBuf *b : {&t.XLx, &t.XLy, &t.YLx, &t.YLy, &t.T0, &t.T1, &t.perm, &t.leafid})
        FMM2D_TRY(b->ensure(sizeof(int32_t) * n));
    return hipSuccess;
}

// Step 1 of the build: sort each coordinate by (value, index), with the
// ranks of the points (yorder is kept in YLx until the lists are made).
hipError_t tree_sort(fmm2d_ctx *c, int64_t n) {
    TreeState &t = c->tree;
    FMM2D_TRY(tree_point_buffers(t, n));
    return sort_finish(c, n, t.xsorted.as<double>(), t.ysorted.as<double>(), t.xorder.as<int32_t>(),
                       t.YLx.as<int32_t>(), t.T0.as<int32_t>(), t.T1.as<int32_t>());
}

hipError_t build_tree_device(fmm2d_ctx *c, const double *x, const double *y, bool sorted) {
    TreeState &t = c->tree;
    Scratch &s = c->scr;
    const int64_t n = t.n;
    const int L = t.L;
    const int64_t nbox = level_offset(L + 1);
    const int64_t nleaf = int64_t(1) << (2 * L);
    FMM2D_TRY(tree_point_buffers(t, n));
    FMM2D_TRY(t.starts.ensure(sizeof(int32_t) * (depth_offset(2 * L + 1) + 1)));
    FMM2D_TRY(t.rects.ensure(sizeof(Rect) * nbox));
    FMM2D_TRY(t.geom.ensure(sizeof(double4) * nbox));
    FMM2D_TRY(t.px.ensure(sizeof(double) * n));
    FMM2D_TRY(t.py.ensure(sizeof(double) * n));
    FMM2D_TRY(t.loc.ensure(sizeof(float2) * n));
    const int64_t maxseg = int64_t(1) << (2 * L);
    FMM2D_TRY(s.split0.ensure(sizeof(double) * maxseg));
    FMM2D_TRY(s.split1.ensure(sizeof(double) * maxseg));
    FMM2D_TRY(s.segbase.ensure(sizeof(int32_t) * maxseg));
    const int ntile = (int)((n + PTILE - 1) / PTILE);
    FMM2D_TRY(s.tiles2.ensure(sizeof(int32_t) * (ntile + 1)));

    // 1. sort each coordinate by (value, index); ranks of the points (already
    // queued by the caller when `sorted`)
    int32_t *yorder = t.YLx.as<int32_t>();  // borrowed until the lists are initialised
    int32_t *xrank = t.T0.as<int32_t>(), *yrank = t.T1.as<int32_t>();
    if (!sorted) FMM2D_TRY(tree_sort(c, n));
    // 2. the two rank lists
    // YLx is overwritten last: read yorder (== YLx storage) before writing it.
    // k_init_lists reads yorder[r] and writes YLx[r] for the same r only.
    hipLaunchKernelGGL(k_init_lists, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, t.xorder.as<int32_t>(), yorder,
                       xrank, yrank, n, t.XLx.as<int32_t>(), t.XLy.as<int32_t>(), t.YLx.as<int32_t>(),
                       t.YLy.as<int32_t>());
    int32_t *starts = t.starts.as<int32_t>();
    Rect *rects = t.rects.as<Rect>();
    hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, c->stream, t.xsorted.as<double>(), t.ysorted.as<double>(), n,
                       starts, rects);
    FMM2D_TRY(hipGetLastError());

    // 3. 2L half-levels of median split + stable partition
    int32_t *XLx = t.XLx.as<int32_t>(), *XLy = t.XLy.as<int32_t>();
    int32_t *YLx = t.YLx.as<int32_t>(), *YLy = t.YLy.as<int32_t>();
    int32_t *T0 = t.T0.as<int32_t>(), *T1 = t.T1.as<int32_t>();
    // the fine depths in LDS, from the first depth whose segments (sizes
    // floor or ceil of n / 2^h) fit one workgroup
    int hloc = 0;
    while (hloc < 2 * L && ((n + (int64_t(1) << hloc) - 1) >> hloc) > LOC_M) ++hloc;
    if (2 * L - hloc > 8) hloc = 2 * L - 8;  // at most 2^8 sub-segments per workgroup
    for (int h = 0; h < hloc; ++h) {
        const int64_t nseg = int64_t(1) << h;
        const int32_t *st = starts + depth_offset(h);
        int32_t *st1 = starts + depth_offset(h + 1);
        const bool xsplit = (h & 1) == 0;
        double *split_cur = xsplit ? s.split0.as<double>() : s.split1.as<double>();
        // partition the other list: YL by the x flag, or XL by the y flag
        int32_t *R0 = xsplit ? YLx : XLx;
        int32_t *R1 = xsplit ? YLy : XLy;
        const int keysel = xsplit ? 0 : 1;
        const int32_t *med = xsplit ? XLx : YLy;
        const int nrec_blocks = (int)grid_for(nseg, PT);
        hipLaunchKernelGGL(k_part_count, dim3(ntile + nrec_blocks), dim3(PT), 0, c->stream, h, keysel ? R1 : R0, n,
                           ntile, st, nseg, med, s.tiles2.as<int32_t>(), s.segbase.as<int32_t>(), st1,
                           xsplit ? t.xsorted.as<double>() : t.ysorted.as<double>(), split_cur,
                           s.split0.as<double>(), rects);
        FMM2D_TRY(hipGetLastError());
        if (ntile <= LOCAL_TILES) {
            hipLaunchKernelGGL(k_part_scatter<true>, dim3(ntile), dim3(PT), 0, c->stream, h, R0, R1, keysel, n,
                               ntile, med, s.tiles2.as<int32_t>(), s.segbase.as<int32_t>(), T0, T1);
        } else {
            FMM2D_TRY(scan_exclusive(c, s.tiles2.as<int32_t>(), ntile, s.tiles2.as<int32_t>()));
            hipLaunchKernelGGL(k_part_scatter<false>, dim3(ntile), dim3(PT), 0, c->stream, h, R0, R1, keysel, n,
                               ntile, med, s.tiles2.as<int32_t>(), s.segbase.as<int32_t>(), T0, T1);
        }
        FMM2D_TRY(hipGetLastError());
        if (xsplit) {
            YLx = T0; YLy = T1; T0 = R0; T1 = R1;
        } else {
            XLx = T0; XLy = T1; T0 = R0; T1 = R1;
        }
    }
    if (hloc < 2 * L) {
        hipLaunchKernelGGL(k_part_local, dim3((unsigned)(int64_t(1) << hloc)), dim3(LOC_T), 0, c->stream, hloc, L, n,
                           XLx, XLy, YLx, YLy, starts, t.xsorted.as<double>(), t.ysorted.as<double>(),
                           s.split0.as<double>(), rects);
        FMM2D_TRY(hipGetLastError());
    }

    // 4. geometry of all boxes, leaf-ordered points and local offsets
    hipLaunchKernelGGL(k_geometry, dim3(grid_for(nbox, 256)), dim3(256), 0, c->stream, rects, nbox,
                       t.geom.as<double4>());
    hipLaunchKernelGGL(k_gather, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, XLx, XLy,
                       t.xorder.as<int32_t>(), t.xsorted.as<double>(), t.ysorted.as<double>(),
                       L, n, t.geom.as<double4>() + level_offset(L),
                       t.perm.as<int32_t>(), t.px.as<double>(), t.py.as<double>(), t.loc.as<float2>(),
                       t.leafid.as<int32_t>());
    FMM2D_TRY(hipGetLastError());
    t.shrink = (c->tree_opt & FMM2D_TREE_SHRINK) != 0;
    if (t.shrink) {
        // balls around the points: their bounding boxes, the geometry from
        // those, and the leaf offsets from the new centres
        FMM2D_TRY(t.prect.ensure(sizeof(Rect) * nbox));
        Rect *pr = t.prect.as<Rect>();
        hipLaunchKernelGGL(k_leaf_bbox, dim3(grid_for(nleaf, 256)), dim3(256), 0, c->stream,
                           t.starts.as<int32_t>() + depth_offset(2 * L), t.px.as<double>(), t.py.as<double>(), nleaf,
                           pr + level_offset(L));
        for (int l = L - 1; l >= 0; --l) {
            const int64_t nb = int64_t(1) << (2 * l);
            hipLaunchKernelGGL(k_merge_bbox, dim3(grid_for(nb, 256)), dim3(256), 0, c->stream, nb,
                               pr + level_offset(l + 1), pr + level_offset(l));
        }
        hipLaunchKernelGGL(k_geometry, dim3(grid_for(nbox, 256)), dim3(256), 0, c->stream, pr, nbox,
                           t.geom.as<double4>());
        hipLaunchKernelGGL(k_leaf_offsets, dim3(grid_for(n, 256)), dim3(256), 0, c->stream, t.px.as<double>(),
                           t.py.as<double>(), t.leafid.as<int32_t>(), t.geom.as<double4>() + level_offset(L), n,
                           t.loc.as<float2>());
    }
    return hipGetLastError();
}

}  // namespace fmm2d
