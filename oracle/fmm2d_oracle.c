/*
 * fmm2d_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU reference for the asymmetric adaptive 2D FMM of
 * Engblom, "On well-separated sets and fast multipole methods".  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this library.  It shares no code, header, table or constant with the GPU
 * library; both sides only see the same seeded inputs.
 *
 * Everything is binary64.  OpenMP is used only over independent outputs
 * (targets, boxes); the arithmetic order of each single output is the plain
 * sequential one written below.  Build with -ffp-contract=off so that no
 * multiply-add is fused: the geometry and theta-test must round exactly as
 * written.
 *
 * Notation follows the paper: the interaction sum (1.1), the theta-criterion
 * (Criterion 2.1), the median-split pyramid and the connectivity rule
 * (Section 4), and the classical complex multipole / local representation
 * that the experiments use (Section 5).
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ------------------------------------------------------------------------ */
/* O1: the interaction sum (1.1) with charges, G = log|x - y|, written as the
 * plain definition.  Pairs with identical coordinates (this includes j == i)
 * contribute nothing.  Neumaier-compensated summation over j.               */
/* ------------------------------------------------------------------------ */
static inline void neumaier_add(double *s, double *c, double t)
{
    double u = *s + t;
    if (fabs(*s) >= fabs(t))
        *c += (*s - u) + t;
    else
        *c += (t - u) + *s;
    *s = u;
}

void orc_direct(int64_t n, const double *x, const double *y, const double *q,
                int64_t m, const int64_t *targets, double *phi)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = targets[t];
        double s = 0.0, c = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (x[j] == x[i] && y[j] == y[i])
                continue;
            neumaier_add(&s, &c, q[j] * log(hypot(x[i] - x[j], y[i] - y[j])));
        }
        phi[t] = s + c;
    }
}

/* The gradient of the interaction sum (1.1) at each target, written as the
 * plain definition: d/dx and d/dy of q_j log|x - x_j| are q_j (x - x_j)/r^2
 * and q_j (y - y_j)/r^2 with r = |x - x_j|; coincident pairs contribute
 * nothing.  Neumaier-compensated sums over j.                               */
void orc_direct_field(int64_t n, const double *x, const double *y, const double *q,
                      int64_t m, const int64_t *targets, double *gx, double *gy)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < m; ++t) {
        int64_t i = targets[t];
        double sx = 0.0, cx = 0.0, sy = 0.0, cy = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (x[j] == x[i] && y[j] == y[i])
                continue;
            double dx = x[i] - x[j], dy = y[i] - y[j];
            double r2 = dx * dx + dy * dy;
            neumaier_add(&sx, &cx, q[j] * dx / r2);
            neumaier_add(&sy, &cy, q[j] * dy / r2);
        }
        gx[t] = sx + cx;
        gy[t] = sy + cy;
    }
}

/* ------------------------------------------------------------------------ */
/* O2: the balanced pyramid of median splits (Section 4, Fig. 1.1).
 *
 * A box with n members is split along x: members are ordered by the pair
 * (x_j, j) and the first floor(n/2) form the low side.  Each side is then
 * split along y the same way with the key (y_j, j).  Children of box b are
 * 4b + 2*[high x] + [high y].  The split line is the midpoint of the two
 * straddling order statistics.  Inside a leaf, points are listed by (x_j, j).
 *
 * Outputs: perm[n] (original indices in leaf order), start[4^L + 1] (leaf
 * offsets into perm), rects[nbox_total][4] = (xlo, xhi, ylo, yhi) for every
 * box of every level, level l starting at box (4^l - 1)/3.                 */
/* ------------------------------------------------------------------------ */
static const double *g_key;
static int cmp_key_then_index(const void *a, const void *b)
{
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    if (g_key[i] < g_key[j]) return -1;
    if (g_key[i] > g_key[j]) return 1;
    return (i < j) ? -1 : (i > j);
}

static void sort_by(int64_t *idx, int64_t n, const double *key)
{
    g_key = key; /* the tree build is sequential: a file-scope key is fine */
    qsort(idx, (size_t)n, sizeof(int64_t), cmp_key_then_index);
}

static int64_t level_offset(int l) { return ((((int64_t)1) << (2 * l)) - 1) / 3; }

int orc_tree(int64_t n, const double *x_in, const double *y_in, int L,
             int64_t *perm, int64_t *leaf_start, double *rects)
{
    if (L < 0 || L > 13 || n < (((int64_t)1) << (2 * L)))
        return -1;
    int64_t nleaf = ((int64_t)1) << (2 * L);
    int64_t *start = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nleaf + 1));
    int64_t *nstart = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nleaf + 1));
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    if (!start || !nstart || !x || !y) { free(start); free(nstart); free(x); free(y); return -2; }
    /* A coordinate -0 is the number 0: read it as +0, so that a split line or
     * box edge never depends on which of two equal zeros was met first. */
    for (int64_t i = 0; i < n; ++i) { x[i] = x_in[i] + 0.0; y[i] = y_in[i] + 0.0; }

    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    double xmin = x[0], xmax = x[0], ymin = y[0], ymax = y[0];
    for (int64_t i = 1; i < n; ++i) {
        if (x[i] < xmin) xmin = x[i];
        if (x[i] > xmax) xmax = x[i];
        if (y[i] < ymin) ymin = y[i];
        if (y[i] > ymax) ymax = y[i];
    }
    rects[0] = xmin; rects[1] = xmax; rects[2] = ymin; rects[3] = ymax;
    start[0] = 0; start[1] = n;

    for (int l = 0; l < L; ++l) {
        int64_t nb = ((int64_t)1) << (2 * l);
        for (int64_t b = 0; b < nb; ++b) {
            int64_t a = start[b], e = start[b + 1], nn = e - a;
            const double *R = rects + 4 * (level_offset(l) + b);
            /* x split */
            sort_by(perm + a, nn, x);
            int64_t kx = nn / 2;
            double sx = 0.5 * (x[perm[a + kx - 1]] + x[perm[a + kx]]);
            /* y split of each side */
            int64_t side_a[2] = {a, a + kx}, side_n[2] = {kx, nn - kx};
            for (int s = 0; s < 2; ++s) {
                int64_t sa = side_a[s], sn = side_n[s];
                sort_by(perm + sa, sn, y);
                int64_t ky = sn / 2;
                double sy = 0.5 * (y[perm[sa + ky - 1]] + y[perm[sa + ky]]);
                double xlo = s ? sx : R[0], xhi = s ? R[1] : sx;
                int64_t c0 = 4 * b + 2 * s;
                double *C0 = rects + 4 * (level_offset(l + 1) + c0);
                double *C1 = C0 + 4;
                C0[0] = xlo; C0[1] = xhi; C0[2] = R[2]; C0[3] = sy;
                C1[0] = xlo; C1[1] = xhi; C1[2] = sy;   C1[3] = R[3];
                nstart[c0] = sa;
                nstart[c0 + 1] = sa + ky;
            }
        }
        nstart[4 * nb] = n;
        int64_t *tmp = start; start = nstart; nstart = tmp;
    }
    for (int64_t b = 0; b < nleaf; ++b)
        sort_by(perm + start[b], start[b + 1] - start[b], x);
    memcpy(leaf_start, start, sizeof(int64_t) * (size_t)(nleaf + 1));
    free(start); free(nstart); free(x); free(y);
    return 0;
}

/* The uniform quadtree that Section 5's second experiment compares against
 * (the standard, non-adaptive subdivision): the same root box, every box
 * split at the midpoint of its rectangle in both coordinates at once, all
 * leaves at depth L, so boxes of one level are congruent and may hold any
 * number of points, none included.  Child numbering as in orc_tree
 * (4b + 2 [x high] + [y high]); a point on a split line goes to the high
 * side.  Inside a leaf points are listed by (x, index).  Any n >= 1.
 * Returns 0, -1 for bad arguments, -2 when out of memory.                  */
int orc_tree_midpoint(int64_t n, const double *x_in, const double *y_in, int L,
                      int64_t *perm, int64_t *leaf_start, double *rects)
{
    if (L < 0 || L > 13 || n < 1)
        return -1;
    int64_t nleaf = ((int64_t)1) << (2 * L);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *y = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *leaf = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *fill = (int64_t *)calloc((size_t)(nleaf + 1), sizeof(int64_t));
    if (!x || !y || !leaf || !fill) { free(x); free(y); free(leaf); free(fill); return -2; }
    for (int64_t i = 0; i < n; ++i) { x[i] = x_in[i] + 0.0; y[i] = y_in[i] + 0.0; }
    double xmin = x[0], xmax = x[0], ymin = y[0], ymax = y[0];
    for (int64_t i = 1; i < n; ++i) {
        if (x[i] < xmin) xmin = x[i];
        if (x[i] > xmax) xmax = x[i];
        if (y[i] < ymin) ymin = y[i];
        if (y[i] > ymax) ymax = y[i];
    }
    rects[0] = xmin; rects[1] = xmax; rects[2] = ymin; rects[3] = ymax;
    /* rectangles, level by level: the four quarters of the parent's */
    for (int l = 0; l < L; ++l) {
        int64_t nb = ((int64_t)1) << (2 * l);
        for (int64_t b = 0; b < nb; ++b) {
            const double *R = rects + 4 * (level_offset(l) + b);
            double mx = 0.5 * (R[0] + R[1]);
            double my = 0.5 * (R[2] + R[3]);
            for (int c = 0; c < 4; ++c) {
                double *C = rects + 4 * (level_offset(l + 1) + 4 * b + c);
                int hx = c >> 1, hy = c & 1;
                C[0] = hx ? mx : R[0]; C[1] = hx ? R[1] : mx;
                C[2] = hy ? my : R[2]; C[3] = hy ? R[3] : my;
            }
        }
    }
    /* each point's leaf: down the tree, comparing with the split lines */
    for (int64_t i = 0; i < n; ++i) {
        int64_t b = 0;
        for (int l = 0; l < L; ++l) {
            const double *R = rects + 4 * (level_offset(l) + b);
            double mx = 0.5 * (R[0] + R[1]);
            double my = 0.5 * (R[2] + R[3]);
            b = 4 * b + 2 * (x[i] >= mx) + (y[i] >= my);
        }
        leaf[i] = b;
        ++fill[b + 1];
    }
    for (int64_t b = 0; b < nleaf; ++b) fill[b + 1] += fill[b];
    memcpy(leaf_start, fill, sizeof(int64_t) * (size_t)(nleaf + 1));
    for (int64_t i = 0; i < n; ++i) perm[fill[leaf[i]]++] = i;  /* index order inside each leaf */
    for (int64_t b = 0; b < nleaf; ++b)
        sort_by(perm + leaf_start[b], leaf_start[b + 1] - leaf_start[b], x);
    free(x); free(y); free(leaf); free(fill);
    return 0;
}

/* Box centre and radius of the enclosing ball (half diagonal), each line a
 * single rounded binary64 operation (Criterion 2.1 applied to the tiling
 * rectangle).                                                               */
void orc_geometry(int64_t nbox, const double *rects, double *geom)
{
    for (int64_t b = 0; b < nbox; ++b) {
        const double *R = rects + 4 * b;
        double cx = 0.5 * (R[0] + R[1]);
        double cy = 0.5 * (R[2] + R[3]);
        double w = R[1] - R[0];
        double h = R[3] - R[2];
        double w2 = w * w;
        double h2 = h * h;
        double r = 0.5 * sqrt(w2 + h2);
        geom[3 * b + 0] = cx;
        geom[3 * b + 1] = cy;
        geom[3 * b + 2] = r;
    }
}

/* Criterion 2.1: well separated iff R + theta*r <= theta*d.  The criterion
 * is stated for sets inside two disjoint balls; with theta < 1 the inequality
 * forces d >= R + r, with equality only for two zero-size balls at one point,
 * which are not disjoint: such a pair (d = 0) is never well separated.      */
int orc_theta_test(double theta, const double *gb, const double *gc)
{
    double dx = gb[0] - gc[0];
    double dy = gb[1] - gc[1];
    double dx2 = dx * dx;
    double dy2 = dy * dy;
    double d = sqrt(dx2 + dy2);
    double R = gb[2] > gc[2] ? gb[2] : gc[2];
    double r = gb[2] > gc[2] ? gc[2] : gb[2];
    double lhs = R + theta * r;
    double rhs = theta * d;
    return lhs <= rhs && rhs > 0.0;
}

/* ------------------------------------------------------------------------ */
/* O3: connectivity of one level (Section 4).  For box b with parent P, every
 * child c of every box in S(P) joins W(b) if the theta-criterion holds, else
 * S(b).  Candidates are visited in ascending order, so both lists come out
 * ascending.  geom_l holds (cx, cy, r) of the boxes of level l.
 * Returns 0, or -1 if a capacity is exceeded.                              */
/* ------------------------------------------------------------------------ */
int orc_lists_level(int l, double theta, const double *geom_l,
                    const int64_t *sptr_prev, const int64_t *sidx_prev,
                    int64_t *sptr, int64_t *sidx, int64_t *wptr, int64_t *widx,
                    int64_t cap)
{
    int64_t nb = ((int64_t)1) << (2 * l);
    int64_t ns = 0, nw = 0;
    sptr[0] = 0; wptr[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t P = b / 4;
        for (int64_t t = sptr_prev[P]; t < sptr_prev[P + 1]; ++t) {
            int64_t qbox = sidx_prev[t];
            for (int64_t c = 4 * qbox; c < 4 * qbox + 4; ++c) {
                if (orc_theta_test(theta, geom_l + 3 * b, geom_l + 3 * c)) {
                    if (nw >= cap) return -1;
                    widx[nw++] = c;
                } else {
                    if (ns >= cap) return -1;
                    sidx[ns++] = c;
                }
            }
        }
        sptr[b + 1] = ns;
        wptr[b + 1] = nw;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* The structural optimisations of Section 4 (optional).
 *
 * Interaction via the parent: when all four children of a box q in
 * S(parent(b)) pass the theta-criterion against b, and so does q itself,
 * b interacts with q (one conversion from the coarser level) instead of
 * with its four children.  The criterion between b (level l) and q (level
 * l-1) is Criterion 2.1 on their two balls.
 *
 * Exchanged roles: a strongly coupled pair whose criterion holds once the
 * roles of the radii are exchanged, r + theta R <= theta d (R the larger
 * radius), with the two balls disjoint (d > R + r).  Then the sources of the
 * larger box become a local expansion about the smaller (P2L) and the
 * multipole of the smaller is evaluated at the points of the larger (M2P).
 * The paper applies it at the finest level; `swap` enables it at the level
 * being built, and an exchanged pair is not refined further.            */
int orc_swap_test(double theta, const double *gb, const double *gc)
{
    double dx = gb[0] - gc[0];
    double dy = gb[1] - gc[1];
    double dx2 = dx * dx;
    double dy2 = dy * dy;
    double d = sqrt(dx2 + dy2);
    double R = gb[2] > gc[2] ? gb[2] : gc[2];
    double r = gb[2] > gc[2] ? gc[2] : gb[2];
    double lhs = r + theta * R;
    double rhs = theta * d;
    double sum = R + r;
    return lhs <= rhs && d > sum;
}

/* One level of the optimised lists.  For box b with parent P and every q in
 * S(P) (ascending): if `parent` is set, all four children of q are weak for
 * b and the criterion holds between b and q, q joins V(b) (a level l-1 box);
 * otherwise each child c joins W(b) when weak, else X(b) when `swap` is set
 * and the exchanged criterion holds, else S(b).  All four lists come out
 * ascending.  geom_l / geom_prev: (cx, cy, r) of the boxes of levels l and
 * l-1.  Returns 0, or -1 if a capacity is exceeded.                       */
int orc_lists_level_opt(int l, double theta, int parent, int swap, const double *geom_l,
                        const double *geom_prev, const int64_t *sptr_prev, const int64_t *sidx_prev,
                        int64_t *sptr, int64_t *sidx, int64_t *wptr, int64_t *widx,
                        int64_t *vptr, int64_t *vidx, int64_t *xptr, int64_t *xidx, int64_t cap)
{
    int64_t nb = ((int64_t)1) << (2 * l);
    int64_t ns = 0, nw = 0, nv = 0, nx = 0;
    sptr[0] = 0; wptr[0] = 0; vptr[0] = 0; xptr[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t P = b / 4;
        const double *gb = geom_l + 3 * b;
        for (int64_t t = sptr_prev[P]; t < sptr_prev[P + 1]; ++t) {
            int64_t qbox = sidx_prev[t];
            int weak[4], nweak = 0;
            for (int k = 0; k < 4; ++k) {
                weak[k] = orc_theta_test(theta, gb, geom_l + 3 * (4 * qbox + k));
                nweak += weak[k];
            }
            if (parent && nweak == 4 && orc_theta_test(theta, gb, geom_prev + 3 * qbox)) {
                if (nv >= cap) return -1;
                vidx[nv++] = qbox;
                continue;
            }
            for (int k = 0; k < 4; ++k) {
                int64_t c = 4 * qbox + k;
                if (weak[k]) {
                    if (nw >= cap) return -1;
                    widx[nw++] = c;
                } else if (swap && orc_swap_test(theta, gb, geom_l + 3 * c)) {
                    if (nx >= cap) return -1;
                    xidx[nx++] = c;
                } else {
                    if (ns >= cap) return -1;
                    sidx[ns++] = c;
                }
            }
        }
        sptr[b + 1] = ns;
        wptr[b + 1] = nw;
        vptr[b + 1] = nv;
        xptr[b + 1] = nx;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Locally relaxed theta (Section 4, last paragraph): pairs may be admitted
 * as weak with their own theta_i > theta as long as the mean of
 * theta_i^(p+1) over the admitted pairs stays at most theta^(p+1).
 *
 * theta_i of a pair is read on a fixed grid of thresholds
 *     t_k = theta (k + 1) / k0                        k = 0 .. k0 - 1
 *     t_k = theta + (theta_max - theta)(k - k0 + 1) / k1   k = k0 .. k0 + k1 - 1
 * (t_{k0-1} = theta exactly): the bin of a candidate is the least k whose
 * threshold passes Criterion 2.1, and t_bin^(p+1) stands in for theta_i^(p+1)
 * (an upper bound).  Per level: count the candidates of every bin, then take
 * the largest K >= k0 - 1 such that for every k in k0 - 1 .. K
 *     sum_{j <= k} count_j t_j^(p+1)  <=  theta^(p+1) sum_{j <= k} count_j
 * (sums in j order, powers by p repeated products); candidates of bins up to
 * K are weak, the rest strong.  With theta_max = theta this is the plain
 * rule.  Returns 0, or -1 if a capacity is exceeded.                      */
/* ------------------------------------------------------------------------ */
static double relax_threshold(double theta, double theta_max, int k0, int k1, int k)
{
    if (k < k0) return theta * (double)(k + 1) / (double)k0;
    return theta + (theta_max - theta) * (double)(k - k0 + 1) / (double)k1;
}

static double power_p1(double t, int p)
{
    double e = t;
    for (int i = 0; i < p; ++i) e *= t;
    return e;
}

/* Least k with the criterion true at t_k, or nbin when none is. */
static int relax_bin(const double *tk, int nbin, const double *gb, const double *gc)
{
    for (int k = 0; k < nbin; ++k)
        if (orc_theta_test(tk[k], gb, gc)) return k;
    return nbin;
}

int orc_lists_level_relaxed(int l, double theta, double theta_max, int p, int k0, int k1,
                            const double *geom_l, const int64_t *sptr_prev, const int64_t *sidx_prev,
                            int64_t *sptr, int64_t *sidx, int64_t *wptr, int64_t *widx,
                            int64_t cap, int64_t *count, int *kmax)
{
    if (k0 < 1 || k1 < 1 || k0 + k1 > 256) return -2;
    int nbin = k0 + k1;
    double tk[256];
    for (int k = 0; k < nbin; ++k) tk[k] = relax_threshold(theta, theta_max, k0, k1, k);
    int64_t nb = ((int64_t)1) << (2 * l);
    for (int k = 0; k < nbin; ++k) count[k] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t P = b / 4;
        for (int64_t t = sptr_prev[P]; t < sptr_prev[P + 1]; ++t)
            for (int64_t c = 4 * sidx_prev[t]; c < 4 * sidx_prev[t] + 4; ++c) {
                int k = relax_bin(tk, nbin, geom_l + 3 * b, geom_l + 3 * c);
                if (k < nbin) ++count[k];
            }
    }
    double etheta = power_p1(theta, p);
    double sum = 0.0;
    int64_t n = 0;
    int K = k0 - 1;
    for (int k = 0; k < nbin; ++k) {
        sum += (double)count[k] * power_p1(tk[k], p);
        n += count[k];
        if (k < k0 - 1) continue;
        if (k > k0 - 1 && !(sum <= etheta * (double)n)) break;
        K = k;
    }
    *kmax = K;
    int64_t ns = 0, nw = 0;
    sptr[0] = 0; wptr[0] = 0;
    for (int64_t b = 0; b < nb; ++b) {
        int64_t P = b / 4;
        for (int64_t t = sptr_prev[P]; t < sptr_prev[P + 1]; ++t)
            for (int64_t c = 4 * sidx_prev[t]; c < 4 * sidx_prev[t] + 4; ++c) {
                if (relax_bin(tk, nbin, geom_l + 3 * b, geom_l + 3 * c) <= K) {
                    if (nw >= cap) return -1;
                    widx[nw++] = c;
                } else {
                    if (ns >= cap) return -1;
                    sidx[ns++] = c;
                }
            }
        sptr[b + 1] = ns;
        wptr[b + 1] = nw;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* O4: the expansion operators in the classical complex representation
 * (Section 5), with every expansion normalised by its box scale s.
 *
 *   multipole of a box (centre c, scale s):
 *       phi(z) = A_0 log(z - c) + sum_{k=1..p} A_k (s / (z - c))^k
 *   local expansion about a box (centre c, scale s):
 *       psi(z) = sum_{l=0..p} B_l ((z - c) / s)^l
 * The potential is the real part.                                          */
/* ------------------------------------------------------------------------ */
/* Binomial coefficients by Pascal's rule in binary64 (exact below 2^53),
 * filled once when the library is loaded.                                   */
#define ORC_BINOM_N 160
static double g_binom[ORC_BINOM_N][ORC_BINOM_N];
__attribute__((constructor)) static void orc_fill_binom(void)
{
    for (int i = 0; i < ORC_BINOM_N; ++i) {
        g_binom[i][0] = 1.0;
        g_binom[i][i] = 1.0;
        for (int j = 1; j < i; ++j) g_binom[i][j] = g_binom[i - 1][j - 1] + g_binom[i - 1][j];
    }
}
static double binom(int n, int k)
{
    if (k < 0 || k > n) return 0.0;
    return g_binom[n][k];
}

/* P2M: A_0 = sum q_j,  A_k = -(1/k) sum q_j ((z_j - c)/s)^k.               */
void orc_p2m(int64_t n, const double *x, const double *y, const double *q,
             double cx, double cy, double s, int p, double *A /* 2(p+1) */)
{
    cplx acc[64 + 1];
    for (int k = 0; k <= p; ++k) acc[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        cplx zeta = ((x[j] - cx) + I * (y[j] - cy)) / s;
        cplx pw = 1.0;
        acc[0] += q[j];
        for (int k = 1; k <= p; ++k) {
            pw *= zeta;
            acc[k] += -(q[j] / k) * pw;
        }
    }
    for (int k = 0; k <= p; ++k) { A[2 * k] = creal(acc[k]); A[2 * k + 1] = cimag(acc[k]); }
}

/* M2M: child multipole (centre cc, scale sc) re-expanded about the parent
 * (centre cp, scale sp) and added to Ap.  With delta = (cc - cp)/sp and
 * sigma = sc/sp:
 *   A_0(P) += A_0(c)
 *   A_l(P) += -A_0(c) delta^l / l + sum_{k=1..l} A_k(c) sigma^k delta^(l-k) C(l-1, k-1). */
void orc_m2m(const double *Ac, double ccx, double ccy, double sc,
             double cpx, double cpy, double sp, int p, double *Ap)
{
    cplx delta = ((ccx - cpx) + I * (ccy - cpy)) / sp;
    double sigma = sc / sp;
    cplx a[65], out[65], dpow[65];
    double spow[65];
    for (int k = 0; k <= p; ++k) a[k] = Ac[2 * k] + I * Ac[2 * k + 1];
    dpow[0] = 1.0; spow[0] = 1.0;
    for (int k = 1; k <= p; ++k) { dpow[k] = dpow[k - 1] * delta; spow[k] = spow[k - 1] * sigma; }
    out[0] = a[0];
    for (int l = 1; l <= p; ++l) {
        cplx t = -a[0] * dpow[l] / (double)l;
        for (int k = 1; k <= l; ++k)
            t += a[k] * spow[k] * dpow[l - k] * binom(l - 1, k - 1);
        out[l] = t;
    }
    for (int k = 0; k <= p; ++k) { Ap[2 * k] += creal(out[k]); Ap[2 * k + 1] += cimag(out[k]); }
}

/* M2L: source multipole (centre cs, scale ss) converted to a local expansion
 * about the target (centre ct, scale st) and added to Bt.  With
 * z0 = cs - ct, rho_s = ss/z0, rho_t = st/z0, u_0 = A_0, u_k = A_k rho_s^k:
 *   B_0 += A_0 log|z0| + sum_{k>=1} (-1)^k u_k
 *   B_l += rho_t^l ( -A_0 / l + sum_{k>=1} (-1)^k C(l+k-1, k-1) u_k ),  l >= 1.
 * (Only Re B_0 influences the real potential; the constant imaginary part of
 * A_0 log(-z0) is dropped.)                                                */
void orc_m2l(const double *As, double csx, double csy, double ss,
             double ctx, double cty, double st, int p, double *Bt)
{
    cplx z0 = (csx - ctx) + I * (csy - cty);
    cplx rs = ss / z0, rt = st / z0;
    cplx u[65], rtp[65], out[65];
    cplx pw = 1.0;
    u[0] = As[0] + I * As[1];
    for (int k = 1; k <= p; ++k) { pw *= rs; u[k] = (As[2 * k] + I * As[2 * k + 1]) * pw; }
    rtp[0] = 1.0;
    for (int l = 1; l <= p; ++l) rtp[l] = rtp[l - 1] * rt;
    {
        cplx t = u[0] * log(cabs(z0));
        for (int k = 1; k <= p; ++k) t += ((k & 1) ? -1.0 : 1.0) * u[k];
        out[0] = t;
    }
    for (int l = 1; l <= p; ++l) {
        cplx t = -u[0] / (double)l;
        for (int k = 1; k <= p; ++k)
            t += ((k & 1) ? -1.0 : 1.0) * binom(l + k - 1, k - 1) * u[k];
        out[l] = rtp[l] * t;
    }
    for (int k = 0; k <= p; ++k) { Bt[2 * k] += creal(out[k]); Bt[2 * k + 1] += cimag(out[k]); }
}

/* L2L: parent local expansion (centre cp, scale sp) re-centred at the child
 * (centre cc, scale sc), added to Bc.  With delta = (cc - cp)/sp, tau = sc/sp:
 *   B_l(c) += sum_{k=l..p} B_k(P) C(k, l) tau^l delta^(k-l).               */
void orc_l2l(const double *Bp, double cpx, double cpy, double sp,
             double ccx, double ccy, double sc, int p, double *Bc)
{
    cplx delta = ((ccx - cpx) + I * (ccy - cpy)) / sp;
    double tau = sc / sp;
    cplx b[65], dpow[65];
    double tpow[65];
    for (int k = 0; k <= p; ++k) b[k] = Bp[2 * k] + I * Bp[2 * k + 1];
    dpow[0] = 1.0; tpow[0] = 1.0;
    for (int k = 1; k <= p; ++k) { dpow[k] = dpow[k - 1] * delta; tpow[k] = tpow[k - 1] * tau; }
    for (int l = 0; l <= p; ++l) {
        cplx t = 0;
        for (int k = l; k <= p; ++k) t += b[k] * binom(k, l) * dpow[k - l];
        t *= tpow[l];
        Bc[2 * l] += creal(t);
        Bc[2 * l + 1] += cimag(t);
    }
}

/* L2P: Re sum_l B_l ((z - c)/s)^l at each point, by Horner's rule.          */
void orc_l2p(const double *B, double cx, double cy, double s, int p,
             int64_t n, const double *x, const double *y, double *phi)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx zeta = ((x[i] - cx) + I * (y[i] - cy)) / s;
        cplx v = B[2 * p] + I * B[2 * p + 1];
        for (int l = p - 1; l >= 0; --l) v = v * zeta + (B[2 * l] + I * B[2 * l + 1]);
        phi[i] += creal(v);
    }
}

/* The gradient of the local expansion's potential at each point: with
 * F(z) = sum_l B_l ((z - c)/s)^l analytic, d/dx Re F = Re F'(z) and
 * d/dy Re F = -Im F'(z), F'(z) = sum_{l>=1} l B_l ((z - c)/s)^(l-1) / s.     */
void orc_l2p_grad(const double *B, double cx, double cy, double s, int p,
                  int64_t n, const double *x, const double *y, double *gx, double *gy)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx zeta = ((x[i] - cx) + I * (y[i] - cy)) / s;
        cplx d = 0.0;
        for (int l = p; l >= 1; --l) d = d * zeta + (double)l * (B[2 * l] + I * B[2 * l + 1]);
        d /= s;
        gx[i] += creal(d);
        gy[i] -= cimag(d);
    }
}

/* P2L: the local expansion about (c, s) of the potential of sources z_j
 * that lie outside the ball |z - c| < |z_j - c|, added to B:
 *   log(z - z_j) = log(c - z_j) - sum_{l>=1} (1/l) ((z - c)/(z_j - c))^l, so
 *   B_0 += sum q_j log|c - z_j|,  B_l += -(q_j / l) (s / (z_j - c))^l.     */
void orc_p2l(int64_t n, const double *x, const double *y, const double *q,
             double cx, double cy, double s, int p, double *B /* 2(p+1) */)
{
    cplx acc[64 + 1];
    for (int k = 0; k <= p; ++k) acc[k] = 0;
    for (int64_t j = 0; j < n; ++j) {
        cplx w = (x[j] - cx) + I * (y[j] - cy);
        cplx rho = s / w, pw = 1.0;
        acc[0] += q[j] * log(cabs(w));
        for (int k = 1; k <= p; ++k) {
            pw *= rho;
            acc[k] += -(q[j] / k) * pw;
        }
    }
    for (int k = 0; k <= p; ++k) { B[2 * k] += creal(acc[k]); B[2 * k + 1] += cimag(acc[k]); }
}

/* Multipole expansion evaluated at points (used by the operator pins).      */
void orc_m2p(const double *A, double cx, double cy, double s, int p,
             int64_t n, const double *x, const double *y, double *phi)
{
    for (int64_t i = 0; i < n; ++i) {
        cplx w = (x[i] - cx) + I * (y[i] - cy);
        cplx v = (A[0] + I * A[1]) * clog(w);
        cplx rho = s / w, pw = 1.0;
        for (int k = 1; k <= p; ++k) { pw *= rho; v += (A[2 * k] + I * A[2 * k + 1]) * pw; }
        phi[i] += creal(v);
    }
}

/* ------------------------------------------------------------------------ */
/* O4: the whole FMM on a tree and lists built by orc_tree / orc_lists_level
 * (Section 4): upward pass (P2M at the leaves, M2M to the root), M2L along
 * the weak lists of every level >= 1, L2L downwards, and at the finest level
 * L2P plus the direct sum over the strong list.  The scale of a box is its
 * radius r, or 1 for a box of zero size.  Inputs are in original order;
 * phi is returned in original order.
 *
 * geom: (cx, cy, r) of every box of every level (level offsets (4^l-1)/3).
 * wptr/widx: per level l = 0..L, concatenated; wptr_off[l], widx_off[l] give
 * the start of level l in the two arrays.  sptr_L / sidx_L: finest level.  */
/* ------------------------------------------------------------------------ */
static double box_scale(const double *g) { return g[2] > 0.0 ? g[2] : 1.0; }

/* Optional lists of the structural optimisations, per level l = 0..L
 * concatenated like W (NULL when absent): V (interaction via the parent:
 * boxes of level l-1) and X (exchanged roles).                              */
typedef struct {
    const int64_t *vptr, *vidx, *vptr_off, *vidx_off;
    const int64_t *xptr, *xidx, *xptr_off, *xidx_off;
} opt_lists;

/* Points of box b of level l: the leaves b 4^(L-l) .. (b+1) 4^(L-l) - 1.   */
static void box_points(const int64_t *leaf_start, int L, int l, int64_t b, int64_t *a, int64_t *e)
{
    int64_t sh = 2 * (int64_t)(L - l);
    *a = leaf_start[b << sh];
    *e = leaf_start[(b + 1) << sh];
}

static int fmm_eval_impl(int64_t n, const double *x, const double *y, const double *q,
                         int L, int p, const int64_t *perm, const int64_t *leaf_start,
                         const double *geom, const int64_t *wptr, const int64_t *widx,
                         const int64_t *wptr_off, const int64_t *widx_off,
                         const int64_t *sptr_L, const int64_t *sidx_L, double *phi,
                         double *gx, double *gy, const opt_lists *opt)
{
    if (p < 1 || p > 64) return -1;
    if (opt && gx) return -3;  /* the field is not formed with the optimised lists */
    int64_t nbox = level_offset(L + 1);
    int64_t nleaf = ((int64_t)1) << (2 * L);
    int64_t stride = 2 * (p + 1);
    double *A = (double *)calloc((size_t)(nbox * stride), sizeof(double));
    double *B = (double *)calloc((size_t)(nbox * stride), sizeof(double));
    double *xs = (double *)malloc(sizeof(double) * (size_t)n);
    double *ys = (double *)malloc(sizeof(double) * (size_t)n);
    double *qs = (double *)malloc(sizeof(double) * (size_t)n);
    double *ps = (double *)calloc((size_t)n, sizeof(double));
    double *gxs = gx ? (double *)calloc((size_t)n, sizeof(double)) : NULL;
    double *gys = gx ? (double *)calloc((size_t)n, sizeof(double)) : NULL;
    if (!A || !B || !xs || !ys || !qs || !ps || (gx && (!gxs || !gys))) {
        free(A); free(B); free(xs); free(ys); free(qs); free(ps); free(gxs); free(gys);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) { xs[i] = x[perm[i]]; ys[i] = y[perm[i]]; qs[i] = q[perm[i]]; }
    const int64_t off_L = level_offset(L);

    /* P2M at the leaves */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nleaf; ++b) {
        const double *g = geom + 3 * (off_L + b);
        int64_t a = leaf_start[b], e = leaf_start[b + 1];
        orc_p2m(e - a, xs + a, ys + a, qs + a, g[0], g[1], box_scale(g), p,
                A + stride * (off_L + b));
    }
    /* M2M, finest-but-one level up to the root */
    for (int l = L - 1; l >= 0; --l) {
        int64_t nb = ((int64_t)1) << (2 * l), off = level_offset(l), offc = level_offset(l + 1);
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t P = 0; P < nb; ++P) {
            const double *gp = geom + 3 * (off + P);
            for (int c = 0; c < 4; ++c) {
                int64_t cb = offc + 4 * P + c;
                const double *gc = geom + 3 * cb;
                orc_m2m(A + stride * cb, gc[0], gc[1], box_scale(gc),
                        gp[0], gp[1], box_scale(gp), p, A + stride * (off + P));
            }
        }
    }
    /* downward pass: M2L along W at level l, then L2L to level l+1 */
    for (int l = 1; l <= L; ++l) {
        int64_t nb = ((int64_t)1) << (2 * l), off = level_offset(l);
        const int64_t *wp = wptr + wptr_off[l];
        const int64_t *wi = widx + widx_off[l];
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t b = 0; b < nb; ++b) {
            const double *gt = geom + 3 * (off + b);
            for (int64_t t = wp[b]; t < wp[b + 1]; ++t) {
                int64_t c = wi[t];
                const double *gs = geom + 3 * (off + c);
                orc_m2l(A + stride * (off + c), gs[0], gs[1], box_scale(gs),
                        gt[0], gt[1], box_scale(gt), p, B + stride * (off + b));
            }
        }
        if (opt && opt->vptr) {
            /* interaction via the parent: multipoles of level l-1 boxes */
            const int64_t *vp = opt->vptr + opt->vptr_off[l];
            const int64_t *vi = opt->vidx + opt->vidx_off[l];
            int64_t offp = level_offset(l - 1);
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t b = 0; b < nb; ++b) {
                const double *gt = geom + 3 * (off + b);
                for (int64_t t = vp[b]; t < vp[b + 1]; ++t) {
                    int64_t qb = vi[t];
                    const double *gs = geom + 3 * (offp + qb);
                    orc_m2l(A + stride * (offp + qb), gs[0], gs[1], box_scale(gs),
                            gt[0], gt[1], box_scale(gt), p, B + stride * (off + b));
                }
            }
        }
        if (opt && opt->xptr) {
            /* exchanged roles, target the smaller box: the sources of the
             * larger box as a local expansion about the target (P2L) */
            const int64_t *xp = opt->xptr + opt->xptr_off[l];
            const int64_t *xi = opt->xidx + opt->xidx_off[l];
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t b = 0; b < nb; ++b) {
                const double *gt = geom + 3 * (off + b);
                for (int64_t t = xp[b]; t < xp[b + 1]; ++t) {
                    int64_t c = xi[t];
                    const double *gs = geom + 3 * (off + c);
                    if (!(gt[2] < gs[2])) continue;
                    int64_t a, e;
                    box_points(leaf_start, L, l, c, &a, &e);
                    orc_p2l(e - a, xs + a, ys + a, qs + a, gt[0], gt[1], box_scale(gt), p,
                            B + stride * (off + b));
                }
            }
        }
        if (l < L) {
            int64_t offc = level_offset(l + 1);
#pragma omp parallel for schedule(dynamic, 64)
            for (int64_t P = 0; P < nb; ++P) {
                const double *gp = geom + 3 * (off + P);
                for (int c = 0; c < 4; ++c) {
                    int64_t cb = offc + 4 * P + c;
                    const double *gc = geom + 3 * cb;
                    orc_l2l(B + stride * (off + P), gp[0], gp[1], box_scale(gp),
                            gc[0], gc[1], box_scale(gc), p, B + stride * cb);
                }
            }
        }
    }
    /* L2P and the direct sum over the finest-level strong list */
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t b = 0; b < nleaf; ++b) {
        const double *g = geom + 3 * (off_L + b);
        int64_t a = leaf_start[b], e = leaf_start[b + 1];
        orc_l2p(B + stride * (off_L + b), g[0], g[1], box_scale(g), p, e - a,
                xs + a, ys + a, ps + a);
        if (gx)
            orc_l2p_grad(B + stride * (off_L + b), g[0], g[1], box_scale(g), p, e - a,
                         xs + a, ys + a, gxs + a, gys + a);
        for (int64_t i = a; i < e; ++i) {
            double s = 0.0, c = 0.0, sx = 0.0, cx = 0.0, sy = 0.0, cy = 0.0;
            for (int64_t t = sptr_L[b]; t < sptr_L[b + 1]; ++t) {
                int64_t cb = sidx_L[t];
                for (int64_t j = leaf_start[cb]; j < leaf_start[cb + 1]; ++j) {
                    if (xs[j] == xs[i] && ys[j] == ys[i])
                        continue;
                    neumaier_add(&s, &c, qs[j] * log(hypot(xs[i] - xs[j], ys[i] - ys[j])));
                    if (gx) {
                        double dx = xs[i] - xs[j], dy = ys[i] - ys[j];
                        double r2 = dx * dx + dy * dy;
                        neumaier_add(&sx, &cx, qs[j] * dx / r2);
                        neumaier_add(&sy, &cy, qs[j] * dy / r2);
                    }
                }
            }
            ps[i] += s + c;
            if (gx) {
                gxs[i] += sx + cx;
                gys[i] += sy + cy;
            }
        }
    }
    if (opt && opt->xptr) {
        /* exchanged roles, target the larger box: the smaller box's
         * multipole evaluated at every point of the target (M2P) */
        for (int l = 1; l <= L; ++l) {
            int64_t nb = ((int64_t)1) << (2 * l), off = level_offset(l);
            const int64_t *xp = opt->xptr + opt->xptr_off[l];
            const int64_t *xi = opt->xidx + opt->xidx_off[l];
#pragma omp parallel for schedule(dynamic, 16)
            for (int64_t b = 0; b < nb; ++b) {
                const double *gt = geom + 3 * (off + b);
                int64_t a, e;
                box_points(leaf_start, L, l, b, &a, &e);
                for (int64_t t = xp[b]; t < xp[b + 1]; ++t) {
                    int64_t c = xi[t];
                    const double *gs = geom + 3 * (off + c);
                    if (!(gt[2] > gs[2])) continue;
                    orc_m2p(A + stride * (off + c), gs[0], gs[1], box_scale(gs), p, e - a, xs + a, ys + a,
                            ps + a);
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) phi[perm[i]] = ps[i];
    if (gx)
        for (int64_t i = 0; i < n; ++i) { gx[perm[i]] = gxs[i]; gy[perm[i]] = gys[i]; }
    free(A); free(B); free(xs); free(ys); free(qs); free(ps); free(gxs); free(gys);
    return 0;
}

int orc_fmm_eval(int64_t n, const double *x, const double *y, const double *q,
                 int L, int p, const int64_t *perm, const int64_t *leaf_start,
                 const double *geom, const int64_t *wptr, const int64_t *widx,
                 const int64_t *wptr_off, const int64_t *widx_off,
                 const int64_t *sptr_L, const int64_t *sidx_L, double *phi)
{
    return fmm_eval_impl(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wptr_off, widx_off,
                         sptr_L, sidx_L, phi, NULL, NULL, NULL);
}

/* orc_fmm_eval with the lists of the structural optimisations: V (via the
 * parent) and X (exchanged roles), per level, concatenated like W.          */
int orc_fmm_eval_opt(int64_t n, const double *x, const double *y, const double *q,
                     int L, int p, const int64_t *perm, const int64_t *leaf_start,
                     const double *geom, const int64_t *wptr, const int64_t *widx,
                     const int64_t *wptr_off, const int64_t *widx_off,
                     const int64_t *sptr_L, const int64_t *sidx_L,
                     const int64_t *vptr, const int64_t *vidx, const int64_t *vptr_off, const int64_t *vidx_off,
                     const int64_t *xptr, const int64_t *xidx, const int64_t *xptr_off, const int64_t *xidx_off,
                     double *phi)
{
    opt_lists o = {vptr, vidx, vptr_off, vidx_off, xptr, xidx, xptr_off, xidx_off};
    return fmm_eval_impl(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wptr_off, widx_off,
                         sptr_L, sidx_L, phi, NULL, NULL, &o);
}

/* The FMM with the gradient of the potential as well (the field of
 * Section 5's first experiment, here for the logarithmic kernel): at the
 * leaves the derivative of the local expansion plus the direct sum of the
 * gradient over the strong list.                                            */
int orc_fmm_eval_field(int64_t n, const double *x, const double *y, const double *q,
                       int L, int p, const int64_t *perm, const int64_t *leaf_start,
                       const double *geom, const int64_t *wptr, const int64_t *widx,
                       const int64_t *wptr_off, const int64_t *widx_off,
                       const int64_t *sptr_L, const int64_t *sidx_L, double *phi,
                       double *gx, double *gy)
{
    return fmm_eval_impl(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wptr_off, widx_off,
                         sptr_L, sidx_L, phi, gx, gy, NULL);
}
