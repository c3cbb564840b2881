/*
 * Test infrastructure: drives every entry point of the C oracle
 * (oracle/fmm2d_oracle.c) once over small inputs, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer (tests/test_oracle_sanitized.py).
 *
 * Inputs: a clustered set with exact duplicates and a point repeated many
 * times (with the median tree and with the uniform quadtree, whose leaves
 * are empty or hold hundreds of points), and a uniform set of exactly 4^L
 * points.  Each is taken through the tree, the geometry, the plain,
 * optimised and relaxed lists of every level, the three FMM evaluations and
 * both direct sums, and the FMM potentials are compared with the direct sum
 * (a loose check: the sanitizers are the point).
 * Prints "ok" and returns 0 when everything ran and agreed.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void orc_direct(int64_t n, const double *x, const double *y, const double *q, int64_t m, const int64_t *targets,
                double *phi);
void orc_direct_field(int64_t n, const double *x, const double *y, const double *q, int64_t m,
                      const int64_t *targets, double *gx, double *gy);
int orc_tree(int64_t n, const double *x, const double *y, int L, int64_t *perm, int64_t *leaf_start, double *rects);
int orc_tree_midpoint(int64_t n, const double *x, const double *y, int L, int64_t *perm, int64_t *leaf_start,
                      double *rects);
void orc_geometry(int64_t nbox, const double *rects, double *geom);
int orc_lists_level(int l, double theta, const double *geom_l, const int64_t *sptr_prev, const int64_t *sidx_prev,
                    int64_t *sptr, int64_t *sidx, int64_t *wptr, int64_t *widx, int64_t cap);
int orc_lists_level_opt(int l, double theta, int parent, int swap, const double *geom_l, const double *geom_prev,
                        const int64_t *sptr_prev, const int64_t *sidx_prev, int64_t *sptr, int64_t *sidx,
                        int64_t *wptr, int64_t *widx, int64_t *vptr, int64_t *vidx, int64_t *xptr, int64_t *xidx,
                        int64_t cap);
int orc_lists_level_relaxed(int l, double theta, double theta_max, int p, int k0, int k1, const double *geom_l,
                            const int64_t *sptr_prev, const int64_t *sidx_prev, int64_t *sptr, int64_t *sidx,
                            int64_t *wptr, int64_t *widx, int64_t cap, int64_t *count, int *kmax);
int orc_fmm_eval(int64_t n, const double *x, const double *y, const double *q, int L, int p, const int64_t *perm,
                 const int64_t *leaf_start, const double *geom, const int64_t *wptr, const int64_t *widx,
                 const int64_t *wptr_off, const int64_t *widx_off, const int64_t *sptr_L, const int64_t *sidx_L,
                 double *phi);
int orc_fmm_eval_opt(int64_t n, const double *x, const double *y, const double *q, int L, int p,
                     const int64_t *perm, const int64_t *leaf_start, const double *geom, const int64_t *wptr,
                     const int64_t *widx, const int64_t *wptr_off, const int64_t *widx_off, const int64_t *sptr_L,
                     const int64_t *sidx_L, const int64_t *vptr, const int64_t *vidx, const int64_t *vptr_off,
                     const int64_t *vidx_off, const int64_t *xptr, const int64_t *xidx, const int64_t *xptr_off,
                     const int64_t *xidx_off, double *phi);
int orc_fmm_eval_field(int64_t n, const double *x, const double *y, const double *q, int L, int p,
                       const int64_t *perm, const int64_t *leaf_start, const double *geom, const int64_t *wptr,
                       const int64_t *widx, const int64_t *wptr_off, const int64_t *widx_off,
                       const int64_t *sptr_L, const int64_t *sidx_L, double *phi, double *gx, double *gy);

#define MAXL 8
#define FAIL(...)                                 \
    do {                                          \
        fprintf(stderr, __VA_ARGS__);             \
        fputc('\n', stderr);                      \
        exit(1);                                  \
    } while (0)

static uint64_t rng_state;
static double urand(void) {  /* splitmix64, top 53 bits */
    uint64_t z = (rng_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    return (double)(z >> 11) * 0x1p-53;
}

static int64_t level_offset(int l) { return ((((int64_t)1) << (2 * l)) - 1) / 3; }

/* Per-level lists concatenated as the evaluations take them: the row
 * pointers of level l start at ptr_off[l], the entries at idx_off[l]. */
typedef struct {
    int64_t *ptr[MAXL + 1], *idx[MAXL + 1], nidx[MAXL + 1];
} LevelLists;

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) FAIL("out of memory");
    return p;
}

static void concat(const LevelLists *ls, int L, int64_t **ptr, int64_t **idx, int64_t *ptr_off, int64_t *idx_off) {
    int64_t np = 0, ni = 0;
    for (int l = 0; l <= L; ++l) {
        ptr_off[l] = np;
        idx_off[l] = ni;
        np += ((int64_t)1 << (2 * l)) + 1;
        ni += ls->nidx[l];
    }
    *ptr = xmalloc(sizeof(int64_t) * (size_t)np);
    *idx = xmalloc(sizeof(int64_t) * (size_t)(ni ? ni : 1));
    (*idx)[0] = 0;
    for (int l = 0; l <= L; ++l) {
        memcpy(*ptr + ptr_off[l], ls->ptr[l], sizeof(int64_t) * (size_t)(((int64_t)1 << (2 * l)) + 1));
        if (ls->nidx[l]) memcpy(*idx + idx_off[l], ls->idx[l], sizeof(int64_t) * (size_t)ls->nidx[l]);
    }
}

static void free_lists(LevelLists *ls, int L) {
    for (int l = 0; l <= L; ++l) {
        free(ls->ptr[l]);
        free(ls->idx[l]);
    }
}

/* Exact-size copies of a level's lists out of the working buffers. */
static void keep(LevelLists *ls, int l, const int64_t *ptr, const int64_t *idx) {
    int64_t nb = (int64_t)1 << (2 * l);
    ls->ptr[l] = xmalloc(sizeof(int64_t) * (size_t)(nb + 1));
    memcpy(ls->ptr[l], ptr, sizeof(int64_t) * (size_t)(nb + 1));
    ls->nidx[l] = ptr[nb];
    ls->idx[l] = xmalloc(sizeof(int64_t) * (size_t)(ptr[nb] ? ptr[nb] : 1));
    if (ptr[nb]) memcpy(ls->idx[l], idx, sizeof(int64_t) * (size_t)ptr[nb]);
}

static void level0(LevelLists *S, LevelLists *Wl) {
    int64_t sp[2] = {0, 1}, si[1] = {0}, wp[2] = {0, 0};
    keep(S, 0, sp, si);
    keep(Wl, 0, wp, si);
}

static double max_rel_diff(const double *a, const double *b, int64_t n) {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        num = fmax(num, fabs(a[i] - b[i]));
        den = fmax(den, fabs(b[i]));
    }
    return num / den;
}

static void run(const char *name, int64_t n, const double *x, const double *y, const double *q, int L,
                int midpoint) {
    const int p = 10;
    const double theta = 0.5;
    const int64_t nbox = level_offset(L + 1), nleaf = (int64_t)1 << (2 * L);
    int64_t *perm = xmalloc(sizeof(int64_t) * (size_t)n);
    int64_t *leaf_start = xmalloc(sizeof(int64_t) * (size_t)(nleaf + 1));
    double *rects = xmalloc(sizeof(double) * 4 * (size_t)nbox);
    double *geom = xmalloc(sizeof(double) * 3 * (size_t)nbox);
    if ((midpoint ? orc_tree_midpoint(n, x, y, L, perm, leaf_start, rects) : orc_tree(n, x, y, L, perm, leaf_start,
                                                                                         rects)) != 0)
        FAIL("%s: tree", name);
    orc_geometry(nbox, rects, geom);

    int64_t *tg = xmalloc(sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) tg[i] = i;
    double *ex = xmalloc(sizeof(double) * (size_t)n), *phi = xmalloc(sizeof(double) * (size_t)n);
    double *gx = xmalloc(sizeof(double) * (size_t)n), *gy = xmalloc(sizeof(double) * (size_t)n);
    double *egx = xmalloc(sizeof(double) * (size_t)n), *egy = xmalloc(sizeof(double) * (size_t)n);
    orc_direct(n, x, y, q, n, tg, ex);
    orc_direct_field(n, x, y, q, n, tg, egx, egy);

    /* plain, optimised (parent interaction, exchanged roles at every level)
     * and relaxed lists, level by level, each from its own strong lists */
    LevelLists S = {0}, Wl = {0}, So = {0}, Wo = {0}, Vo = {0}, Xo = {0}, Sr = {0}, Wr = {0};
    level0(&S, &Wl);
    level0(&So, &Wo);
    level0(&Sr, &Wr);
    {
        int64_t zp[2] = {0, 0}, zi[1] = {0};
        keep(&Vo, 0, zp, zi);
        keep(&Xo, 0, zp, zi);
    }
    for (int l = 1; l <= L; ++l) {
        int64_t nb = (int64_t)1 << (2 * l);
        const double *gl = geom + 3 * level_offset(l), *gp = geom + 3 * level_offset(l - 1);
        int64_t *bp[4], *bi[4];
        for (int k = 0; k < 4; ++k) bp[k] = xmalloc(sizeof(int64_t) * (size_t)(nb + 1));
        int64_t cap = 16 * S.nidx[l - 1];
        for (int k = 0; k < 4; ++k) bi[k] = xmalloc(sizeof(int64_t) * (size_t)(cap ? cap : 1));
        if (orc_lists_level(l, theta, gl, S.ptr[l - 1], S.idx[l - 1], bp[0], bi[0], bp[1], bi[1], cap) != 0)
            FAIL("%s: lists level %d", name, l);
        keep(&S, l, bp[0], bi[0]);
        keep(&Wl, l, bp[1], bi[1]);
        for (int k = 0; k < 4; ++k) free(bi[k]);
        cap = 16 * So.nidx[l - 1];
        for (int k = 0; k < 4; ++k) bi[k] = xmalloc(sizeof(int64_t) * (size_t)(cap ? cap : 1));
        if (orc_lists_level_opt(l, theta, 1, 1, gl, gp, So.ptr[l - 1], So.idx[l - 1], bp[0], bi[0], bp[1], bi[1],
                                bp[2], bi[2], bp[3], bi[3], cap) != 0)
            FAIL("%s: optimised lists level %d", name, l);
        keep(&So, l, bp[0], bi[0]);
        keep(&Wo, l, bp[1], bi[1]);
        keep(&Vo, l, bp[2], bi[2]);
        keep(&Xo, l, bp[3], bi[3]);
        for (int k = 0; k < 4; ++k) free(bi[k]);
        cap = 16 * Sr.nidx[l - 1];
        for (int k = 0; k < 2; ++k) bi[k] = xmalloc(sizeof(int64_t) * (size_t)(cap ? cap : 1));
        int64_t count[32];
        int kmax = -1;
        if (orc_lists_level_relaxed(l, theta, 0.9, p, 16, 16, gl, Sr.ptr[l - 1], Sr.idx[l - 1], bp[0], bi[0],
                                    bp[1], bi[1], cap, count, &kmax) != 0)
            FAIL("%s: relaxed lists level %d", name, l);
        if (kmax < 15 || kmax > 31) FAIL("%s: relaxed admitted bin %d", name, kmax);
        keep(&Sr, l, bp[0], bi[0]);
        keep(&Wr, l, bp[1], bi[1]);
        for (int k = 0; k < 2; ++k) free(bi[k]);
        for (int k = 0; k < 4; ++k) free(bp[k]);
    }

    int64_t *wptr, *widx, wpo[MAXL + 1], wio[MAXL + 1];
    concat(&Wl, L, &wptr, &widx, wpo, wio);
    if (orc_fmm_eval(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wpo, wio, S.ptr[L], S.idx[L], phi) != 0)
        FAIL("%s: fmm_eval", name);
    double e = max_rel_diff(phi, ex, n);
    if (!(e < 1e-3)) FAIL("%s: plain FMM error %g", name, e);
    if (orc_fmm_eval_field(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wpo, wio, S.ptr[L], S.idx[L], phi,
                           gx, gy) != 0)
        FAIL("%s: fmm_eval_field", name);
    e = fmax(max_rel_diff(gx, egx, n), max_rel_diff(gy, egy, n));
    if (!(e < 1e-2)) FAIL("%s: field error %g", name, e);
    free(wptr);
    free(widx);

    int64_t *vptr, *vidx, vpo[MAXL + 1], vio[MAXL + 1], *xptr, *xidx, xpo[MAXL + 1], xio[MAXL + 1];
    concat(&Wo, L, &wptr, &widx, wpo, wio);
    concat(&Vo, L, &vptr, &vidx, vpo, vio);
    concat(&Xo, L, &xptr, &xidx, xpo, xio);
    if (orc_fmm_eval_opt(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wpo, wio, So.ptr[L], So.idx[L], vptr,
                         vidx, vpo, vio, xptr, xidx, xpo, xio, phi) != 0)
        FAIL("%s: fmm_eval_opt", name);
    e = max_rel_diff(phi, ex, n);
    if (!(e < 1e-3)) FAIL("%s: optimised FMM error %g", name, e);
    free(wptr); free(widx); free(vptr); free(vidx); free(xptr); free(xidx);

    concat(&Wr, L, &wptr, &widx, wpo, wio);
    if (orc_fmm_eval(n, x, y, q, L, p, perm, leaf_start, geom, wptr, widx, wpo, wio, Sr.ptr[L], Sr.idx[L], phi) != 0)
        FAIL("%s: fmm_eval on relaxed lists", name);
    e = max_rel_diff(phi, ex, n);
    if (!(e < 1e-3)) FAIL("%s: relaxed FMM error %g", name, e);
    free(wptr);
    free(widx);

    free_lists(&S, L); free_lists(&Wl, L); free_lists(&So, L); free_lists(&Wo, L);
    free_lists(&Vo, L); free_lists(&Xo, L); free_lists(&Sr, L); free_lists(&Wr, L);
    free(perm); free(leaf_start); free(rects); free(geom); free(tg);
    free(ex); free(phi); free(gx); free(gy); free(egx); free(egy);
    printf("%s: n=%lld L=%d done\n", name, (long long)n, L);
}

int main(void) {
    /* clustered: three Gaussian-like clusters of very different widths, 40
     * exact duplicates and one point repeated 25 times */
    const int64_t n1 = 3000;
    double *x = xmalloc(sizeof(double) * (size_t)n1), *y = xmalloc(sizeof(double) * (size_t)n1);
    double *q = xmalloc(sizeof(double) * (size_t)n1);
    rng_state = 12345;
    const double cx[3] = {0.2, 0.7, 0.71}, cy[3] = {0.3, 0.6, 0.62}, sd[3] = {1e-1, 1e-3, 1e-6};
    for (int64_t i = 0; i < n1; ++i) {
        int c = (int)(i % 3);
        double u = urand() + urand() + urand() - 1.5, v = urand() + urand() + urand() - 1.5;
        x[i] = cx[c] + sd[c] * u;
        y[i] = cy[c] + sd[c] * v;
        q[i] = 2.0 * urand() - 1.0;
    }
    for (int64_t i = 0; i < 40; ++i) {
        x[n1 - 1 - i] = x[i];
        y[n1 - 1 - i] = y[i];
    }
    for (int64_t i = 100; i < 125; ++i) {
        x[i] = 0.5;
        y[i] = 0.5;
    }
    run("clustered", n1, x, y, q, 4, 0);
    run("clustered, uniform quadtree", n1, x, y, q, 4, 1);
    free(x); free(y); free(q);

    /* uniform, exactly 4^L points (one leaf size) */
    const int64_t n2 = 1024;
    x = xmalloc(sizeof(double) * (size_t)n2);
    y = xmalloc(sizeof(double) * (size_t)n2);
    q = xmalloc(sizeof(double) * (size_t)n2);
    for (int64_t i = 0; i < n2; ++i) {
        x[i] = urand();
        y[i] = urand();
        q[i] = 2.0 * urand() - 1.0;
    }
    run("uniform", n2, x, y, q, 5, 0);
    free(x); free(y); free(q);
    printf("ok\n");
    return 0;
}
