/*
 * oracle.c -- plain, slow FP64 CPU oracle of the magnification-map hot path.
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  The product path
 * (the HIP library) never links, loads or calls it, and it shares no code,
 * header, table or constant with that path.
 *
 * What it computes, in the paper's order and notation (Weisenbach 2025,
 * "Rootin' Tootin' Efficient Ray Shootin'"):
 *
 *   lens equation (sec. 2.2)         w = (1-k) z + g conj(z) - a_*(z) - a_s(z)
 *   star deflection (sec. 2.2)       a_*(z) = sum_i m_i / (conj(z) - conj(z_i))
 *   compensating sheet (sec. 3.1)    a_s = -k_* z  (|z| <= R_*),  -k_* R_*^2 / conj(z)  outside
 *   rectangular sheet (app. B)       the closed form with four complex logarithms
 *   IRS (sec. 2.3, 4): one ray per grid cell, counted in the pixel it lands in
 *   shooting region (sec. 2.3, app. A)
 *   FMM (sec. 3.3, app. C): tree, P2M, M2M, M2L, P2L, L2L, L2P + near field
 *   IPM (sec. 3.2): each grid cell split into two triangles, each mapped
 *       triangle's image-plane area apportioned to source pixels in proportion
 *       to (mapped triangle n pixel area) / (mapped triangle area).
 *
 * The IPM here computes that area fraction from its definition: for every
 * pixel of the triangle's bounding box, the triangle is clipped against the
 * pixel's four half-planes and the piece's area taken by the shoelace formula.
 *
 * Units: theta_* = 1 (lengths in Einstein radii of a unit mass).
 * Everything is IEEE double; compiled without floating-point contraction.
 */
#include <complex.h>
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

typedef double complex cplx;

static const double ORC_PI = 3.14159265358979323846;

/* ------------------------------------------------------------------------ */
/* threading helper                                                          */
/* ------------------------------------------------------------------------ */

typedef void (*range_fn)(void *ctx, long lo, long hi);
typedef struct { range_fn fn; void *ctx; long lo, hi; } range_job;

static void *range_thread(void *arg)
{
    range_job *j = (range_job *)arg;
    j->fn(j->ctx, j->lo, j->hi);
    return NULL;
}

static int resolve_threads(int nthreads)
{
    if (nthreads > 0) return nthreads;
    long n = sysconf(_SC_NPROCESSORS_ONLN);
    return n > 0 ? (int)n : 1;
}

/* run fn over [0, n) split into contiguous chunks, one per thread */
static void parallel_for(long n, int nthreads, range_fn fn, void *ctx)
{
    nthreads = resolve_threads(nthreads);
    if (nthreads > 256) nthreads = 256;
    if (n < 2 * nthreads || nthreads == 1) { if (n > 0) fn(ctx, 0, n); return; }
    pthread_t th[256];
    range_job jobs[256];
    long chunk = (n + nthreads - 1) / nthreads;
    int used = 0;
    for (int t = 0; t < nthreads; ++t) {
        long lo = t * chunk, hi = lo + chunk;
        if (lo >= n) break;
        if (hi > n) hi = n;
        jobs[t].fn = fn; jobs[t].ctx = ctx; jobs[t].lo = lo; jobs[t].hi = hi;
        if (pthread_create(&th[t], NULL, range_thread, &jobs[t]) != 0) {
            fn(ctx, lo, hi);            /* fall back to running it here */
            jobs[t].fn = NULL;
        }
        used = t + 1;
    }
    for (int t = 0; t < used; ++t)
        if (jobs[t].fn) pthread_join(th[t], NULL);
}

/* ------------------------------------------------------------------------ */
/* star deflection by direct summation (sec. 2.2)                           */
/* ------------------------------------------------------------------------ */

/* Neumaier-compensated running sum */
typedef struct { double s, c; } ksum;
static inline void ksum_add(ksum *k, double v)
{
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}

typedef struct {
    long n; const double *sx, *sy, *sm;
    const double *zx, *zy; double *ax, *ay;
} direct_ctx;

/* a_*(z) = sum_i m_i / conj(z - z_i) = sum_i m_i (z - z_i) / |z - z_i|^2 */
static void direct_range(void *vctx, long lo, long hi)
{
    direct_ctx *c = (direct_ctx *)vctx;
    for (long q = lo; q < hi; ++q) {
        ksum rx = {0, 0}, ry = {0, 0};
        for (long i = 0; i < c->n; ++i) {
            double dx = c->zx[q] - c->sx[i];
            double dy = c->zy[q] - c->sy[i];
            double r2 = dx * dx + dy * dy;
            ksum_add(&rx, c->sm[i] * dx / r2);
            ksum_add(&ry, c->sm[i] * dy / r2);
        }
        c->ax[q] = rx.s + rx.c;
        c->ay[q] = ry.s + ry.c;
    }
}

void orc_alpha_direct(long n, const double *sx, const double *sy, const double *sm,
                      long npts, const double *zx, const double *zy,
                      double *ax, double *ay, int nthreads)
{
    direct_ctx c = {n, sx, sy, sm, zx, zy, ax, ay};
    parallel_for(npts, nthreads, direct_range, &c);
}

/* same sum taken over the stars in reverse order (summation-order check) */
void orc_alpha_direct_reversed(long n, const double *sx, const double *sy, const double *sm,
                               long npts, const double *zx, const double *zy,
                               double *ax, double *ay)
{
    for (long q = 0; q < npts; ++q) {
        ksum rx = {0, 0}, ry = {0, 0};
        for (long i = n - 1; i >= 0; --i) {
            double dx = zx[q] - sx[i], dy = zy[q] - sy[i];
            double r2 = dx * dx + dy * dy;
            ksum_add(&rx, sm[i] * dx / r2);
            ksum_add(&ry, sm[i] * dy / r2);
        }
        ax[q] = rx.s + rx.c;
        ay[q] = ry.s + ry.c;
    }
}

/* ------------------------------------------------------------------------ */
/* macro model + compensating sheet (sec. 2.2, sec. 3.1)                     */
/* ------------------------------------------------------------------------ */

typedef struct {
    double kappa_star, kappa_smooth, gamma;
    int sheet;           /* 0: none; 1: circular sheet of radius e1 = R_*;
                            2: rectangular sheet with corner (e1, e2) = (c1, c2) */
    double e1, e2;
    double psi3[4];      /* third derivatives of the macro potential at the
                            expansion point (app. D): psi_111, psi_112, psi_122, psi_222 */
} orc_lens;

static void lens_set_psi3(orc_lens *L, const double *psi3)
{
    for (int k = 0; k < 4; ++k) L->psi3[k] = psi3 ? psi3[k] : 0.0;
}

/*
 * Deflection of the macro potential's third-order Taylor term (app. D: the
 * potential expanded past second order near a macro critical curve),
 * psi_3(x) = (1/6) sum_ijk psi_ijk x_i x_j x_k, i.e. its gradient
 *   a_3,i = (1/2) sum_jk psi_ijk x_j x_k
 * with the four independent psi_111, psi_112, psi_122, psi_222.
 */
static void macro3_alpha(const orc_lens *L, double x, double y, double *ax, double *ay)
{
    const double a = L->psi3[0], b = L->psi3[1], c = L->psi3[2], d = L->psi3[3];
    *ax = 0.5 * (a * x * x + 2.0 * b * x * y + c * y * y);
    *ay = 0.5 * (b * x * x + 2.0 * c * x * y + d * y * y);
}

/*
 * Deflection of a sheet of convergence -k_* spread over the rectangle
 * [-c1, c1] x [-c2, c2] (app. B), in complex form with c = c1 + i c2 and the
 * principal logarithm:
 *   a_s = (-k_* i / pi) [ (c - zb) log(c - zb) - (cb - zb) log(cb - zb)
 *                         + (-c - zb) log(-c - zb) - (-cb - zb) log(-cb - zb) ]
 *         - k_* (c + cb + z + zb) B_(c1,c2)(z)
 *         - k_* 2 (c + cb) B_(inf,c2)(z) H(Re z - c1)
 * B the boxcar of the rectangle (or of the band |Im z| <= c2), H the step.
 */
static cplx sheet_rect(double ks, double c1, double c2, cplx z)
{
    cplx c = c1 + I * c2, cb = conj(c), zb = conj(z);
    cplx t = (c - zb) * clog(c - zb) - (cb - zb) * clog(cb - zb)
           + (-c - zb) * clog(-c - zb) - (-cb - zb) * clog(-cb - zb);
    cplx a = (-ks * I / ORC_PI) * t;
    double x = creal(z), y = cimag(z);
    int band = (-c2 <= y && y <= c2);
    if (band && -c1 <= x && x <= c1) a -= ks * (c + cb + z + zb);
    if (band && x - c1 >= 0.0) a -= ks * 2.0 * (c + cb);
    return a;
}

/* a_s of the lens's sheet at z */
static void sheet_alpha(const orc_lens *L, double x, double y, double *sx, double *sy)
{
    *sx = *sy = 0.0;
    if (L->sheet == 1) {
        double r2 = x * x + y * y;
        if (r2 <= L->e1 * L->e1) {
            *sx = -L->kappa_star * x;
            *sy = -L->kappa_star * y;
        } else {
            /* -k_* R^2 / conj(z) = -k_* R^2 z / |z|^2 */
            double f = -L->kappa_star * L->e1 * L->e1 / r2;
            *sx = f * x;
            *sy = f * y;
        }
    } else if (L->sheet == 2) {
        cplx a = sheet_rect(L->kappa_star, L->e1, L->e2, x + I * y);
        *sx = creal(a);
        *sy = cimag(a);
    }
}

/* w = (1-kappa) z + gamma conj(z) - a_3(z) - a_*(z) - a_s(z), kappa = kappa_* + kappa_s
   (a_3: the macro potential's third-order term, zero unless psi3 is set) */
static void lens_equation(const orc_lens *L, double x, double y, double ax, double ay,
                          double *wx, double *wy)
{
    double kappa = L->kappa_star + L->kappa_smooth;
    double w1 = (1.0 - kappa) * x + L->gamma * x - ax;
    double w2 = (1.0 - kappa) * y - L->gamma * y - ay;
    double sx, sy, mx, my;
    sheet_alpha(L, x, y, &sx, &sy);
    macro3_alpha(L, x, y, &mx, &my);
    *wx = w1 - mx - sx;
    *wy = w2 - my - sy;
}

void orc_lens_equation(double kappa_star, double kappa_smooth, double gamma, int sheet,
                       double e1, double e2, const double *psi3, long npts, const double *zx, const double *zy,
                       const double *ax, const double *ay, double *wx, double *wy)
{
    orc_lens L = {kappa_star, kappa_smooth, gamma, sheet, e1, e2, {0, 0, 0, 0}};
    lens_set_psi3(&L, psi3);
    for (long q = 0; q < npts; ++q)
        lens_equation(&L, zx[q], zy[q], ax[q], ay[q], &wx[q], &wy[q]);
}

/* the sheet's deflection a_s alone at points z */
void orc_sheet_alpha(double kappa_star, int sheet, double e1, double e2, long npts, const double *zx,
                     const double *zy, double *ax, double *ay)
{
    orc_lens L = {kappa_star, 0.0, 0.0, sheet, e1, e2, {0, 0, 0, 0}};
    for (long q = 0; q < npts; ++q) sheet_alpha(&L, zx[q], zy[q], &ax[q], &ay[q]);
}

/* corner (c1, c2) of the star rectangle of aspect c2 / c1 whose area
   4 c1 c2 = pi sum m / kappa_* realises kappa_* (sec. 2.1, theta_* = 1) */
void orc_star_rect(long n, const double *m, double kappa_star, double aspect, double *c1, double *c2)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += m[i];
    *c1 = *c2 = 0.0;
    if (n == 0 || kappa_star <= 0.0 || aspect <= 0.0) return;
    *c1 = sqrt(ORC_PI * s / (4.0 * kappa_star * aspect));
    *c2 = aspect * *c1;
}

/* R_* from kappa_* = N <m> / R_*^2  (sec. 2.1, theta_* = 1) */
double orc_star_radius(long n, const double *m, double kappa_star)
{
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += m[i];
    if (n == 0 || kappa_star <= 0.0) return 0.0;
    return sqrt(s / kappa_star);
}

/* ------------------------------------------------------------------------ */
/* shooting region and ray grid (sec. 2.3, appendix A)                       */
/* ------------------------------------------------------------------------ */

typedef struct {
    /* inputs */
    double y1c, y2c, hw1, hw2;
    long n1, n2;
    double rays_per_pixel;
    long nray1, nray2;        /* explicit vertex counts (0: from rays_per_pixel) */
    double flux_fraction;     /* f of appendix A */
    double dx1_set, dx2_set;  /* explicit image-plane half-sizes (0: derived) */
    double x1c_set, x2c_set;  /* explicit image-plane centre, used when centre_set */
    long centre_set;
    /* outputs */
    double kappa, lam1, lam2, mu_macro;
    double mean_m, mean_m2, border;
    double X1, X2, dX1, dX2;
    double pix1, pix2;
    long nr1, nr2;
    double d1, d2, x0, y0;
    double L0;                /* FMM root half-length: power of two */
} orc_region;

/*
 * Region (sec. 2.3):  centre X = (Y1 / (1-k+g), Y2 / (1-k-g)),
 * half-size dX_i = (dY_i + r) / |1-k+-g|, with the border r of appendix A:
 * r = theta_* sqrt(k_* <m^2> / (f <m>)).
 * Grid: rays_per_pixel rho gives cells of side pix_i / sqrt(rho) ("rays per
 * pixel in the absence of lensing", sec. 4) and n_r = ceil(2 dX / Delta) + 1
 * vertices centred on X; explicit vertex counts span exactly [-dX, dX].
 * Returns 0 on success, 1 for invalid input, 2 for a degenerate macro model.
 */
int orc_region_setup(orc_region *R, double kappa_star, double kappa_smooth, double gamma,
                     long n, const double *sx, const double *sy, const double *sm, int macro3)
{
    if (!(R->hw1 > 0) || !(R->hw2 > 0) || R->n1 <= 0 || R->n2 <= 0) return 1;
    R->kappa = kappa_star + kappa_smooth;
    R->lam1 = 1.0 - R->kappa + gamma;
    R->lam2 = 1.0 - R->kappa - gamma;
    /* with third-order macro terms (app. D) the images of the map need not sit
       at the linear ones, and a critical line may cross the expansion point:
       the caller gives the shooting region (centre and half-sizes) */
    if (macro3 && !(R->centre_set && R->dx1_set > 0 && R->dx2_set > 0)) return 1;
    if (!macro3 && (fabs(R->lam1) < 1e-9 || fabs(R->lam2) < 1e-9)) return 2;
    R->mu_macro = 1.0 / (R->lam1 * R->lam2);

    double s1 = 0.0, s2 = 0.0;
    for (long i = 0; i < n; ++i) { s1 += sm[i]; s2 += sm[i] * sm[i]; }
    R->mean_m = n ? s1 / n : 0.0;
    R->mean_m2 = n ? s2 / n : 0.0;
    double f = R->flux_fraction > 0 ? R->flux_fraction : 0.01;
    R->border = (n && kappa_star > 0) ? sqrt(kappa_star * R->mean_m2 / (f * R->mean_m)) : 0.0;

    R->X1 = R->centre_set ? R->x1c_set : R->y1c / R->lam1;
    R->X2 = R->centre_set ? R->x2c_set : R->y2c / R->lam2;
    R->dX1 = R->dx1_set > 0 ? R->dx1_set : (R->hw1 + R->border) / fabs(R->lam1);
    R->dX2 = R->dx2_set > 0 ? R->dx2_set : (R->hw2 + R->border) / fabs(R->lam2);
    R->pix1 = 2.0 * R->hw1 / (double)R->n1;
    R->pix2 = 2.0 * R->hw2 / (double)R->n2;

    if (R->nray1 > 1 && R->nray2 > 1) {
        R->nr1 = R->nray1;
        R->nr2 = R->nray2;
        R->d1 = 2.0 * R->dX1 / (double)(R->nr1 - 1);
        R->d2 = 2.0 * R->dX2 / (double)(R->nr2 - 1);
    } else {
        double rho = R->rays_per_pixel > 0 ? R->rays_per_pixel : 1.0;
        R->d1 = R->pix1 / sqrt(rho);
        R->d2 = R->pix2 / sqrt(rho);
        R->nr1 = (long)ceil(2.0 * R->dX1 / R->d1) + 1;
        R->nr2 = (long)ceil(2.0 * R->dX2 / R->d2) + 1;
    }
    R->x0 = R->X1 - 0.5 * (double)(R->nr1 - 1) * R->d1;
    R->y0 = R->X2 - 0.5 * (double)(R->nr2 - 1) * R->d2;

    /* root of the tree: square centred on the origin containing every star and
       every ray; half-length = smallest power of two above the largest |coord| */
    double amax = 0.0;
    for (long i = 0; i < n; ++i) {
        if (fabs(sx[i]) > amax) amax = fabs(sx[i]);
        if (fabs(sy[i]) > amax) amax = fabs(sy[i]);
    }
    double e1 = fabs(R->X1) + 0.5 * (double)(R->nr1 - 1) * R->d1;
    double e2 = fabs(R->X2) + 0.5 * (double)(R->nr2 - 1) * R->d2;
    if (e1 > amax) amax = e1;
    if (e2 > amax) amax = e2;
    int ex;
    frexp(amax > 0 ? amax : 1.0, &ex);
    R->L0 = ldexp(1.0, ex);
    return 0;
}

/* vertex (a, b) of the ray grid */
static inline double grid_x(const orc_region *R, long a) { return R->x0 + (double)a * R->d1; }
static inline double grid_y(const orc_region *R, long b) { return R->y0 + (double)b * R->d2; }

void orc_grid_points(const orc_region *R, long row_lo, long row_hi, double *zx, double *zy)
{
    long k = 0;
    for (long b = row_lo; b < row_hi; ++b)
        for (long a = 0; a < R->nr1; ++a, ++k) {
            zx[k] = grid_x(R, a);
            zy[k] = grid_y(R, b);
        }
}

/* ------------------------------------------------------------------------ */
/* FMM (sec. 3.3, appendix C)                                                */
/* ------------------------------------------------------------------------ */

#define KEY_BITS 24            /* square index bits per axis at the finest level */

typedef struct {
    int level;
    long i, j;                 /* square indices at this level */
    int leaf;
    long s_lo, s_hi;           /* this square's stars (Morton-sorted order) */
    long block;                /* stars in the 3x3 block of same-level squares */
    long parent;
    long child[4];             /* child (2i+qi, 2j+qj) at child[qi + 2 qj] */
} node_t;

typedef struct {
    int p, nmax, lmax, nlevels;
    double L0;
    long n;
    double *x, *y, *m;         /* stars, Morton-sorted */
    uint64_t *key;
    long nnodes;
    node_t *nodes;
    long *level_lo, *level_hi; /* node index range of each level */
    cplx *a;                   /* multipole coefficients, (p+1) per node */
    cplx *c;                   /* local (Taylor) coefficients, (p+1) per node */
    double binom[64][64];
} orc_fmm;

static uint64_t spread_bits(uint64_t v)
{
    uint64_t r = 0;
    for (int b = 0; b < KEY_BITS; ++b) r |= ((v >> b) & 1ull) << (2 * b);
    return r;
}
static uint64_t morton(uint64_t i, uint64_t j) { return spread_bits(i) | (spread_bits(j) << 1); }

/* square index of coordinate t at `level` (root [-L0, L0), power-of-two L0) */
static long cell_index(double t, double L0, int level)
{
    int e;
    frexp(L0, &e);                      /* L0 = 2^(e-1) */
    double u = ldexp(t + L0, level - e); /* (t + L0) * 2^level / (2 L0), exact scaling */
    long k = (long)floor(u);
    long nmax = 1l << level;
    if (k < 0) k = 0;
    if (k >= nmax) k = nmax - 1;
    return k;
}

static double node_half(const orc_fmm *F, int level) { return ldexp(F->L0, -level); }
static double node_cx(const orc_fmm *F, int level, long i)
{
    double L = node_half(F, level);
    return -F->L0 + (double)(2 * i + 1) * L;
}

typedef struct { uint64_t key; long idx; } keyed;
static int keyed_cmp(const void *A, const void *B)
{
    const keyed *a = A, *b = B;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    return a->idx < b->idx ? -1 : (a->idx > b->idx);
}

static long lower_bound_key(const uint64_t *k, long n, uint64_t v)
{
    long lo = 0, hi = n;
    while (lo < hi) { long mid = (lo + hi) / 2; if (k[mid] < v) lo = mid + 1; else hi = mid; }
    return lo;
}

/* star index range of square (level, i, j); empty if outside the root */
static void square_range(const orc_fmm *F, int level, long i, long j, long *lo, long *hi)
{
    long side = 1l << level;
    if (i < 0 || j < 0 || i >= side || j >= side) { *lo = *hi = 0; return; }
    int sh = 2 * (KEY_BITS - level);
    /* the square's stars are the keys sharing its Morton prefix */
    uint64_t a = morton((uint64_t)i << (KEY_BITS - level), (uint64_t)j << (KEY_BITS - level));
    uint64_t b = a + (1ull << sh);
    *lo = lower_bound_key(F->key, F->n, a);
    *hi = lower_bound_key(F->key, F->n, b);
}

static long square_count(const orc_fmm *F, int level, long i, long j)
{
    long lo, hi;
    square_range(F, level, i, j, &lo, &hi);
    return hi - lo;
}

/* node index of square (level, i, j), -1 if it is not a node of the tree */
static long find_node(const orc_fmm *F, int level, long i, long j)
{
    if (level >= F->nlevels) return -1;
    long side = 1l << level;
    if (i < 0 || j < 0 || i >= side || j >= side) return -1;
    uint64_t want = morton((uint64_t)i, (uint64_t)j);
    long lo = F->level_lo[level], hi = F->level_hi[level];
    while (lo < hi) {
        long mid = (lo + hi) / 2;
        uint64_t k = morton((uint64_t)F->nodes[mid].i, (uint64_t)F->nodes[mid].j);
        if (k < want) lo = mid + 1; else hi = mid;
    }
    if (lo < F->level_hi[level] && F->nodes[lo].i == i && F->nodes[lo].j == j) return lo;
    return -1;
}

static long block_count(const orc_fmm *F, int level, long i, long j)
{
    long s = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) s += square_count(F, level, i + di, j + dj);
    return s;
}

/*
 * Tree (appendix C.1): the root square is centred on the origin and holds
 * every star; a node is divided into 4 children when the stars in the node
 * and its neighbours exceed nmax.  Neighbours are the same-level squares that
 * share a side or a corner with the node, so the test counts the stars of the
 * 3x3 block of same-level squares around it.  Division stops at level lmax.
 */
static int build_tree(orc_fmm *F)
{
    long cap = 1024, nn = 0;
    F->nodes = malloc(cap * sizeof(node_t));
    F->level_lo = calloc(KEY_BITS + 2, sizeof(long));
    F->level_hi = calloc(KEY_BITS + 2, sizeof(long));
    if (!F->nodes || !F->level_lo || !F->level_hi) return -1;
    node_t root = {0, 0, 0, 0, 0, F->n, F->n, -1, {-1, -1, -1, -1}};
    F->nodes[nn++] = root;
    F->level_lo[0] = 0; F->level_hi[0] = 1;
    int level = 0;
    for (;;) {
        long lo = F->level_lo[level], hi = F->level_hi[level];
        long nsplit = 0;
        for (long q = lo; q < hi; ++q) {
            node_t *nd = &F->nodes[q];
            square_range(F, level, nd->i, nd->j, &nd->s_lo, &nd->s_hi);
            nd->block = block_count(F, level, nd->i, nd->j);
            nd->leaf = !(nd->block > F->nmax && level < F->lmax);
            if (!nd->leaf) ++nsplit;
        }
        if (nsplit == 0) { F->nlevels = level + 1; break; }
        if (nn + 4 * nsplit > cap) {
            while (nn + 4 * nsplit > cap) cap *= 2;
            node_t *t = realloc(F->nodes, cap * sizeof(node_t));
            if (!t) return -1;
            F->nodes = t;
        }
        F->level_lo[level + 1] = nn;
        for (long q = lo; q < hi; ++q) {
            if (F->nodes[q].leaf) continue;
            /* children in Morton order of their (qi, qj): (0,0) (1,0) (0,1) (1,1) */
            for (int qj = 0; qj < 2; ++qj)
                for (int qi = 0; qi < 2; ++qi) {
                    node_t ch = {level + 1, 2 * F->nodes[q].i + qi, 2 * F->nodes[q].j + qj,
                                 0, 0, 0, 0, q, {-1, -1, -1, -1}};
                    F->nodes[q].child[qi + 2 * qj] = nn;
                    F->nodes[nn++] = ch;
                }
        }
        F->level_hi[level + 1] = nn;
        ++level;
    }
    F->nnodes = nn;
    return 0;
}

/* P2M (appendix C.2): a_0 = sum m_i, a_k = -(1/k) sum m_i z_i^k, with z_i in
   units of the node half-length relative to the node centre */
static void p2m(const orc_fmm *F, long q, cplx *a)
{
    const node_t *nd = &F->nodes[q];
    double L = node_half(F, nd->level);
    cplx cen = node_cx(F, nd->level, nd->i) + I * node_cx(F, nd->level, nd->j);
    for (int k = 0; k <= F->p; ++k) a[k] = 0;
    for (long s = nd->s_lo; s < nd->s_hi; ++s) {
        cplx zi = ((F->x[s] + I * F->y[s]) - cen) / L;
        a[0] += F->m[s];
        cplx pw = 1;
        for (int k = 1; k <= F->p; ++k) {
            pw *= zi;
            a[k] += -F->m[s] * pw / (double)k;
        }
    }
}

/* M2M (appendix C.2): shift a child's expansion to its parent,
   b_l = z0^l [ -a_0/l + sum_{k=1}^{l} a_k z0^-k C(l-1, k-1) ],
   z0 = child centre relative to the parent centre in child half-lengths,
   then b_l / 2^l for the parent's half-length. */
/* zp[k] = z^k, k = 0..n (repeated multiplication) */
static void powers(cplx z, int n, cplx *zp)
{
    zp[0] = 1;
    for (int k = 1; k <= n; ++k) zp[k] = zp[k - 1] * z;
}

static void m2m_add(const orc_fmm *F, const cplx *a, cplx z0, cplx *b)
{
    cplx zp[32], zm[32];
    powers(z0, F->p, zp);
    powers(1.0 / z0, F->p, zm);
    b[0] += a[0];
    for (int l = 1; l <= F->p; ++l) {
        cplx s = -a[0] / (double)l;
        for (int k = 1; k <= l; ++k) s += a[k] * zm[k] * F->binom[l - 1][k - 1];
        b[l] += zp[l] * s / ldexp(1.0, l);
    }
}

/* M2L (appendix C.2), l >= 1:
   c_l = z0^-l [ -b_0/l + sum_{k=1}^{p} b_k (-z0)^-k C(l+k-1, k-1) ],
   z0 = centre of the interaction node relative to the given node, in units of
   their (common) half-length.  c_0 only shifts the potential, not the
   deflection, and is not formed. */
static void m2l_add(const orc_fmm *F, const cplx *b, cplx z0, cplx *c)
{
    cplx nm[32], zm[32];
    powers(-1.0 / z0, F->p, nm);   /* (-z0)^-k */
    powers(1.0 / z0, F->p, zm);    /* z0^-l */
    for (int l = 1; l <= F->p; ++l) {
        cplx s = -b[0] / (double)l;
        for (int k = 1; k <= F->p; ++k) s += b[k] * nm[k] * F->binom[l + k - 1][k - 1];
        c[l] += zm[l] * s;
    }
}

/* P2L (appendix C.2), l >= 1: c_l = sum_i -m_i / (l z_i^l), z_i relative to the
   given node's centre in its half-length units */
static void p2l_add(const orc_fmm *F, long s_lo, long s_hi, cplx cen, double L, cplx *c)
{
    for (long s = s_lo; s < s_hi; ++s) {
        cplx zi = ((F->x[s] + I * F->y[s]) - cen) / L;
        cplx pw = 1;
        for (int l = 1; l <= F->p; ++l) {
            pw *= zi;
            c[l] += -F->m[s] / ((double)l * pw);
        }
    }
}

/* L2L (appendix C.2): d_l = sum_{k=l}^{p} c_k (-z0)^(k-l) C(k, l), then d_l / 2^l.
   The shift is the exact re-expansion when z0 is the parent's centre relative
   to the child's, in parent half-lengths. */
static void l2l_add(const orc_fmm *F, const cplx *c, cplx z0, cplx *d)
{
    cplx np[32];
    powers(-z0, F->p, np);         /* (-z0)^n */
    for (int l = 0; l <= F->p; ++l) {
        cplx s = 0;
        for (int k = l; k <= F->p; ++k) s += c[k] * np[k - l] * F->binom[k][l];
        d[l] += s / ldexp(1.0, l);
    }
}

typedef struct { orc_fmm *F; int level; } level_ctx;

static void upward_range(void *vctx, long lo, long hi)
{
    level_ctx *ctx = vctx;
    orc_fmm *F = ctx->F;
    int P1 = F->p + 1;
    for (long q = F->level_lo[ctx->level] + lo; q < F->level_lo[ctx->level] + hi; ++q) {
        node_t *nd = &F->nodes[q];
        cplx *a = &F->a[q * P1];
        if (nd->leaf) { p2m(F, q, a); continue; }
        for (int k = 0; k <= F->p; ++k) a[k] = 0;
        for (int qj = 0; qj < 2; ++qj)
            for (int qi = 0; qi < 2; ++qi) {
                long ch = nd->child[qi + 2 * qj];
                /* child centre relative to parent, in child half-lengths: +-1 +-i */
                cplx z0 = (double)(2 * qi - 1) + I * (double)(2 * qj - 1);
                m2m_add(F, &F->a[ch * P1], z0, a);
            }
    }
}

static void downward_range(void *vctx, long lo, long hi)
{
    level_ctx *ctx = vctx;
    orc_fmm *F = ctx->F;
    int level = ctx->level, P1 = F->p + 1;
    for (long q = F->level_lo[level] + lo; q < F->level_lo[level] + hi; ++q) {
        node_t *nd = &F->nodes[q];
        cplx *c = &F->c[q * P1];
        for (int k = 0; k <= F->p; ++k) c[k] = 0;
        if (level < 2) continue;    /* every star is a neighbour at levels 0, 1 */
        const node_t *par = &F->nodes[nd->parent];
        /* L2L from the parent: parent centre relative to child, parent units */
        long qi = nd->i - 2 * par->i, qj = nd->j - 2 * par->j;
        cplx z0 = -((double)(2 * qi - 1) + I * (double)(2 * qj - 1)) * 0.5;
        l2l_add(F, &F->c[nd->parent * P1], z0, c);
        /* interaction squares: children of the parent's 3x3 block that are not
           in the node's own 3x3 block (at most 27) */
        double L = node_half(F, level);
        cplx cen = node_cx(F, level, nd->i) + I * node_cx(F, level, nd->j);
        for (long pj = par->j - 1; pj <= par->j + 1; ++pj)
            for (long pi = par->i - 1; pi <= par->i + 1; ++pi)
                for (int cj = 0; cj < 2; ++cj)
                    for (int ci = 0; ci < 2; ++ci) {
                        long si = 2 * pi + ci, sj = 2 * pj + cj;
                        if (labs(si - nd->i) <= 1 && labs(sj - nd->j) <= 1) continue;
                        long side = 1l << level;
                        if (si < 0 || sj < 0 || si >= side || sj >= side) continue;
                        long src = find_node(F, level, si, sj);
                        if (src >= 0) {
                            cplx off = 2.0 * (double)(si - nd->i) + I * 2.0 * (double)(sj - nd->j);
                            m2l_add(F, &F->a[src * P1], off, c);
                        } else {
                            /* the square lies inside a coarser leaf: its stars
                               enter the Taylor series directly */
                            long lo2, hi2;
                            square_range(F, level, si, sj, &lo2, &hi2);
                            p2l_add(F, lo2, hi2, cen, L, c);
                        }
                    }
    }
}

static void binomials(double b[64][64])
{
    memset(b, 0, sizeof(double) * 64 * 64);
    for (int n = 0; n < 64; ++n) {
        b[n][0] = 1.0;
        for (int k = 1; k <= n; ++k) b[n][k] = b[n - 1][k - 1] + (k <= n - 1 ? b[n - 1][k] : 0.0);
    }
}

void orc_fmm_free(void *vF)
{
    orc_fmm *F = vF;
    if (!F) return;
    free(F->x); free(F->y); free(F->m); free(F->key);
    free(F->nodes); free(F->level_lo); free(F->level_hi);
    free(F->a); free(F->c);
    free(F);
}

void *orc_fmm_build(long n, const double *sx, const double *sy, const double *sm,
                    double L0, int p, int nmax, int lmax, int nthreads)
{
    if (p < 1 || p > 31 || nmax < 1 || lmax < 0 || lmax > KEY_BITS) return NULL;
    orc_fmm *F = calloc(1, sizeof(orc_fmm));
    if (!F) return NULL;
    F->p = p; F->nmax = nmax; F->lmax = lmax; F->L0 = L0; F->n = n;
    binomials(F->binom);
    F->x = malloc((n + 1) * sizeof(double));
    F->y = malloc((n + 1) * sizeof(double));
    F->m = malloc((n + 1) * sizeof(double));
    F->key = malloc((n + 1) * sizeof(uint64_t));
    keyed *kk = malloc((n + 1) * sizeof(keyed));
    if (!F->x || !F->y || !F->m || !F->key || !kk) { free(kk); orc_fmm_free(F); return NULL; }
    for (long s = 0; s < n; ++s) {
        long i = cell_index(sx[s], L0, KEY_BITS), j = cell_index(sy[s], L0, KEY_BITS);
        kk[s].key = morton((uint64_t)i, (uint64_t)j);
        kk[s].idx = s;
    }
    qsort(kk, n, sizeof(keyed), keyed_cmp);
    for (long s = 0; s < n; ++s) {
        F->key[s] = kk[s].key;
        F->x[s] = sx[kk[s].idx]; F->y[s] = sy[kk[s].idx]; F->m[s] = sm[kk[s].idx];
    }
    free(kk);
    if (build_tree(F) != 0) { orc_fmm_free(F); return NULL; }
    long P1 = p + 1;
    F->a = calloc(F->nnodes * P1, sizeof(cplx));
    F->c = calloc(F->nnodes * P1, sizeof(cplx));
    if (!F->a || !F->c) { orc_fmm_free(F); return NULL; }
    /* upward pass: leaves by P2M, parents by M2M, deepest level first */
    for (int level = F->nlevels - 1; level >= 0; --level) {
        level_ctx ctx = {F, level};
        parallel_for(F->level_hi[level] - F->level_lo[level], nthreads, upward_range, &ctx);
    }
    /* downward pass: L2L + M2L + P2L, root first */
    for (int level = 0; level < F->nlevels; ++level) {
        level_ctx ctx = {F, level};
        parallel_for(F->level_hi[level] - F->level_lo[level], nthreads, downward_range, &ctx);
    }
    return F;
}

long orc_fmm_num_nodes(const void *vF) { return ((const orc_fmm *)vF)->nnodes; }
int orc_fmm_num_levels(const void *vF) { return ((const orc_fmm *)vF)->nlevels; }

void orc_fmm_nodes(const void *vF, int *level, long *i, long *j, int *leaf, long *nstars, long *block)
{
    const orc_fmm *F = vF;
    for (long q = 0; q < F->nnodes; ++q) {
        level[q] = F->nodes[q].level; i[q] = F->nodes[q].i; j[q] = F->nodes[q].j;
        leaf[q] = F->nodes[q].leaf; nstars[q] = F->nodes[q].s_hi - F->nodes[q].s_lo;
        block[q] = F->nodes[q].block;
    }
}

/* coefficients as interleaved (re, im) doubles, (p+1) per node */
void orc_fmm_coeffs(const void *vF, double *a, double *c)
{
    const orc_fmm *F = vF;
    long tot = F->nnodes * (F->p + 1);
    for (long t = 0; t < tot; ++t) {
        if (a) { a[2 * t] = creal(F->a[t]); a[2 * t + 1] = cimag(F->a[t]); }
        if (c) { c[2 * t] = creal(F->c[t]); c[2 * t + 1] = cimag(F->c[t]); }
    }
}

/* leaf holding point z: the first level whose square around z is a leaf */
static long find_leaf(const orc_fmm *F, double x, double y)
{
    for (int level = 0; level < F->nlevels; ++level) {
        long q = find_node(F, level, cell_index(x, F->L0, level), cell_index(y, F->L0, level));
        if (q < 0) return -1;
        if (F->nodes[q].leaf) return q;
    }
    return -1;
}

typedef struct { const orc_fmm *F; const double *zx, *zy; double *ax, *ay; long *leaf_out; } eval_ctx;

/* a_*(z) = near field by direct sum over the leaf's 3x3 block of squares
   + conj of d/dz of the leaf's Taylor series:  (1/L) sum_{l>=1} l c_l zeta^(l-1) */
static void eval_range(void *vctx, long lo, long hi)
{
    eval_ctx *e = vctx;
    const orc_fmm *F = e->F;
    int P1 = F->p + 1;
    for (long q = lo; q < hi; ++q) {
        double x = e->zx[q], y = e->zy[q];
        long nd = find_leaf(F, x, y);
        if (e->leaf_out) e->leaf_out[q] = nd;
        if (nd < 0) { e->ax[q] = NAN; e->ay[q] = NAN; continue; }
        const node_t *N = &F->nodes[nd];
        double ax = 0.0, ay = 0.0;
        for (long dj = -1; dj <= 1; ++dj)
            for (long di = -1; di <= 1; ++di) {
                long slo, shi;
                square_range(F, N->level, N->i + di, N->j + dj, &slo, &shi);
                for (long s = slo; s < shi; ++s) {
                    double dx = x - F->x[s], dy = y - F->y[s];
                    double r2 = dx * dx + dy * dy;
                    ax += F->m[s] * dx / r2;
                    ay += F->m[s] * dy / r2;
                }
            }
        double L = node_half(F, N->level);
        cplx zeta = ((x + I * y) - (node_cx(F, N->level, N->i) + I * node_cx(F, N->level, N->j))) / L;
        const cplx *c = &F->c[nd * P1];
        cplx d = 0;
        for (int l = F->p; l >= 1; --l) d = d * zeta + (double)l * c[l];
        d /= L;
        e->ax[q] = ax + creal(d);
        e->ay[q] = ay - cimag(d);
    }
}

void orc_fmm_alpha(const void *vF, long npts, const double *zx, const double *zy,
                   double *ax, double *ay, long *leaf_out, int nthreads)
{
    eval_ctx e = {vF, zx, zy, ax, ay, leaf_out};
    parallel_for(npts, nthreads, eval_range, &e);
}

/* Multipole expansion of node q evaluated at points z (far from the node):
   d psi/dz = a_0 / zeta - sum_k k a_k zeta^-(k+1), divided by L.  Used by the
   tests to pin P2M and M2M against the direct sum. */
void orc_fmm_eval_multipole(const void *vF, long q, long npts, const double *zx, const double *zy,
                            double *gx, double *gy)
{
    const orc_fmm *F = vF;
    const node_t *N = &F->nodes[q];
    double L = node_half(F, N->level);
    cplx cen = node_cx(F, N->level, N->i) + I * node_cx(F, N->level, N->j);
    const cplx *a = &F->a[q * (F->p + 1)];
    for (long t = 0; t < npts; ++t) {
        cplx zeta = ((zx[t] + I * zy[t]) - cen) / L;
        cplx g = a[0] / zeta, pw = 1.0 / zeta;
        for (int k = 1; k <= F->p; ++k) { pw /= zeta; g -= (double)k * a[k] * pw; }
        g /= L;
        gx[t] = creal(g); gy[t] = cimag(g);
    }
}

/* Taylor series of node q: (1/L) sum_{l>=1} l c_l zeta^(l-1) at points z */
void orc_fmm_eval_local(const void *vF, long q, long npts, const double *zx, const double *zy,
                        double *gx, double *gy)
{
    const orc_fmm *F = vF;
    const node_t *N = &F->nodes[q];
    double L = node_half(F, N->level);
    cplx cen = node_cx(F, N->level, N->i) + I * node_cx(F, N->level, N->j);
    const cplx *c = &F->c[q * (F->p + 1)];
    for (long t = 0; t < npts; ++t) {
        cplx zeta = ((zx[t] + I * zy[t]) - cen) / L;
        cplx d = 0;
        for (int l = F->p; l >= 1; --l) d = d * zeta + (double)l * c[l];
        d /= L;
        gx[t] = creal(d); gy[t] = cimag(d);
    }
}

/* the stars in the FMM's Morton-sorted order; returns the count */
long orc_fmm_sorted_stars(const void *vF, double *x, double *y, double *m)
{
    const orc_fmm *F = vF;
    for (long s = 0; s < F->n; ++s) { x[s] = F->x[s]; y[s] = F->y[s]; m[s] = F->m[s]; }
    return F->n;
}

/* standalone translation operators for the identity tests (appendix C.2) */
void orc_op_m2m(int p, const double *a_ri, double z0x, double z0y, double *b_ri)
{
    orc_fmm F; memset(&F, 0, sizeof F); F.p = p; binomials(F.binom);
    cplx a[32] = {0}, b[32] = {0};
    for (int k = 0; k <= p; ++k) { a[k] = a_ri[2 * k] + I * a_ri[2 * k + 1]; b[k] = 0; }
    m2m_add(&F, a, z0x + I * z0y, b);
    for (int k = 0; k <= p; ++k) { b_ri[2 * k] = creal(b[k]); b_ri[2 * k + 1] = cimag(b[k]); }
}

void orc_op_m2l(int p, const double *b_ri, double z0x, double z0y, double *c_ri)
{
    orc_fmm F; memset(&F, 0, sizeof F); F.p = p; binomials(F.binom);
    cplx b[32] = {0}, c[32] = {0};
    for (int k = 0; k <= p; ++k) { b[k] = b_ri[2 * k] + I * b_ri[2 * k + 1]; c[k] = 0; }
    m2l_add(&F, b, z0x + I * z0y, c);
    for (int k = 0; k <= p; ++k) { c_ri[2 * k] = creal(c[k]); c_ri[2 * k + 1] = cimag(c[k]); }
}

void orc_op_l2l(int p, const double *c_ri, double z0x, double z0y, double *d_ri)
{
    orc_fmm F; memset(&F, 0, sizeof F); F.p = p; binomials(F.binom);
    cplx c[32] = {0}, d[32] = {0};
    for (int k = 0; k <= p; ++k) { c[k] = c_ri[2 * k] + I * c_ri[2 * k + 1]; d[k] = 0; }
    l2l_add(&F, c, z0x + I * z0y, d);
    for (int k = 0; k <= p; ++k) { d_ri[2 * k] = creal(d[k]); d_ri[2 * k + 1] = cimag(d[k]); }
}

/* ------------------------------------------------------------------------ */
/* IPM: apportion mapped triangles among pixels (sec. 3.2)                   */
/* ------------------------------------------------------------------------ */

typedef struct { double x, y; } pt;

/* keep the part of polygon `in` (n vertices) with s*(coord - c) >= 0, where
   coord is x (axis 0) or y (axis 1); Sutherland-Hodgman step */
static int clip_halfplane(const pt *in, int n, int axis, double c, double s, pt *out)
{
    int m = 0;
    for (int k = 0; k < n; ++k) {
        pt P = in[k], Q = in[(k + 1) % n];
        double dp = s * ((axis ? P.y : P.x) - c);
        double dq = s * ((axis ? Q.y : Q.x) - c);
        if (dp >= 0) out[m++] = P;
        if ((dp >= 0) != (dq >= 0)) {
            double t = dp / (dp - dq);
            pt X = {P.x + t * (Q.x - P.x), P.y + t * (Q.y - P.y)};
            if (axis) X.y = c; else X.x = c;
            out[m++] = X;
        }
    }
    return m;
}

/* shoelace formula, signed */
static double shoelace(const pt *v, int n)
{
    double s = 0.0;
    for (int k = 0; k < n; ++k) {
        pt P = v[k], Q = v[(k + 1) % n];
        s += P.x * Q.y - Q.x * P.y;
    }
    return 0.5 * s;
}

/* signed area of triangle T intersected with pixel [i, i+1] x [j, j+1]
   (coordinates in pixel units) */
double orc_tri_pixel_area(const double *tx, const double *ty, long i, long j)
{
    pt a[8], b[8];
    /* shift the origin to the pixel corner: small coordinates, exact shifts */
    for (int k = 0; k < 3; ++k) { a[k].x = tx[k] - (double)i; a[k].y = ty[k] - (double)j; }
    int n = 3;
    n = clip_halfplane(a, n, 0, 0.0, +1.0, b); if (n < 3) return 0.0;
    n = clip_halfplane(b, n, 0, 1.0, -1.0, a); if (n < 3) return 0.0;
    n = clip_halfplane(a, n, 1, 0.0, +1.0, b); if (n < 3) return 0.0;
    n = clip_halfplane(b, n, 1, 1.0, -1.0, a); if (n < 3) return 0.0;
    return shoelace(a, n);
}

typedef struct {
    double dep_total;   /* sum of deposits into the map (theta^2) */
    double a_out;       /* image area whose source falls outside the map */
    double a_skip;      /* image area of skipped non-finite triangles */
    long n_skip;        /* number of skipped triangles */
    long n_zero;        /* number of zero-area mapped triangles */
} orc_ipm_stats;

/* apportion one mapped triangle with image-plane area AT (pixel coordinates
   u, v; map n1 x n2); deposits in theta^2 units into dep[j*n1+i] */
static void apportion(double AT, const double *u, const double *v, long n1, long n2,
                      double *dep, orc_ipm_stats *st)
{
    for (int k = 0; k < 3; ++k)
        if (!isfinite(u[k]) || !isfinite(v[k])) { st->n_skip++; st->a_skip += AT; return; }
    double S = 0.5 * ((u[1] - u[0]) * (v[2] - v[0]) - (u[2] - u[0]) * (v[1] - v[0]));
    if (S == 0.0) {
        /* no source-plane area: the whole image area goes to the pixel holding
           the centroid */
        st->n_zero++;
        double cu = (u[0] + u[1] + u[2]) / 3.0, cv = (v[0] + v[1] + v[2]) / 3.0;
        long i = (long)floor(cu), j = (long)floor(cv);
        if (i >= 0 && j >= 0 && i < n1 && j < n2) { dep[j * n1 + i] += AT; st->dep_total += AT; }
        else st->a_out += AT;
        return;
    }
    double umin = fmin(u[0], fmin(u[1], u[2])), umax = fmax(u[0], fmax(u[1], u[2]));
    double vmin = fmin(v[0], fmin(v[1], v[2])), vmax = fmax(v[0], fmax(v[1], v[2]));
    long i0 = (long)floor(umin), i1 = (long)floor(umax);
    long j0 = (long)floor(vmin), j1 = (long)floor(vmax);
    if (i0 < 0) i0 = 0;
    if (j0 < 0) j0 = 0;
    if (i1 > n1 - 1) i1 = n1 - 1;
    if (j1 > n2 - 1) j1 = n2 - 1;
    double inside = 0.0;
    for (long j = j0; j <= j1; ++j)
        for (long i = i0; i <= i1; ++i) {
            double a = orc_tri_pixel_area(u, v, i, j);
            if (a == 0.0) continue;
            double d = AT * (a / S);
            dep[j * n1 + i] += d;
            inside += d;
        }
    st->dep_total += inside;
    st->a_out += AT - inside;
}

/*
 * IPM over cell rows [row_lo, row_hi) of the grid (sec. 3.2).  The vertex
 * positions w of vertex rows row_lo .. row_hi (inclusive) are given, nr1 per
 * row, as source-plane coordinates.  Cell (a, b) with corners
 * v00 = (a, b), v10 = (a+1, b), v11 = (a+1, b+1), v01 = (a, b+1) splits along
 * v00-v11 into T1 = (v00, v10, v11) and T2 = (v00, v11, v01); each has image
 * area D1 D2 / 2.  Deposits accumulate into dep (n2 x n1, row-major, theta^2).
 */
void orc_ipm_rows(const orc_region *R, long row_lo, long row_hi, const double *wx,
                  const double *wy, double *dep, double *stats_out)
{
    orc_ipm_stats st = {0, 0, 0, 0, 0};
    double ylo1 = R->y1c - R->hw1, ylo2 = R->y2c - R->hw2;
    double AT = 0.5 * R->d1 * R->d2;
    long nr1 = R->nr1;
    for (long b = row_lo; b < row_hi; ++b) {
        const double *rx0 = wx + (b - row_lo) * nr1, *ry0 = wy + (b - row_lo) * nr1;
        const double *rx1 = rx0 + nr1, *ry1 = ry0 + nr1;
        for (long a = 0; a + 1 < nr1; ++a) {
            double u00 = (rx0[a] - ylo1) / R->pix1, v00 = (ry0[a] - ylo2) / R->pix2;
            double u10 = (rx0[a + 1] - ylo1) / R->pix1, v10 = (ry0[a + 1] - ylo2) / R->pix2;
            double u11 = (rx1[a + 1] - ylo1) / R->pix1, v11 = (ry1[a + 1] - ylo2) / R->pix2;
            double u01 = (rx1[a] - ylo1) / R->pix1, v01 = (ry1[a] - ylo2) / R->pix2;
            double t1u[3] = {u00, u10, u11}, t1v[3] = {v00, v10, v11};
            double t2u[3] = {u00, u11, u01}, t2v[3] = {v00, v11, v01};
            apportion(AT, t1u, t1v, R->n1, R->n2, dep, &st);
            apportion(AT, t2u, t2v, R->n1, R->n2, dep, &st);
        }
    }
    stats_out[0] += st.dep_total;
    stats_out[1] += st.a_out;
    stats_out[2] += st.a_skip;
    stats_out[3] += (double)st.n_skip;
    stats_out[4] += (double)st.n_zero;
}

/* magnification of each pixel: deposited image area / pixel area (sec. 3.2) */
void orc_normalise(const orc_region *R, const double *dep, double *mu)
{
    double Apix = R->pix1 * R->pix2;
    for (long k = 0; k < R->n1 * R->n2; ++k) mu[k] = dep[k] / Apix;
}

/* ------------------------------------------------------------------------ */
/* whole map                                                                  */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_region *R; const orc_lens *L;
    long n; const double *sx, *sy, *sm;
    const void *F;                 /* FMM or NULL for direct summation */
    long row_lo; double *wx, *wy;
} shoot_ctx;

static void shoot_rows(void *vctx, long lo, long hi)
{
    shoot_ctx *c = vctx;
    long nr1 = c->R->nr1;
    double *zx = malloc(nr1 * sizeof(double)), *zy = malloc(nr1 * sizeof(double));
    double *ax = malloc(nr1 * sizeof(double)), *ay = malloc(nr1 * sizeof(double));
    for (long r = lo; r < hi; ++r) {
        long b = c->row_lo + r;
        for (long a = 0; a < nr1; ++a) { zx[a] = grid_x(c->R, a); zy[a] = grid_y(c->R, b); }
        if (c->F) orc_fmm_alpha(c->F, nr1, zx, zy, ax, ay, NULL, 1);
        else orc_alpha_direct(c->n, c->sx, c->sy, c->sm, nr1, zx, zy, ax, ay, 1);
        for (long a = 0; a < nr1; ++a)
            lens_equation(c->L, zx[a], zy[a], ax[a], ay[a], &c->wx[r * nr1 + a], &c->wy[r * nr1 + a]);
    }
    free(zx); free(zy); free(ax); free(ay);
}

/* source positions of vertex rows [row_lo, row_hi) */
void orc_shoot_rows(const orc_region *R, double kappa_star, double kappa_smooth, double gamma,
                    int sheet, double e1, double e2, const double *psi3, long n, const double *sx, const double *sy,
                    const double *sm, const void *F, long row_lo, long row_hi,
                    double *wx, double *wy, int nthreads)
{
    orc_lens L = {kappa_star, kappa_smooth, gamma, sheet, e1, e2, {0, 0, 0, 0}};
    lens_set_psi3(&L, psi3);
    shoot_ctx c = {R, &L, n, sx, sy, sm, F, row_lo, wx, wy};
    parallel_for(row_hi - row_lo, nthreads, shoot_rows, &c);
}

/* ------------------------------------------------------------------------ */
/* inverse ray shooting (sec. 2.3, 4)                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    const orc_region *R; const orc_lens *L;
    long n; const double *sx, *sy, *sm;
    const void *F;
    long row_lo; double *wx, *wy;
} irs_ctx;

/* source positions of the rays at the centres of the cells of some rows */
static void irs_shoot(void *vctx, long lo, long hi)
{
    irs_ctx *c = vctx;
    long nc = c->R->nr1 - 1;
    double *zx = malloc(nc * sizeof(double)), *zy = malloc(nc * sizeof(double));
    double *ax = malloc(nc * sizeof(double)), *ay = malloc(nc * sizeof(double));
    for (long r = lo; r < hi; ++r) {
        long b = c->row_lo + r;
        for (long a = 0; a < nc; ++a) {
            zx[a] = c->R->x0 + ((double)a + 0.5) * c->R->d1;
            zy[a] = c->R->y0 + ((double)b + 0.5) * c->R->d2;
        }
        if (c->F) orc_fmm_alpha(c->F, nc, zx, zy, ax, ay, NULL, 1);
        else orc_alpha_direct(c->n, c->sx, c->sy, c->sm, nc, zx, zy, ax, ay, 1);
        for (long a = 0; a < nc; ++a)
            lens_equation(c->L, zx[a], zy[a], ax[a], ay[a], &c->wx[r * nc + a], &c->wy[r * nc + a]);
    }
    free(zx); free(zy); free(ax); free(ay);
}

/*
 * IRS over cell rows [row_lo, row_hi): one ray at the centre of every grid
 * cell (a, b), z = (x0 + (a + 1/2) D1, y0 + (b + 1/2) D2), is deflected and
 * counted in the pixel (floor u, floor v) it lands in, u = (w1 - ylo1) / pix1,
 * v = (w2 - ylo2) / pix2, when that pixel is inside the map: counts[j n1 + i]
 * += 1.  A ray stands for its cell's image area D1 D2, so the magnification
 * is counts D1 D2 / (pix1 pix2).  uv (may be NULL) receives every ray's
 * (u, v), row by row.  Returns the number of rays landing outside the map.
 */
long orc_irs_rows(const orc_region *R, double kappa_star, double kappa_smooth, double gamma, int sheet,
                  double e1, double e2, const double *psi3, long n, const double *sx, const double *sy,
                  const double *sm, const void *F, long row_lo, long row_hi, long *counts, double *uv, int nthreads)
{
    orc_lens L = {kappa_star, kappa_smooth, gamma, sheet, e1, e2, {0, 0, 0, 0}};
    lens_set_psi3(&L, psi3);
    long nc = R->nr1 - 1, nrays = (row_hi - row_lo) * nc;
    double *wx = malloc((nrays > 0 ? nrays : 1) * sizeof(double));
    double *wy = malloc((nrays > 0 ? nrays : 1) * sizeof(double));
    irs_ctx c = {R, &L, n, sx, sy, sm, F, row_lo, wx, wy};
    parallel_for(row_hi - row_lo, nthreads, irs_shoot, &c);
    double ylo1 = R->y1c - R->hw1, ylo2 = R->y2c - R->hw2;
    long out = 0;
    for (long k = 0; k < nrays; ++k) {
        double u = (wx[k] - ylo1) / R->pix1, v = (wy[k] - ylo2) / R->pix2;
        if (uv) { uv[2 * k] = u; uv[2 * k + 1] = v; }
        double fu = floor(u), fv = floor(v);
        if (fu >= 0.0 && fv >= 0.0 && fu < (double)R->n1 && fv < (double)R->n2)
            counts[(long)fv * R->n1 + (long)fu] += 1;
        else
            ++out;
    }
    free(wx); free(wy);
    return out;
}

/* ------------------------------------------------------------------------ */
/* cell refinement (not in the paper, which does no subdivision, sec. 3.2):  */
/* the plain test the learned variant is judged against                     */
/* ------------------------------------------------------------------------ */

static double sgn(double x) { return (x > 0.0) - (x < 0.0); }

/* twice the signed area of (a, b, c) */
static double area2(double ua, double va, double ub, double vb, double uc, double vc)
{
    return (ub - ua) * (vc - va) - (uc - ua) * (vb - va);
}

/* Features of a mapped cell: corners (u, v) in pixel units in the order
   00, 10, 11, 01; f[0..7] = sign(d) log(1 + |d|) of each corner's offset
   from the corner of the pixel holding the mean of the four (so both the
   cell's shape and where it falls on the pixel grid show), f[8..11] = signs
   of the mapped ears at the corners (00: (00, 10, 01); 10: (10, 11, 00);
   11: (11, 01, 10); 01: (01, 00, 11)), which all agree unless the cell is
   folded. */
void orc_cell_features(const double *u4, const double *v4, double *f)
{
    double cu = floor(0.25 * (u4[0] + u4[1] + u4[2] + u4[3]));
    double cv = floor(0.25 * (v4[0] + v4[1] + v4[2] + v4[3]));
    for (int k = 0; k < 4; ++k) {
        double du = u4[k] - cu, dv = v4[k] - cv;
        f[2 * k] = sgn(du) * log1p(fabs(du));
        f[2 * k + 1] = sgn(dv) * log1p(fabs(dv));
    }
    for (int k = 0; k < 4; ++k) {
        int p = (k + 3) % 4, q = (k + 1) % 4;   /* neighbours in the cycle 00, 10, 11, 01 */
        f[8 + k] = sgn(area2(u4[k], v4[k], u4[q], v4[q], u4[p], v4[p]));
    }
}

typedef struct {
    const orc_region *R;
    orc_lens L;
    long n;
    const double *sx, *sy, *sm;
    const void *F;
    double tau;
    int max_depth, window;
    double *dmap;              /* image-area deposits of (refined - plain) */
    long n_tested, n_refined, n_large;
} refine_ctx;

/* source position of image point (A d1 + x0, B d2 + y0), in pixel units */
static void refine_shoot(const refine_ctx *c, double A, double B, double *u, double *v)
{
    const orc_region *R = c->R;
    double x = R->x0 + A * R->d1, y = R->y0 + B * R->d2;
    double ax, ay;
    if (c->F) orc_fmm_alpha(c->F, 1, &x, &y, &ax, &ay, NULL, 1);
    else orc_alpha_direct(c->n, c->sx, c->sy, c->sm, 1, &x, &y, &ax, &ay, 1);
    double wx, wy;
    lens_equation(&c->L, x, y, ax, ay, &wx, &wy);
    *u = (wx - (R->y1c - R->hw1)) / R->pix1;
    *v = (wy - (R->y2c - R->hw2)) / R->pix2;
}

/* image-area deposit of triangle (u, v) of image area AT into pixel (i, j) */
static double tri_dep(double AT, const double *u, const double *v, long i, long j)
{
    double S = 0.5 * area2(u[0], v[0], u[1], v[1], u[2], v[2]);
    if (!(S != 0.0) || !isfinite(S)) return 0.0;
    double a = orc_tri_pixel_area(u, v, i, j);
    return a == 0.0 ? 0.0 : AT * (a / S);
}

/* a (sub)cell's two triangles, corners in the order 00, 10, 11, 01 */
static void cell_tris(const double *u4, const double *v4, double tu[2][3], double tv[2][3])
{
    const int t[2][3] = {{0, 1, 2}, {0, 2, 3}};
    for (int k = 0; k < 2; ++k)
        for (int m = 0; m < 3; ++m) { tu[k][m] = u4[t[k][m]]; tv[k][m] = v4[t[k][m]]; }
}

static void add_cell(refine_ctx *c, double AT, const double *u4, const double *v4, double sign)
{
    double tu[2][3], tv[2][3];
    cell_tris(u4, v4, tu, tv);
    const orc_region *R = c->R;
    for (int k = 0; k < 2; ++k) {
        int ok = 1;
        for (int m = 0; m < 3; ++m) ok &= isfinite(tu[k][m]) && isfinite(tv[k][m]);
        if (!ok) continue;
        double umin = fmin(tu[k][0], fmin(tu[k][1], tu[k][2])), umax = fmax(tu[k][0], fmax(tu[k][1], tu[k][2]));
        double vmin = fmin(tv[k][0], fmin(tv[k][1], tv[k][2])), vmax = fmax(tv[k][0], fmax(tv[k][1], tv[k][2]));
        long i0 = (long)floor(umin), i1 = (long)floor(umax), j0 = (long)floor(vmin), j1 = (long)floor(vmax);
        if (i0 < 0) i0 = 0;
        if (j0 < 0) j0 = 0;
        if (i1 > R->n1 - 1) i1 = R->n1 - 1;
        if (j1 > R->n2 - 1) j1 = R->n2 - 1;
        for (long j = j0; j <= j1; ++j)
            for (long i = i0; i <= i1; ++i) c->dmap[j * R->n1 + i] += sign * tri_dep(AT, tu[k], tv[k], i, j);
    }
}

/* The test of one (sub)cell at depth d (image corners A0 + {0, h} x
   B0 + {0, h} in grid units, source corners u4, v4):  refine if the mapped
   ears disagree, or if splitting it 2 x 2 changes its in-map deposits by
   more than tau times its image area (L1 over the pixels).  Cells whose
   parent or child triangles span more than `window` pixels along an axis
   are not refined.  A refined cell is replaced by its four children, each
   tested again while d + 1 < max_depth.  Deposits of (leaves - cell) go to
   dmap.  Returns whether the cell was refined. */
static int refine_rec(refine_ctx *c, double A0, double B0, double h, int d, const double *u4, const double *v4)
{
    const orc_region *R = c->R;
    c->n_tested++;
    double f[12];
    orc_cell_features(u4, v4, f);
    int fold = !(f[8] == f[9] && f[9] == f[10] && f[10] == f[11]);
    /* children: grid vertices (A0 + {0, h/2, h}, B0 + {0, h/2, h}) */
    double gu[3][3], gv[3][3];
    gu[0][0] = u4[0]; gv[0][0] = v4[0];
    gu[0][2] = u4[1]; gv[0][2] = v4[1];
    gu[2][2] = u4[2]; gv[2][2] = v4[2];
    gu[2][0] = u4[3]; gv[2][0] = v4[3];
    double hh = 0.5 * h;
    refine_shoot(c, A0 + hh, B0, &gu[0][1], &gv[0][1]);
    refine_shoot(c, A0, B0 + hh, &gu[1][0], &gv[1][0]);
    refine_shoot(c, A0 + hh, B0 + hh, &gu[1][1], &gv[1][1]);
    refine_shoot(c, A0 + h, B0 + hh, &gu[1][2], &gv[1][2]);
    refine_shoot(c, A0 + hh, B0 + h, &gu[2][1], &gv[2][1]);
    /* extent of parent and children */
    double umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            umin = fmin(umin, gu[r][s]); umax = fmax(umax, gu[r][s]);
            vmin = fmin(vmin, gv[r][s]); vmax = fmax(vmax, gv[r][s]);
        }
    if (!(umax - umin <= c->window && vmax - vmin <= c->window)) { c->n_large++; return 0; }
    double AT = 0.5 * (h * R->d1) * (h * R->d2);   /* image area of one parent triangle */
    int refine = fold;
    if (!refine) {
        /* L1 change of the in-map deposits */
        long i0 = (long)floor(umin), i1 = (long)floor(umax), j0 = (long)floor(vmin), j1 = (long)floor(vmax);
        if (i0 < 0) i0 = 0;
        if (j0 < 0) j0 = 0;
        if (i1 > R->n1 - 1) i1 = R->n1 - 1;
        if (j1 > R->n2 - 1) j1 = R->n2 - 1;
        double l1 = 0.0;
        double pu[2][3], pv[2][3];
        cell_tris(u4, v4, pu, pv);
        for (long j = j0; j <= j1; ++j)
            for (long i = i0; i <= i1; ++i) {
                double diff = -tri_dep(AT, pu[0], pv[0], i, j) - tri_dep(AT, pu[1], pv[1], i, j);
                for (int r = 0; r < 2; ++r)
                    for (int s = 0; s < 2; ++s) {
                        double cu[4] = {gu[r][s], gu[r][s + 1], gu[r + 1][s + 1], gu[r + 1][s]};
                        double cv[4] = {gv[r][s], gv[r][s + 1], gv[r + 1][s + 1], gv[r + 1][s]};
                        double tu[2][3], tv[2][3];
                        cell_tris(cu, cv, tu, tv);
                        diff += tri_dep(0.25 * AT, tu[0], tv[0], i, j) + tri_dep(0.25 * AT, tu[1], tv[1], i, j);
                    }
                l1 += fabs(diff);
            }
        refine = l1 > c->tau * 2.0 * AT;
    }
    if (!refine) return 0;
    c->n_refined++;
    add_cell(c, AT, u4, v4, -1.0);
    for (int r = 0; r < 2; ++r)
        for (int s = 0; s < 2; ++s) {
            double cu[4] = {gu[r][s], gu[r][s + 1], gu[r + 1][s + 1], gu[r + 1][s]};
            double cv[4] = {gv[r][s], gv[r][s + 1], gv[r + 1][s + 1], gv[r + 1][s]};
            double a0 = A0 + s * hh, b0 = B0 + r * hh;
            add_cell(c, 0.25 * AT, cu, cv, +1.0);   /* a refined child takes this back itself */
            if (d + 1 < c->max_depth) refine_rec(c, a0, b0, hh, d + 1, cu, cv);
        }
    return 1;
}

/* The plain refinement of cells (a[k], b[k]) of the ray grid: label[k] = 1
   if the cell itself is refined; dmap (n2 x n1, image-area units, not
   normalised) receives the refined minus the plain deposits; stats =
   {tested (sub)cells, refined (sub)cells, skipped as too large}. */
void orc_refine_cells(const orc_region *R, double kappa_star, double kappa_smooth, double gamma, int sheet,
                      double e1, double e2, const double *psi3, long n, const double *sx, const double *sy,
                      const double *sm, const void *F,
                      long ncells, const long *ca, const long *cb, double tau, int max_depth, int window,
                      unsigned char *label, double *dmap, long *stats)
{
    refine_ctx c = {R, {kappa_star, kappa_smooth, gamma, sheet, e1, e2, {0, 0, 0, 0}}, n, sx, sy, sm, F, tau,
                    max_depth, window, dmap, 0, 0, 0};
    lens_set_psi3(&c.L, psi3);
    for (long k = 0; k < ncells; ++k) {
        double u4[4], v4[4];
        double A = (double)ca[k], B = (double)cb[k];
        refine_shoot(&c, A, B, &u4[0], &v4[0]);
        refine_shoot(&c, A + 1.0, B, &u4[1], &v4[1]);
        refine_shoot(&c, A + 1.0, B + 1.0, &u4[2], &v4[2]);
        refine_shoot(&c, A, B + 1.0, &u4[3], &v4[3]);
        label[k] = (unsigned char)(max_depth > 0 ? refine_rec(&c, A, B, 1.0, 0, u4, v4) : 0);
    }
    stats[0] += c.n_tested;
    stats[1] += c.n_refined;
    stats[2] += c.n_large;
}
