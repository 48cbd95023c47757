/*
 * mlmap.h -- C ABI of the MI355X microlensing magnification-map library.
 *
 * The library computes source-plane magnification maps of a field of point
 * mass microlenses embedded in a macro model (convergence kappa, shear gamma),
 * following Weisenbach 2025, "Rootin' Tootin' Efficient Ray Shootin'":
 *
 *   lens equation (sec. 2.2)   w = (1-kappa) z + gamma conj(z) - a_*(z) - a_s(z)
 *   star deflection            a_*(z) = sum_i m_i / conj(z - z_i), evaluated with a
 *                              quadtree fast multipole method (sec. 3.3, app. C)
 *   compensating sheet         a_s(z) = -kappa_* z inside the star disc (sec. 3.1)
 *   map                        inverse polygon mapping of the ray grid's triangular
 *                              cells onto source pixels (sec. 3.2)
 *
 * Units: theta_* = 1 (lengths in Einstein radii of a unit-mass lens).
 * Complex positions are passed as interleaved (x1, x2) double pairs.
 *
 * General rules
 *   - Every call returns an mlm_status; the library never aborts or exits.
 *     On error, out-parameters are left untouched and mlm_last_error()
 *     returns a description (per calling thread).
 *   - "device" pointers are HIP device allocations of the current device
 *     (for example the data_ptr() of a torch tensor on cuda:0); "host"
 *     pointers are ordinary process memory.  Which one a pointer is is
 *     stated by an explicit flag, never guessed.
 *   - Objects returned through `**out` are owned by the library and must be
 *     released with the matching destroy call.  Caller arrays are copied on
 *     entry; the library keeps no reference to them.
 *   - A lens may be used from several threads, but map calls on one lens are
 *     serialised (they share the lens's device workspace).
 */
#ifndef MLMAP_H
#define MLMAP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define MLM_ABI_VERSION 6

typedef enum mlm_status {
    MLM_OK = 0,
    MLM_EINVAL = 1,       /* invalid argument (NaN, negative size, bad enum, NULL) */
    MLM_EDEGENERATE = 2,  /* |1 - kappa +- gamma| < 1e-9: shooting region unbounded */
    MLM_ERANGE = 3,       /* a size exceeds what the library supports */
    MLM_ENOMEM = 4,       /* host or device allocation failed */
    MLM_EDEVICE = 5,      /* a HIP runtime call failed */
    MLM_ENOTSUP = 6       /* option not supported by this build */
} mlm_status;

/* ABI version of the loaded library (MLM_ABI_VERSION of its build). */
int32_t mlm_abi_version(void);

/* Static, human-readable name of a status code. */
const char *mlm_status_str(mlm_status s);

/* Detail of the last failing call on this thread ("" if none).  The pointer
   stays valid until the next failing call on the same thread. */
const char *mlm_last_error(void);

/* ------------------------------------------------------------------------ */
/* lens                                                                      */
/* ------------------------------------------------------------------------ */

enum { MLM_SHEET_CIRCLE = 0, MLM_SHEET_NONE = 1, MLM_SHEET_RECT = 2 };

/*
 * Macro model and microlens field (sec. 2.1-2.2, 3.1, app. B).
 *   kappa_star   convergence in microlenses, >= 0.  The stars are taken to
 *                fill a region of area pi sum(m_i) / kappa_star (sec. 2.1
 *                with theta_* = 1), so the realised kappa_* is the requested
 *                one, and a compensating sheet of -kappa_star over that
 *                region is added:
 *                MLM_SHEET_CIRCLE: a disc of radius R_* = sqrt(sum m_i /
 *                kappa_star); a_s = -kappa_* z for |z| <= R_* and
 *                -kappa_* R_*^2 / conj(z) outside (sec. 3.1, both branches
 *                of its footnote);
 *                MLM_SHEET_RECT: the rectangle [-c1, c1] x [-c2, c2] with
 *                c2 = rect_aspect c1 and 4 c1 c2 = pi sum m_i / kappa_star;
 *                a_s is app. B's closed form with four complex logarithms
 *                and its branch-cut terms, valid inside and outside.
 *   kappa_smooth smooth convergence; kappa = kappa_star + kappa_smooth.
 *   gamma        external shear, real (the frame is rotated onto it, sec. 2.1).
 *   sheet        MLM_SHEET_CIRCLE, MLM_SHEET_RECT or MLM_SHEET_NONE (no
 *                compensating sheet: for isolated lenses such as the point
 *                lens).
 *   rect_aspect  c2 / c1 of the star rectangle (MLM_SHEET_RECT, > 0).
 */
typedef struct mlm_lens_params {
    double kappa_star;
    double kappa_smooth;
    double gamma;
    int32_t sheet;
    int32_t reserved;
    double rect_aspect;
    /* Third derivatives of the macro potential at the expansion point (app. D:
     * near a macro critical curve the potential is expanded past second order):
     * psi3 = (psi_111, psi_112, psi_122, psi_222).  The lens equation gains
     * -a_3 with a_3,i = (1/2) sum_jk psi_ijk x_j x_k (the gradient of
     * (1/6) sum_ijk psi_ijk x_i x_j x_k), in every kernel that shoots rays.
     * All zero (the default): the second-order model of sec. 2.1.  With any
     * nonzero, 1 - kappa -+ gamma may vanish (a fold through the expansion
     * point), and the shooting region is the request's (x1c, x2c, dx1, dx2)
     * when it sets centre_set, else derived as described at mlm_map_region. */
    double psi3[4];
} mlm_lens_params;

typedef struct mlm_lens mlm_lens;

/*
 * Create a lens from a star field: x[i], y[i] position (theta_*), m[i] > 0
 * mass, i < n, n >= 0.  With device_ptrs != 0 the three arrays are device
 * pointers, else host pointers; either way they are copied.  The stars are
 * kept resident in device memory for the lens's lifetime.
 * Errors: MLM_EINVAL for NULL out, n < 0, non-finite values, m <= 0,
 * kappa_star < 0 (or kappa_star == 0 with stars and a sheet); MLM_ENOMEM;
 * MLM_EDEVICE.
 */
mlm_status mlm_lens_create(const mlm_lens_params *params, const double *x, const double *y,
                           const double *m, int64_t n, int32_t device_ptrs, mlm_lens **out);

/* Release a lens (NULL is accepted). */
void mlm_lens_destroy(mlm_lens *lens);

/* Derived lens quantities (sec. 2.1, 3.1). */
typedef struct mlm_lens_info {
    int64_t n_stars;
    double mass_sum;      /* sum m_i */
    double mean_m;        /* <m> */
    double mean_m2;       /* <m^2> */
    double r_star;        /* radius of the star disc, sqrt(sum m / kappa_*) */
    double kappa;         /* kappa_* + kappa_s */
    double mu_macro;      /* 1 / ((1-kappa)^2 - gamma^2) */
    double max_abs;       /* max over stars of max(|x|, |y|) */
    double extent1;       /* star region: R_* (disc) or c1 (rectangle); 0 without a sheet */
    double extent2;       /* R_* (disc) or c2 (rectangle) */
} mlm_lens_info;

mlm_status mlm_lens_get_info(const mlm_lens *lens, mlm_lens_info *out);

/*
 * The lens's stars, in the order they were given or drawn: up to cap of
 * them into host arrays x, y, m (any may be NULL); *n receives the count.
 * Lets a checker consume exactly the field the library holds.
 * Errors: MLM_EINVAL (NULL lens or n), MLM_ERANGE (cap < count: nothing
 * copied, *n set), MLM_EDEVICE.
 */
mlm_status mlm_lens_stars(const mlm_lens *lens, double *x, double *y, double *m, int64_t cap, int64_t *n);


/* ------------------------------------------------------------------------ */
/* map request                                                               */
/* ------------------------------------------------------------------------ */

enum { MLM_PREC_FP64 = 0, MLM_PREC_MIXED = 1 };
enum { MLM_REFINE_NONE = 0, MLM_REFINE_PLAIN = 1, MLM_REFINE_LEARNED = 2 };
enum { MLM_METHOD_FMM = 0, MLM_METHOD_DIRECT = 1 };
enum { MLM_MAP_IPM = 0, MLM_MAP_IRS = 1 };

/*
 * Map request.  Fill with mlm_map_request_init() and override fields.
 *
 *   y1c, y2c       source-plane map centre (Y1, Y2)                  (sec. 2.3)
 *   hw1, hw2       map half-widths (dY1, dY2) > 0
 *   n1, n2         pixels along y1 and y2, >= 1
 *   rays_per_pixel ray-grid density "in the absence of lensing": cell side
 *                  pix_i / sqrt(rho) (sec. 4), default 1
 *   nray1, nray2   explicit ray-grid vertex counts (> 1 both), spanning
 *                  exactly [X - dX, X + dX]; 0 = derive from rays_per_pixel
 *   flux_fraction  f of appendix A: border r = sqrt(kappa_* <m^2> / (f <m>)),
 *                  default 0.01
 *   dx1, dx2       explicit image-plane half-sizes of the shooting region;
 *                  0 = (dY_i + r) / |1 - kappa +- gamma| (sec. 2.3)
 *   order          FMM expansion order p in [1, 31]; 0 = the rule of
 *                  appendix C.3 with the accuracy `eps`
 *   leaf_max       maximum stars in a node's 3x3 block of same-level
 *                  squares before it is divided (app. C.1), default 32
 *   max_level      deepest tree level, default and maximum 24
 *   precision      MLM_PREC_FP64 (everything in double) or MLM_PREC_MIXED:
 *                  the near field, the Taylor series' variation across a
 *                  leaf (its terms l >= 1 in the leaf's local coordinate)
 *                  and the column pass of the IPM in FP32; the multipole
 *                  and Taylor coefficients (app. C.2), the far field at
 *                  each leaf centre, grid positions, leaf centres and
 *                  offsets from them, the macro model, the sheet, triangle
 *                  set-up, thin triangles (squared extent above 256 x
 *                  twice the area, the ones folded across caustics), the
 *                  row-band pass and every pixel sum in FP64 (the paper's
 *                  single-precision mode, sec. 5, with FP64 kept where the
 *                  field's magnitude or caustics need it).  With
 *                  MLM_METHOD_DIRECT it gives MLM_ENOTSUP.
 *   method         MLM_METHOD_FMM or MLM_METHOD_DIRECT (every star summed
 *                  for every ray; the no-FMM reference of sec. 4)
 *   refine         cell refinement after the IPM (the paper apportions
 *                  each cell as two triangles, sec. 3.2; refinement splits
 *                  cells where that is coarse): MLM_REFINE_PLAIN tests every
 *                  cell: refine if the mapped ears disagree in orientation
 *                  or a 2 x 2 split changes the cell's in-map deposits by
 *                  more than refine_tau times its image area (L1), children
 *                  tested again down to refine_depth levels, cells wider
 *                  than refine_window pixels left alone; MLM_REFINE_LEARNED
 *                  runs the same test only on the cells `refiner` flags
 *                  (logit > refine_threshold) and on every folded cell.
 *                  FP64 with the FMM only (else MLM_ENOTSUP).
 *   device_out     != 0: `mu` (and `w_out`) are device pointers
 *   eps            absolute deflection accuracy for the automatic order,
 *                  default 1e-7
 *   row_begin,     map only the ray-grid cell rows [row_begin, row_end);
 *   row_end        row_end < 0 means all rows.  Maps are additive over
 *                  disjoint row ranges.
 *   stream         hipStream_t to run on (NULL: the default stream).  The
 *                  call returns after the work on it has completed.
 *   w_out          optional: receives the mapped source positions (y1, y2)
 *                  of the vertex rows row_begin .. row_end (inclusive),
 *                  nray1 per row, interleaved doubles (2 * nr1 * rows).
 *   mapping        MLM_MAP_IPM: inverse polygon mapping of the grid's
 *                  triangular cells (sec. 3.2); MLM_MAP_IRS: inverse ray
 *                  shooting (sec. 2.3, 4), one ray at the centre of every
 *                  grid cell, counted in the pixel it lands in, so that
 *                  mu = count x (cell area) / (pixel area); with the
 *                  paper's 10^2 - 10^3 rays per pixel.  IRS rows are the
 *                  same cell rows, so IRS maps are additive over row
 *                  ranges too; it takes no w_out and no refinement.
 *   timing         1: record device times of each stage into the stats;
 *                  2: also count the IPM kernels' work (n_big_rows,
 *                  n_band_rows, n_band_pieces, n_small, n_col_items,
 *                  n_col_pieces), which adds a little device work
 */
typedef struct mlm_map_request {
    double y1c, y2c, hw1, hw2;
    int32_t n1, n2;
    double rays_per_pixel;
    int32_t nray1, nray2;
    double flux_fraction;
    double dx1, dx2;
    int32_t order;
    int32_t leaf_max;
    int32_t max_level;
    int32_t precision;
    int32_t method;
    int32_t device_out;
    double eps;
    int64_t row_begin, row_end;
    void *stream;
    double *w_out;
    int32_t timing;
    int32_t refine;            /* MLM_REFINE_NONE, _PLAIN or _LEARNED */
    int32_t refine_depth;      /* levels of 2 x 2 splitting, 1..4 (default 3) */
    int32_t refine_window;     /* widest (sub)cell image refined, pixels (default 8) */
    double refine_tau;         /* L1 threshold over the cell's image area (default 1e-3) */
    double refine_threshold;   /* logit above which the network flags a cell (default 0) */
    struct mlm_refiner *refiner;   /* network for MLM_REFINE_LEARNED */
    int32_t mapping;           /* MLM_MAP_IPM (default) or MLM_MAP_IRS */
    int32_t one_stream;        /* 0 (default): the large-triangle passes of the IPM run on a
                                  second stream of the lens beside the cell pass (fork and join
                                  through events on req->stream); 1: every kernel on req->stream */
    double x1c, x2c;           /* image-plane centre of the shooting region, used when
                                  centre_set (with dx1, dx2 > 0 as its half-sizes) */
    int32_t centre_set;
    int32_t big_pixels;        /* IPM: a triangle whose bounding box covers more pixels than this
                                  goes through the row-band pass (0: 64; the batch's autotuner
                                  picks it per class of map) */
} mlm_map_request;

void mlm_map_request_init(mlm_map_request *req);

/* Shooting region, ray grid and tree root of a request (sec. 2.3, app. A). */
typedef struct mlm_region {
    double lam1, lam2;      /* 1 - kappa + gamma, 1 - kappa - gamma */
    double mu_macro;
    double border;          /* r of appendix A */
    double X1, X2;          /* shooting-region centre */
    double dX1, dX2;        /* shooting-region half-sizes */
    double pix1, pix2;      /* pixel sides */
    double d1, d2;          /* ray-grid spacing */
    double x0, y0;          /* position of vertex (0, 0); vertex (a, b) is
                               (x0 + a d1, y0 + b d2) */
    double L0;              /* half-length of the tree's root square (power of 2) */
    int64_t nr1, nr2;       /* ray-grid vertices per row / per column */
    int32_t order;          /* expansion order the map would use (0 if it needs the tree) */
    int32_t reserved;
} mlm_region;

/* Compute the region of a request without mapping.  Errors as mlm_map. */
mlm_status mlm_map_region(const mlm_lens *lens, const mlm_map_request *req, mlm_region *out);

/* ------------------------------------------------------------------------ */
/* star fields drawn by the library                                          */
/* ------------------------------------------------------------------------ */

/*
 * Mass functions (the paper names Salpeter and "a variety"; sec. 2.1, 5):
 *   MLM_MASS_EQUAL     every m = m_equal
 *   MLM_MASS_SALPETER  dN/dm ~ m^-2.35 on [m_lo, m_hi]
 *   MLM_MASS_KROUPA    dN/dm ~ m^-1.3 on [m_lo, 0.5), ~ m^-2.3 on [0.5, m_hi],
 *                      continuous at 0.5 (needs m_lo < 0.5 < m_hi)
 * Masses are drawn by inverse CDF; positions uniformly in the disc or
 * rectangle that realises kappa_star for the drawn total mass (the region
 * mlm_lens_params describes).  Star i's draws are Philox4x32-10 blocks with
 * counter (i mod 2^32, i div 2^32, b, 0), b = 0, 1, and key (seed mod 2^32,
 * seed div 2^32): mass from words 0-1 of block 0, then from words 2-3 of
 * block 0 and 0-1 of block 1 the disc's (r^2 / R_*^2, angle / 2 pi) or the
 * rectangle's ((x / c1 + 1) / 2, (y / c2 + 1) / 2); a uniform in (0, 1) is
 * ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53 of two words (a, b).
 */
enum { MLM_MASS_EQUAL = 0, MLM_MASS_SALPETER = 1, MLM_MASS_KROUPA = 2 };

typedef struct mlm_field_params {
    double kappa_star;       /* > 0 */
    int32_t mass_fn;         /* MLM_MASS_* */
    int32_t shape;           /* MLM_SHEET_CIRCLE (disc) or MLM_SHEET_RECT */
    double m_equal;          /* MLM_MASS_EQUAL's mass, > 0 (default 1) */
    double m_lo, m_hi;       /* power-law range (defaults 0.1, 1) */
    int64_t n_stars;         /* > 0: this many; 0: kappa_star extent / (pi <m>)
                                with the mass function's <m> (sec. 2.1), rounded */
    double extent1, extent2; /* n_stars == 0: disc radius (extent1), or the
                                rectangle's half-sides */
    double rect_aspect;      /* rectangle c2 / c1 (> 0; 0 with n_stars == 0:
                                extent2 / extent1) */
    uint64_t seed;
} mlm_field_params;

void mlm_field_params_init(mlm_field_params *f);

/* The mass function's <m> and <m^2> (exact integrals). */
mlm_status mlm_field_moments(const mlm_field_params *f, double *mean_m, double *mean_m2);

/* The number of stars a field has (n_stars, or the count its extent gives). */
mlm_status mlm_field_count(const mlm_field_params *f, int64_t *n);

/*
 * Draw a field into host arrays of capacity cap: *n stars; extent1/extent2
 * (may be NULL) receive the realised region (R_*, R_* or c1, c2).
 * Errors: MLM_EINVAL (bad parameters), MLM_ERANGE (cap below the count:
 * nothing written but *n).
 */
mlm_status mlm_field_sample(const mlm_field_params *f, double *x, double *y, double *m, int64_t cap, int64_t *n,
                            double *extent1, double *extent2);

/*
 * The star region that covers a map request's shooting region (sec. 2.3,
 * 3.1: "somewhat larger"): margin times the disc radius reaching the
 * rectangle's farthest corner, or margin times the rectangle
 * (|X1| + dX1, |X2| + dX2); the border r of appendix A uses the mass
 * function's exact <m>, <m^2>.  With f->n_stars = 0 and these extents,
 * mlm_field_count gives the paper's star count for the map.
 */
mlm_status mlm_field_cover(const mlm_lens_params *params, const mlm_field_params *f, const mlm_map_request *req,
                           double margin, double *extent1, double *extent2);

/*
 * Create a lens from a field the library draws (mlm_field_sample's stars):
 * params->kappa_star must equal f->kappa_star, and params->sheet must be
 * f->shape or MLM_SHEET_NONE; a rectangle's aspect is taken from the field.
 */
mlm_status mlm_lens_create_sampled(const mlm_lens_params *params, const mlm_field_params *f, mlm_lens **out);

/* The published Philox4x32-10 block (Salmon et al. 2011) the sampler draws
 * from: out = philox(counter, key). */
void mlm_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4]);

typedef struct mlm_map_stats {
    int64_t n_rays;          /* grid vertices shot */
    int64_t n_cells;         /* grid cells apportioned (2 triangles each) */
    int64_t n_skipped;       /* triangles skipped for a non-finite vertex */
    int64_t n_nodes, n_leaves;
    int32_t n_levels, order;
    int64_t near_pairs;      /* ray-star pairs summed directly */
    int64_t n_tiles;         /* ray tiles launched */
    double tri_area;         /* image-plane area of one triangle, d1 d2 / 2 */
    double t_tree_ms;        /* sort + tree + lists (device time, if timing) */
    double t_fmm_ms;         /* P2M, M2M, M2L/P2L/L2L, leaf tables */
    double t_shoot_ms;       /* ray shooting kernels */
    double t_ipm_ms;         /* IPM kernels */
    double t_total_ms;       /* whole call, device time */
    int32_t n_shoot_launches, n_ipm_launches;
    int64_t n_big;           /* triangles apportioned row by row (large mapped area) */
    int64_t n_big_rows;      /* pixel rows those triangles cover inside the map (if timing 2) */
    /* the following are filled only when req->timing is set (counts: timing 2) */
    double t_cells_ms;       /* per-cell IPM kernel (ordinary triangles) */
    double t_band_ms;        /* per-band IPM kernel (large triangles) */
    int64_t n_band_rows;     /* (large triangle, pixel row) pairs the per-band kernel visits */
    int64_t n_band_pieces;   /* column differences those rows deposit inside the map */
    int64_t n_refine_candidates;   /* cells the refinement test ran on */
    int64_t n_refined;       /* cells refined (their own test passed) */
    int64_t n_refine_tests;  /* (sub)cells tested, all depths */
    int64_t n_refine_large;  /* (sub)cells left alone for their width */
    double t_refine_ms;      /* features, network and refinement (if timing) */
    int64_t n_small;         /* triangles within 2 x 2 pixels, apportioned in place (if timing) */
    int64_t n_col_items;     /* (triangle, pixel column) items of the cell pass (if timing) */
    int64_t n_col_pieces;    /* pixel pieces those columns evaluate (if timing) */
    int64_t n_pieces;        /* (triangle, pixel) pairs that meet inside the map, over all
                                paths: the pieces the apportioning deposits (timing 2) */
    int32_t leaf_max;        /* the split threshold the tree used (tuned in batches) */
    int32_t big_pixels;      /* the IPM's band threshold used (tuned in batches) */
} mlm_map_stats;

/*
 * Magnification map (sec. 3.2): mu[j * n1 + i] is the magnification of pixel
 * (i, j) = [y1c - hw1 + i pix1, +pix1) x [y2c - hw2 + j pix2, +pix2), i.e.
 * row-major with rows along y2 ascending.  `mu` (n1 * n2 doubles, caller
 * owned, host or device per req->device_out) is overwritten.  stats may be
 * NULL.
 * Errors: MLM_EINVAL (bad request), MLM_EDEGENERATE (|1-kappa+-gamma| < 1e-9),
 * MLM_ERANGE (grid larger than 2^31 vertices per row or 2^31 rows),
 * MLM_ENOMEM, MLM_EDEVICE, MLM_ENOTSUP.
 */
mlm_status mlm_map(mlm_lens *lens, const mlm_map_request *req, double *mu, mlm_map_stats *stats);

/*
 * mlm_map without device allocation, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and errors as mlm_map; every buffer the
 * map needs beyond the lens, `mu` and `w_out` (the tree, coefficients, leaf
 * tables, vertex strips, IPM work lists, and `mu`'s device copy when it goes
 * to the host) is carved from a static device array of
 * MLM_NOALLOC_SCRATCH_MIB MiB that the library holds on each device it runs
 * on until the process ends; no hipMalloc, hipFree or pinned host
 * allocation is made (small host-side bookkeeping uses the C++ heap).
 *   - Calls on one device share its array and are serialised by a lock of
 *     the library's (a call returns after its work has completed); processes
 *     each have their own array.
 *   - The vertex strip is sized to what the array holds, so large grids run
 *     in more strips than under mlm_map.
 *   - MLM_ERANGE when the map cannot fit: at entry, if the sorted stars (48
 *     bytes each), two vertex rows and the host-bound map copy already
 *     exceed the array; later, if data-dependent lists (large triangles,
 *     row bands) exhaust it.  mlm_map takes such maps.
 *   - MLM_ENOTSUP for cell refinement.
 */
#define MLM_NOALLOC_SCRATCH_MIB 64
mlm_status mlm_map_noalloc(mlm_lens *lens, const mlm_map_request *req, double *mu, mlm_map_stats *stats);

/*
 * Products of a map (sec. 4.1, 5: light curves and magnification
 * histograms, the quantities the paper compares maps by).  `req` is the
 * request that made the map: its pixel geometry (y1c, y2c, hw1, hw2, n1,
 * n2), where the buffers live (device_out: device pointers, else host) and
 * its stream.
 *
 * Light curve of a point source moving along a straight track: mu at npts
 * points evenly spaced from (y1a, y2a) to (y1b, y2b), both ends included,
 * by bilinear interpolation between pixel centres (within half a pixel of
 * the map's edge the nearest row or column is repeated); NaN at points
 * outside the map.  out: npts doubles.
 */
mlm_status mlm_light_curve(const mlm_map_request *req, const double *mu, double y1a, double y2a, double y1b,
                           double y2b, int64_t npts, double *out);

/*
 * Histogram of log10(mu) over the map's n1 x n2 pixels: counts[0] holds the
 * pixels with mu <= 0 or log10(mu) < lo, counts[1 + b] those in
 * [lo + b w, lo + (b + 1) w) with w = (hi - lo) / nbins, counts[nbins + 1]
 * those at or above hi (and NaN).  counts: nbins + 2 int64 (host or device
 * per req->device_out).  Errors: MLM_EINVAL for nbins < 1 or hi <= lo.
 */
mlm_status mlm_histogram(const mlm_map_request *req, const double *mu, double lo, double hi, int32_t nbins,
                         int64_t *counts);

/*
 * Batched maps: many lenses and requests in one call, each map as mlm_map
 * would make it, but with the ray shooting and the IPM of many maps fused
 * into persistent launches that walk the concatenated work of all maps (so
 * small maps do not leave the GPU idle).  The per-map tree, FMM and leaf
 * tables are built first, one map after another; the maps are then taken in
 * chunks whose grids fit `vertex_budget` vertices at once.
 *   lenses[i], reqs[i]: map i (distinct lenses: each holds its map's tree
 *       until the call returns); requests must cover all rows, use the FMM,
 *       have no w_out and agree in device_out; reqs[0].stream is used.
 *   mus[i]: n2 x n1 output of map i (host or device per device_out).
 *   stats: NULL or nmaps per-map statistics (times of the fused stages are
 *       in `bstats`, not per map).
 *   opts: NULL for the defaults.
 *   bstats: NULL or the batch's statistics.
 * With opts->autotune, each map's leaf size (app. C.1's split threshold,
 * which trades near-field pairs against tree and expansion work) is chosen
 * among 8, 16, 32 and 64 by timing tree + FMM + shooting of a sample of the
 * map's rows for each, and the choice is cached per class of map (precision,
 * expansion order and rays per star in powers of two) for the process.
 * Errors: as mlm_map; MLM_EINVAL also for an empty or inconsistent batch;
 * MLM_ENOTSUP for a map the fused row bands cannot hold: more than 8192
 * pixels per row, or more bands (of 1 to 16 pixel rows) than a workgroup's
 * LDS can index (about 13 600 on MI355X).  mlm_map takes such maps.
 */
typedef struct mlm_batch_opts {
    int64_t vertex_budget;   /* vertices held at once, 0: 2^28 (at least the largest map) */
    int32_t autotune;        /* != 0: choose each map's leaf size by timed trials */
    int32_t reserved0;
    int64_t reserved[6];
} mlm_batch_opts;

typedef struct mlm_batch_stats {
    int64_t n_maps, n_chunks, n_rays, n_cells, n_big;
    double t_prep_ms;        /* host wall time of the preparing threads (trees, FMM, leaf tables,
                                tile plans, tuning); the map passes of prepared chunks overlap it */
    double t_shoot_ms;       /* fused ray shooting */
    double t_ipm_ms;         /* fused IPM passes */
    double t_total_ms;       /* whole call, device time */
    int64_t reserved[4];
} mlm_batch_stats;

mlm_status mlm_map_batch(mlm_lens *const *lenses, const mlm_map_request *reqs, int32_t nmaps, double *const *mus,
                         mlm_map_stats *stats, const mlm_batch_opts *opts, mlm_batch_stats *bstats);

/*
 * The refinement network (learned variant of the cell refinement, see
 * mlm_map_request.refine): 12 -> 64 -> 64 -> 1, ReLU, logit out; BF16
 * weights and activations with FP32 accumulation, FP32 master weights.
 * Parameters, FP32, MLM_REFINER_PARAMS of them in this order: W1 [12][64],
 * b1 [64], W2 [64][64], b2 [64], W3 [64], b3; layer l computes
 * relu(h W_l + b_l).  Features of a cell (corners 00, 10, 11, 01 mapped to
 * pixel units): sign(d) log(1 + |d|) of each corner's (u, v) offset from
 * the corner of the pixel holding the four corners' mean (8 values), then
 * the signs (+1, -1, 0) of the
 * mapped ears at the corners, ear k = (k, k + 1, k - 1) in that cyclic order.
 * Loss: mean [ pos_weight y softplus(-z) + (1 - y) softplus(z) ].
 * The refiner lives on the current device; calls on one refiner must not
 * overlap.
 */
#define MLM_REFINER_PARAMS 5057
typedef struct mlm_refiner mlm_refiner;

/* params: NULL for He-normal weights drawn with `seed` and zero biases. */
mlm_status mlm_refiner_create(const float *params, uint64_t seed, mlm_refiner **out);
void mlm_refiner_destroy(mlm_refiner *r);
mlm_status mlm_refiner_get_params(mlm_refiner *r, float *params);
mlm_status mlm_refiner_set_params(mlm_refiner *r, const float *params);

/* Logits of n feature rows (n x 12 floats); host or device pointers. */
mlm_status mlm_refiner_predict(mlm_refiner *r, const float *feats, int64_t n, float *logits, int32_t device_ptrs,
                               void *stream);

/* Loss of n labelled rows and its gradient (MLM_REFINER_PARAMS floats),
 * from the training kernels (one batch of n). */
mlm_status mlm_refiner_grads(mlm_refiner *r, const float *feats, const uint8_t *labels, int64_t n, float pos_weight,
                             float *grads, double *loss, int32_t device_ptrs, void *stream);

typedef struct mlm_train_opts {
    int32_t epochs;          /* default 4 */
    int32_t batch;           /* samples per step, default 4096 */
    float lr;                /* Adam step, default 1e-3 */
    float pos_weight;        /* weight of positive labels, default 1 */
    uint64_t seed;           /* shuffling */
    int32_t device_ptrs;     /* feats and labels on the device */
    int32_t graph;           /* 1 (default): an epoch's steps are captured once in a
                                HIP graph and replayed per epoch; 0: launched one by one */
    void *stream;            /* the training runs on a stream of the refiner's own,
                                after the work already queued on this one */
} mlm_train_opts;

void mlm_train_opts_init(mlm_train_opts *o);

/* Adam on the weighted cross-entropy over n labelled rows, `epochs` passes
 * in seeded random order; loss_per_epoch (host, epochs values) may be NULL. */
mlm_status mlm_refiner_train(mlm_refiner *r, const mlm_train_opts *opts, const float *feats, const uint8_t *labels,
                             int64_t n, float *loss_per_epoch);

/* Training samples of a map request: for cells (a, b) of its ray grid
 * (cells[2k], cells[2k + 1]), the features (n x 12) and the label of the
 * plain test at the first level (1: refine), from the request's tree
 * (FP64, FMM).  Host or device pointers per device_ptrs. */
mlm_status mlm_cell_samples(mlm_lens *lens, const mlm_map_request *req, const int64_t *cells, int64_t n, float *feats,
                            uint8_t *labels, int32_t device_ptrs);

/*
 * Source positions w(z) of arbitrary image-plane points through the same
 * FMM (or direct sum) the map uses (sec. 2.2, app. C): z_xy and w_xy are n
 * interleaved (x1, x2) pairs, host or device per req->device_out.  Points
 * outside the tree's root square (mlm_map_region's L0) give MLM_ERANGE.
 */
mlm_status mlm_deflect(mlm_lens *lens, const mlm_map_request *req, const double *z_xy, int64_t n,
                       double *w_xy);

/*
 * Export of the FMM tree and coefficients built for a request (app. C), for
 * inspection and parity checks.  Host buffers of capacity `cap` nodes; the
 * call fails with MLM_ERANGE if the tree has more nodes (info is still
 * filled).  Per node q: level, square indices (ix, iy) at that level, leaf
 * flag, stars in the node, stars in its 3x3 block; mult and local hold the
 * (order + 1) multipole and Taylor coefficients as interleaved (re, im)
 * doubles, in units of the node half-length (local[0] is not formed and is
 * zero).  Any output pointer may be NULL.
 */
typedef struct mlm_tree_info {
    int64_t n_nodes, n_leaves;
    int32_t n_levels, order;
    double L0;
} mlm_tree_info;

mlm_status mlm_fmm_export(mlm_lens *lens, const mlm_map_request *req, mlm_tree_info *info,
                          int32_t *level, int64_t *ix, int64_t *iy, int32_t *leaf, int64_t *nstars,
                          int64_t *block, double *mult, double *local, int64_t cap);

#ifdef __cplusplus
}
#endif

#endif /* MLMAP_H */
