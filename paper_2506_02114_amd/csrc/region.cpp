// Shooting region, ray grid, tree root and expansion order of a map request.
// Host arithmetic only; built with -ffp-contract=off so every formula is
// evaluated as written (plain IEEE double operations).
#include <cmath>

#include "internal.hpp"

namespace mlm {

/*
 * sec. 2.3 and appendix A:
 *   centre      X = (Y1 / (1-k+g), Y2 / (1-k-g))
 *   half-size   dX_i = (dY_i + r) / |1-k+-g|,  r = sqrt(k_* <m^2> / (f <m>))
 * The ray grid has cells of side pix_i / sqrt(rho) ("rays per pixel in the
 * absence of lensing", sec. 4) and n_r = ceil(2 dX / Delta) + 1 vertices
 * centred on X; explicit vertex counts span exactly [X - dX, X + dX].
 * The tree's root square is centred on the origin (app. C.1); its half-length
 * is the smallest power of two above every star and ray coordinate, which
 * makes every square's centre and size exact binary fractions.
 */
bool has_psi3(const mlm_lens_params &P) { return P.psi3[0] != 0 || P.psi3[1] != 0 || P.psi3[2] != 0 || P.psi3[3] != 0; }

/*
 * With third-order macro terms (app. D) and no region stated, the images of
 * the map are found by sampling: the macro map (no stars) is evaluated on a
 * LAT x LAT lattice over the star region's bounding box (rays beyond it would
 * meet no microlenses), the lattice points whose images land in the map
 * widened by the border r are kept, and their bounding box widened by one
 * lattice step is shot.  The paper leaves the inversion open (algebraic or
 * perturbative); this one holds for any third-order model, at the cost of
 * shooting the box around all macroimages together.
 */
constexpr int LAT = 2048;

void cubic_region(const mlm_lens_params &P, double ext1, double ext2, double border, const mlm_map_request &q,
                  double &X1, double &X2, double &dX1, double &dX2)
{
    if (!(ext1 > 0) || !(ext2 > 0))
        fail(MLM_EINVAL, "a lens with third-order terms and no stars needs its shooting region stated "
                         "(centre_set, x1c, x2c, dx1, dx2)");
    const double kappa = P.kappa_star + P.kappa_smooth;
    const double lam1 = 1.0 - kappa + P.gamma, lam2 = 1.0 - kappa - P.gamma;
    const double a = P.psi3[0], b = P.psi3[1], c = P.psi3[2], d = P.psi3[3];
    const double lo1 = q.y1c - q.hw1 - border, hi1 = q.y1c + q.hw1 + border;
    const double lo2 = q.y2c - q.hw2 - border, hi2 = q.y2c + q.hw2 + border;
    const double s1 = 2.0 * ext1 / (LAT - 1), s2 = 2.0 * ext2 / (LAT - 1);
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int j = 0; j < LAT; ++j) {
        const double y = -ext2 + j * s2;
        for (int i = 0; i < LAT; ++i) {
            const double x = -ext1 + i * s1;
            const double w1 = lam1 * x - 0.5 * (a * x * x + 2.0 * b * x * y + c * y * y);
            const double w2 = lam2 * y - 0.5 * (b * x * x + 2.0 * c * x * y + d * y * y);
            if (w1 >= lo1 && w1 <= hi1 && w2 >= lo2 && w2 <= hi2) {
                xmin = std::fmin(xmin, x);
                xmax = std::fmax(xmax, x);
                ymin = std::fmin(ymin, y);
                ymax = std::fmax(ymax, y);
            }
        }
    }
    if (xmin > xmax) fail(MLM_ERANGE, "no image of the map inside the star region");
    xmin = std::fmax(xmin - s1, -ext1);
    xmax = std::fmin(xmax + s1, ext1);
    ymin = std::fmax(ymin - s2, -ext2);
    ymax = std::fmin(ymax + s2, ext2);
    X1 = 0.5 * (xmin + xmax);
    X2 = 0.5 * (ymin + ymax);
    dX1 = 0.5 * (xmax - xmin);
    dX2 = 0.5 * (ymax - ymin);
}

void shooting_region(const mlm_lens_params &P, double mean_m, double mean_m2, double ext1, double ext2,
                     const mlm_map_request &q, double &X1, double &X2, double &dX1, double &dX2)
{
    const double kappa = P.kappa_star + P.kappa_smooth;
    const double lam1 = 1.0 - kappa + P.gamma, lam2 = 1.0 - kappa - P.gamma;
    const bool cubic = has_psi3(P);
    const double f = q.flux_fraction > 0 ? q.flux_fraction : 0.01;
    const double border = (mean_m > 0 && P.kappa_star > 0) ? std::sqrt(P.kappa_star * mean_m2 / (f * mean_m)) : 0.0;
    if (q.centre_set) {
        if (!(q.dx1 > 0) || !(q.dx2 > 0) || !std::isfinite(q.x1c) || !std::isfinite(q.x2c))
            fail(MLM_EINVAL, "a stated shooting region needs a finite centre and dx1, dx2 > 0");
        X1 = q.x1c;
        X2 = q.x2c;
        dX1 = q.dx1;
        dX2 = q.dx2;
        return;
    }
    if (cubic) {
        cubic_region(P, ext1, ext2, border, q, X1, X2, dX1, dX2);
        if (q.dx1 > 0) dX1 = q.dx1;
        if (q.dx2 > 0) dX2 = q.dx2;
        return;
    }
    if (std::fabs(lam1) < 1e-9 || std::fabs(lam2) < 1e-9)
        fail(MLM_EDEGENERATE, "|1-kappa+-gamma| = (%g, %g): the shooting region is unbounded", std::fabs(lam1),
             std::fabs(lam2));
    X1 = q.y1c / lam1;
    X2 = q.y2c / lam2;
    dX1 = q.dx1 > 0 ? q.dx1 : (q.hw1 + border) / std::fabs(lam1);
    dX2 = q.dx2 > 0 ? q.dx2 : (q.hw2 + border) / std::fabs(lam2);
}

mlm_status setup_region(const mlm_lens *lens, const mlm_map_request *q, Region *R)
{
    if (!(q->hw1 > 0) || !(q->hw2 > 0) || !std::isfinite(q->hw1) || !std::isfinite(q->hw2) ||
        q->n1 <= 0 || q->n2 <= 0 || !std::isfinite(q->y1c) || !std::isfinite(q->y2c))
        fail(MLM_EINVAL, "map centre/half-widths must be finite, half-widths > 0, pixels >= 1");
    if (!(q->rays_per_pixel >= 0) || !(q->flux_fraction >= 0) || !(q->dx1 >= 0) || !(q->dx2 >= 0))
        fail(MLM_EINVAL, "rays_per_pixel, flux_fraction, dx1, dx2 must be >= 0");
    if ((q->nray1 != 0 || q->nray2 != 0) && (q->nray1 < 2 || q->nray2 < 2))
        fail(MLM_EINVAL, "explicit ray-grid vertex counts must both be >= 2");
    const mlm_lens_params &P = lens->params;
    R->kappa = P.kappa_star + P.kappa_smooth;
    R->lam1 = 1.0 - R->kappa + P.gamma;
    R->lam2 = 1.0 - R->kappa - P.gamma;
    R->mu_macro = 1.0 / (R->lam1 * R->lam2);

    // the sample moments of the lens's own stars
    int64_t n = lens->n;
    R->mean_m = n ? lens->mass_sum / (double)n : 0.0;
    R->mean_m2 = n ? lens->mass2_sum / (double)n : 0.0;
    double f = q->flux_fraction > 0 ? q->flux_fraction : 0.01;
    R->border = (n && P.kappa_star > 0) ? std::sqrt(P.kappa_star * R->mean_m2 / (f * R->mean_m)) : 0.0;
    double ext1 = lens->ext1, ext2 = lens->ext2;
    if (P.sheet == MLM_SHEET_NONE || !(ext1 > 0)) ext1 = ext2 = n ? lens->max_abs : 0.0;
    shooting_region(P, R->mean_m, R->mean_m2, ext1, ext2, *q, R->X1, R->X2, R->dX1, R->dX2);
    R->pix1 = 2.0 * q->hw1 / (double)q->n1;
    R->pix2 = 2.0 * q->hw2 / (double)q->n2;

    if (q->nray1 > 1 && q->nray2 > 1) {
        R->nr1 = q->nray1;
        R->nr2 = q->nray2;
        R->d1 = 2.0 * R->dX1 / (double)(R->nr1 - 1);
        R->d2 = 2.0 * R->dX2 / (double)(R->nr2 - 1);
    } else {
        double rho = q->rays_per_pixel > 0 ? q->rays_per_pixel : 1.0;
        R->d1 = R->pix1 / std::sqrt(rho);
        R->d2 = R->pix2 / std::sqrt(rho);
        double c1 = std::ceil(2.0 * R->dX1 / R->d1), c2 = std::ceil(2.0 * R->dX2 / R->d2);
        if (!(c1 < 2147483000.0) || !(c2 < 2147483000.0))
            fail(MLM_ERANGE, "ray grid of %g x %g vertices is too large", c1 + 1, c2 + 1);
        R->nr1 = (int64_t)c1 + 1;
        R->nr2 = (int64_t)c2 + 1;
    }
    R->x0 = R->X1 - 0.5 * (double)(R->nr1 - 1) * R->d1;
    R->y0 = R->X2 - 0.5 * (double)(R->nr2 - 1) * R->d2;

    double amax = lens->max_abs;
    double e1 = std::fabs(R->X1) + 0.5 * (double)(R->nr1 - 1) * R->d1;
    double e2 = std::fabs(R->X2) + 0.5 * (double)(R->nr2 - 1) * R->d2;
    if (e1 > amax) amax = e1;
    if (e2 > amax) amax = e2;
    int ex;
    std::frexp(amax > 0 ? amax : 1.0, &ex);
    R->L0 = std::ldexp(1.0, ex);
    R->L0_exp = ex + 1;   // L0 = 2^(L0_exp - 1): 2 L0 = 2^L0_exp
    if (!std::isfinite(R->L0)) fail(MLM_ERANGE, "coordinates too large");
    return MLM_OK;
}

/* appendix C.3: smallest integer p with p > log2((<m^2>/<m>) / (L eps)), in [1, 31] */
int auto_order(double mean_m, double mean_m2, double L, double eps)
{
    if (mean_m <= 0) return 1;
    double t = std::log2((mean_m2 / mean_m) / (L * eps));
    int p = (int)std::floor(t) + 1;
    if (p < 1) p = 1;
    if (p > MAX_ORDER) p = MAX_ORDER;
    return p;
}

}  // namespace mlm
