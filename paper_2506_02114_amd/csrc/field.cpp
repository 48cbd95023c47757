// Star fields drawn by the library (sec. 2.1, 3.1): masses from a mass
// function by inverse CDF, positions uniform in the disc or rectangle that
// realises the requested kappa_*.  Host arithmetic only; built with
// -ffp-contract=off like the region set-up.
//
// Random numbers come from the counter-based Philox4x32-10 generator (Salmon,
// Moraes, Dror & Shaw 2011, "Parallel random numbers: as easy as 1, 2, 3"):
// star i's draws are a pure function of (seed, i), so a field is the same
// however it is split or ordered, and any other implementation of the
// published generator reproduces it.
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.hpp"

namespace mlm {

namespace {

constexpr double KROUPA_BREAK = 0.5;
constexpr double SALPETER_SLOPE = 2.35;
constexpr double KROUPA_SLOPE_LO = 1.3, KROUPA_SLOPE_HI = 2.3;

// one Philox4x32 round: two 32 x 32 -> 64-bit products, then the
// published permutation and key mixing
inline void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
}

// uniform in (0, 1) from two 32-bit words: 53 bits, offset by half a step
inline double unit(uint32_t a, uint32_t b)
{
    const uint64_t v = ((uint64_t)(a >> 5) << 26) | (uint64_t)(b >> 6);
    return ((double)v + 0.5) * 0x1.0p-53;
}

// inverse CDF of dN/dm ~ m^-s on [lo, hi] (s != 1)
double powerlaw_icdf(double u, double lo, double hi, double s)
{
    const double e = 1.0 - s;
    const double a = std::pow(lo, e), b = std::pow(hi, e);
    return std::pow(a + u * (b - a), 1.0 / e);
}

// integral of m^(k - s) over [lo, hi] (k - s != -1)
double powerlaw_moment(double lo, double hi, double s, int k)
{
    const double e = (double)k - s + 1.0;
    return (std::pow(hi, e) - std::pow(lo, e)) / e;
}

void check_field(const mlm_field_params &F)
{
    if (!(F.kappa_star > 0) || !std::isfinite(F.kappa_star)) fail(MLM_EINVAL, "kappa_star must be finite and > 0");
    if (F.shape != MLM_SHEET_CIRCLE && F.shape != MLM_SHEET_RECT) fail(MLM_EINVAL, "unknown field shape %d", F.shape);
    switch (F.mass_fn) {
    case MLM_MASS_EQUAL:
        if (!(F.m_equal > 0) || !std::isfinite(F.m_equal)) fail(MLM_EINVAL, "m_equal must be finite and > 0");
        break;
    case MLM_MASS_SALPETER:
        if (!(F.m_lo > 0) || !(F.m_hi > F.m_lo) || !std::isfinite(F.m_hi))
            fail(MLM_EINVAL, "the Salpeter mass function needs 0 < m_lo < m_hi");
        break;
    case MLM_MASS_KROUPA:
        if (!(F.m_lo > 0) || !(F.m_lo < KROUPA_BREAK) || !(F.m_hi > KROUPA_BREAK) || !std::isfinite(F.m_hi))
            fail(MLM_EINVAL, "the Kroupa mass function needs 0 < m_lo < 0.5 < m_hi");
        break;
    default: fail(MLM_EINVAL, "unknown mass function %d", F.mass_fn);
    }
    if (F.n_stars < 0) fail(MLM_EINVAL, "n_stars must be >= 0");
    if (F.n_stars == 0) {
        if (!(F.extent1 > 0) || !std::isfinite(F.extent1) ||
            (F.shape == MLM_SHEET_RECT && (!(F.extent2 > 0) || !std::isfinite(F.extent2))))
            fail(MLM_EINVAL, "n_stars = 0 needs the region's extent (disc radius, or both rectangle half-sides)");
    }
    if (F.shape == MLM_SHEET_RECT && F.n_stars > 0 && !(F.rect_aspect > 0))
        fail(MLM_EINVAL, "a rectangle of n_stars stars needs rect_aspect > 0");
    if (!(F.rect_aspect >= 0) || !std::isfinite(F.rect_aspect)) fail(MLM_EINVAL, "rect_aspect must be finite and >= 0");
}

// Kroupa: density m^-1.3 below the break, 0.5^(2.3 - 1.3) m^-2.3 above
// (continuous there); weights of the two pieces
void kroupa_weights(double lo, double hi, double &w1, double &w2)
{
    w1 = powerlaw_moment(lo, KROUPA_BREAK, KROUPA_SLOPE_LO, 0);
    w2 = std::pow(KROUPA_BREAK, KROUPA_SLOPE_HI - KROUPA_SLOPE_LO) * powerlaw_moment(KROUPA_BREAK, hi, KROUPA_SLOPE_HI, 0);
}

double draw_mass(const mlm_field_params &F, double u)
{
    switch (F.mass_fn) {
    case MLM_MASS_SALPETER: return powerlaw_icdf(u, F.m_lo, F.m_hi, SALPETER_SLOPE);
    case MLM_MASS_KROUPA: {
        double w1, w2;
        kroupa_weights(F.m_lo, F.m_hi, w1, w2);
        const double p1 = w1 / (w1 + w2);
        if (u < p1) return powerlaw_icdf(u / p1, F.m_lo, KROUPA_BREAK, KROUPA_SLOPE_LO);
        return powerlaw_icdf((u - p1) / (1.0 - p1), KROUPA_BREAK, F.m_hi, KROUPA_SLOPE_HI);
    }
    default: return F.m_equal;
    }
}

// the words of star i's block `blk` of draws
inline void star_block(uint64_t seed, int64_t i, uint32_t blk, uint32_t out[4])
{
    const uint32_t ctr[4] = {(uint32_t)(uint64_t)i, (uint32_t)((uint64_t)i >> 32), blk, 0u};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    mlm_philox4x32_10(ctr, key, out);
}

}  // namespace

void field_moments(const mlm_field_params &F, double &mean_m, double &mean_m2)
{
    switch (F.mass_fn) {
    case MLM_MASS_SALPETER: {
        const double z = powerlaw_moment(F.m_lo, F.m_hi, SALPETER_SLOPE, 0);
        mean_m = powerlaw_moment(F.m_lo, F.m_hi, SALPETER_SLOPE, 1) / z;
        mean_m2 = powerlaw_moment(F.m_lo, F.m_hi, SALPETER_SLOPE, 2) / z;
        return;
    }
    case MLM_MASS_KROUPA: {
        double w1, w2;
        kroupa_weights(F.m_lo, F.m_hi, w1, w2);
        const double c = std::pow(KROUPA_BREAK, KROUPA_SLOPE_HI - KROUPA_SLOPE_LO);
        mean_m = (powerlaw_moment(F.m_lo, KROUPA_BREAK, KROUPA_SLOPE_LO, 1) +
                  c * powerlaw_moment(KROUPA_BREAK, F.m_hi, KROUPA_SLOPE_HI, 1)) / (w1 + w2);
        mean_m2 = (powerlaw_moment(F.m_lo, KROUPA_BREAK, KROUPA_SLOPE_LO, 2) +
                   c * powerlaw_moment(KROUPA_BREAK, F.m_hi, KROUPA_SLOPE_HI, 2)) / (w1 + w2);
        return;
    }
    default:
        mean_m = F.m_equal;
        mean_m2 = F.m_equal * F.m_equal;
    }
}

// kappa_* = pi N <m> / A (sec. 2.1, theta_* = 1): the count that fills the
// given region on average
int64_t field_count(const mlm_field_params &F)
{
    check_field(F);
    if (F.n_stars > 0) return F.n_stars;
    double mm, mm2;
    field_moments(F, mm, mm2);
    const double area = F.shape == MLM_SHEET_RECT ? 4.0 * F.extent1 * F.extent2 : M_PI * F.extent1 * F.extent1;
    const double n = std::round(F.kappa_star * area / (M_PI * mm));
    if (!(n < 1e9)) fail(MLM_ERANGE, "the region holds %g stars", n);
    return (int64_t)n;
}

// the star region that realises kappa_* exactly for a total mass: the disc
// R_* = sqrt(sum m / kappa_*) (its sheet, sec. 3.1), or the rectangle of
// aspect c2 / c1 with 4 c1 c2 = pi sum m / kappa_* (app. B)
void field_extent(int shape, double kappa_star, double mass_sum, double aspect, double &e1, double &e2)
{
    if (shape == MLM_SHEET_RECT) {
        e1 = std::sqrt(M_PI * mass_sum / (4.0 * kappa_star * aspect));
        e2 = aspect * e1;
    } else {
        e1 = e2 = std::sqrt(mass_sum / kappa_star);
    }
}

int64_t field_sample(const mlm_field_params &F, std::vector<double> &x, std::vector<double> &y,
                     std::vector<double> &m, double &e1, double &e2)
{
    const int64_t n = field_count(F);
    x.assign(n, 0.0);
    y.assign(n, 0.0);
    m.assign(n, 0.0);
    double msum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        uint32_t w[4];
        star_block(F.seed, i, 0u, w);
        m[i] = draw_mass(F, unit(w[0], w[1]));
        msum += m[i];
    }
    const double aspect = F.rect_aspect > 0 ? F.rect_aspect : (F.shape == MLM_SHEET_RECT ? F.extent2 / F.extent1 : 1.0);
    field_extent(F.shape, F.kappa_star, msum, aspect, e1, e2);
    for (int64_t i = 0; i < n; ++i) {
        uint32_t a[4], b[4];
        star_block(F.seed, i, 0u, a);
        star_block(F.seed, i, 1u, b);
        const double u = unit(a[2], a[3]), v = unit(b[0], b[1]);
        if (F.shape == MLM_SHEET_RECT) {
            x[i] = e1 * (2.0 * u - 1.0);
            y[i] = e2 * (2.0 * v - 1.0);
        } else {
            const double r = e1 * std::sqrt(u), phi = 2.0 * M_PI * v;
            x[i] = r * std::cos(phi);
            y[i] = r * std::sin(phi);
        }
    }
    return n;
}

}  // namespace mlm

using namespace mlm;

extern "C" {

void mlm_philox4x32_10(const uint32_t counter[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {counter[0], counter[1], counter[2], counter[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    std::memcpy(out, c, sizeof c);
}

void mlm_field_params_init(mlm_field_params *f)
{
    if (!f) return;
    std::memset(f, 0, sizeof *f);
    f->mass_fn = MLM_MASS_EQUAL;
    f->shape = MLM_SHEET_CIRCLE;
    f->m_equal = 1.0;
    f->m_lo = 0.1;
    f->m_hi = 1.0;
}

}  // extern "C"
