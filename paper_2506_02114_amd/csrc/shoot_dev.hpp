// Device code shared by the kernels that shoot rays: grid positions, the
// leaf containing a point, and the deflection from a leaf's tables
// (sec. 2.2, app. C).
#pragma once

#include "dev.hpp"

namespace mlm {

// grid coordinate of vertex a: x0 + a d, evaluated as written (no fused multiply-add)
__device__ inline double grid_pos(double x0, double d, int64_t a)
{
#pragma clang fp contract(off)
    return x0 + (double)a * d;
}

// point a of a lattice offset by h cells: x0 + (a + h) d (h = 0: the grid's
// vertices, the same value as grid_pos; h = 1/2: the centres of its cells)
__device__ inline double grid_pos(double x0, double d, int64_t a, double h)
{
#pragma clang fp contract(off)
    return x0 + ((double)a + h) * d;
}

// Inverse ray shooting: a ray landing at uv (pixel units) counts once in the
// pixel (floor u, floor v) if that lies in the map.  Lanes of a wavefront
// that land in the same pixel are added together first (one device atomic
// per distinct pixel: neighbouring rays mostly share a pixel).
__device__ inline void irs_count(bool valid, double2 uv, const MapGeom &g, unsigned long long *__restrict__ counts)
{
    const double fu = floor(uv.x), fv = floor(uv.y);
    const bool in = valid && fu >= 0.0 && fv >= 0.0 && fu < (double)g.n1 && fv < (double)g.n2;
    const long long key = in ? (long long)fv * g.n1 + (long long)fu : -1;
    const int lane = threadIdx.x & 63;
    unsigned long long active = __ballot(in);
    while (active) {
        const int leader = __ffsll(active) - 1;
        const long long lk = __shfl(key, leader, 64);
        const unsigned long long same = __ballot(key == lk);
        if (lane == leader) atomicAdd(counts + lk, (unsigned long long)__popcll(same));
        active &= ~same;
    }
}

// square index of t at level lev (root [-L0, L0)), clamped like the star keys
__device__ inline int64_t level_cell(double t, double L0, double scale_lev, int lev)
{
    double u = floor((t + L0) * scale_lev);
    double top = (double)((1ll << lev) - 1);
    u = u < 0.0 ? 0.0 : (u > top ? top : u);
    return (int64_t)u;
}

// t log t for t = (a, b), principal branch (cut along the negative real axis)
__device__ inline double2 t_log_t(double a, double b)
{
    const double lr = 0.5 * log(a * a + b * b), th = atan2(b, a);
    return make_double2(a * lr - b * th, b * lr + a * th);
}

// deflection of a sheet of convergence -k_* over the rectangle
// [-c1, c1] x [-c2, c2] (app. B): with c = c1 + i c2,
//   a_s = (-k_* i / pi) [ (c - zb) log(c - zb) - (cb - zb) log(cb - zb)
//                         + (-c - zb) log(-c - zb) - (-cb - zb) log(-cb - zb) ]
//         - k_* (2 c1 + 2 x)  inside the rectangle
//         - k_* 4 c1          for x >= c1, |y| <= c2
// (the last two undo the branch cuts the logarithms cross)
__device__ inline void rect_sheet(double x, double y, double ks, double c1, double c2, double &ax, double &ay)
{
    const double2 t1 = t_log_t(c1 - x, c2 + y);     // c - zb
    const double2 t2 = t_log_t(c1 - x, y - c2);     // cb - zb
    const double2 t3 = t_log_t(-c1 - x, y - c2);    // -c - zb
    const double2 t4 = t_log_t(-c1 - x, c2 + y);    // -cb - zb
    const double sr = t1.x - t2.x + t3.x - t4.x, si = t1.y - t2.y + t3.y - t4.y;
    const double k = ks * (1.0 / M_PI);
    ax = k * si;
    ay = -k * sr;
    const bool in_band = fabs(y) <= c2;
    if (in_band && fabs(x) <= c1) ax -= ks * (2.0 * c1 + 2.0 * x);
    if (in_band && x >= c1) ax -= ks * (4.0 * c1);
}

__device__ inline void finish_vertex(const LensConst &lc, const MapGeom &g, double x, double y, double ax,
                                     double ay, double &w1, double &w2, double2 &uv)
{
    // macro model, with its third-order term when the lens has one (app. D):
    // the gradient of (1/6) sum psi_ijk x_i x_j x_k
    w1 = lc.lam1 * x - ax;
    w2 = lc.lam2 * y - ay;
    if (lc.cubic) {
        const double a = lc.psi3[0], b = lc.psi3[1], c = lc.psi3[2], d = lc.psi3[3];
        w1 -= 0.5 * (a * x * x + 2.0 * b * x * y + c * y * y);
        w2 -= 0.5 * (b * x * x + 2.0 * c * x * y + d * y * y);
    }
    if (lc.sheet == 1) {
        // circular sheet: a_s = -k_* z inside R_*, -k_* R_*^2 / conj(z) outside
        double r2 = x * x + y * y;
        double f = (r2 <= lc.r_star2) ? lc.kappa_star : lc.kappa_star * lc.r_star2 / r2;
        w1 += f * x;
        w2 += f * y;
    } else if (lc.sheet == 2) {
        double sx, sy;
        rect_sheet(x, y, lc.kappa_star, lc.c1, lc.c2, sx, sy);
        w1 -= sx;
        w2 -= sy;
    }
    uv = make_double2((w1 - g.ylo1) / g.pix1, (w2 - g.ylo2) / g.pix2);
}

// far field at offset (dx, dy) from a leaf's centre, added to the near field
// (ax, ay) already summed in type R: conj( sum_{l<p} deriv_l zeta^l ), Horner.
// In FP32 the Taylor series is split: its value at the centre (the field of
// every far star, as large as kappa_* |z|) is the leaf's FP64 f0, and FP32
// carries only the variation across the leaf, zeta sum_{l>=1} d_l zeta^(l-1),
// which is of the size of the field's derivative times the leaf's half-length
template <class R>
__device__ inline void far_field(double dx, double dy, const LeafInfo &li, const typename Cx<R>::c2 *dv, int p, R ax,
                                 R ay, double &ax_out, double &ay_out)
{
    const R zr = (R)(dx * li.invL), zi = (R)(dy * li.invL);
    if constexpr (sizeof(R) == sizeof(double)) {
        R sr = dv[p - 1].x, si = dv[p - 1].y;
#pragma unroll 8
        for (int l = p - 2; l >= 0; --l) {
            const typename Cx<R>::c2 c = dv[l];
            const R nr = sr * zr - si * zi + c.x;
            const R ni = sr * zi + si * zr + c.y;
            sr = nr;
            si = ni;
        }
        ax_out = (double)ax + (double)sr;
        ay_out = (double)ay - (double)si;
    } else {
        R vr = 0, vi = 0;   // zeta sum_{l>=1} d_l zeta^(l-1)
        if (p >= 2) {
            R sr = dv[p - 1].x, si = dv[p - 1].y;
#pragma unroll 8
            for (int l = p - 2; l >= 1; --l) {
                const typename Cx<R>::c2 c = dv[l];
                const R nr = sr * zr - si * zi + c.x;
                const R ni = sr * zi + si * zr + c.y;
                sr = nr;
                si = ni;
            }
            vr = sr * zr - si * zi;
            vi = sr * zi + si * zr;
        }
        ax_out = (double)ax + (li.f0x + (double)vr);
        ay_out = (double)ay - (li.f0y + (double)vi);
    }
}

// near field of one star: a_* += m (z - z_i) / |z - z_i|^2, the offset from
// the star formed in FP64 (a ray may pass very close to a star)
template <class R>
__device__ inline void near_star(double dx, double dy, const double4 &st, R &ax, R &ay)
{
    const R ex = (R)(dx - st.x), ey = (R)(dy - st.y);
    const R f = near_div((R)st.z, ex * ex + ey * ey);
    ax += f * ex;
    ay += f * ey;
}

// far-field and near-field deflection at offset (dx, dy) from a leaf's
// centre, in arithmetic type R
template <class R>
__device__ inline void leaf_alpha(double dx, double dy, const LeafInfo &li, const double4 *__restrict__ ns,
                                  const typename Cx<R>::c2 *__restrict__ dv, int p, double &ax_out, double &ay_out)
{
    R ax = 0, ay = 0;
    // unrolled so that several of the wavefront-uniform (scalar) loads are in
    // flight before the first is needed
#pragma unroll 4
    for (int32_t s = 0; s < li.near_cnt; ++s) near_star<R>(dx, dy, ns[s], ax, ay);
    far_field<R>(dx, dy, li, dv, p, ax, ay, ax_out, ay_out);
}

// LDS of a wavefront whose rays all lie in one leaf: the leaf's near stars,
// 64 at a time, and its Taylor coefficients
template <class R> struct LeafLds {
    double4 star[64];
    typename Cx<R>::c2 d[MAX_ORDER + 1];
};

// leaf_alpha for a workgroup of one wavefront whose rays share the leaf: the
// lanes load the leaf's near stars (64 at a time) and coefficients into LDS
// together, so the wavefront waits on memory once per 64 stars instead of
// once per few stars through the scalar cache; the same arithmetic in the
// same order
template <class R>
__device__ inline void leaf_alpha_tile(double dx, double dy, const LeafInfo &li, const double4 *__restrict__ ns,
                                       const typename Cx<R>::c2 *__restrict__ dv, int p, double &ax_out,
                                       double &ay_out, LeafLds<R> &S)
{
    const int lane = (int)threadIdx.x & 63;
    if (lane < p) S.d[lane] = dv[lane];
    R ax = 0, ay = 0;
    for (int32_t base = 0; base < li.near_cnt; base += 64) {
        const int32_t n = min(64, li.near_cnt - base);
        if (lane < n) S.star[lane] = ns[base + lane];
        __syncthreads();
#pragma unroll 2
        for (int32_t s = 0; s < n; ++s) near_star<R>(dx, dy, S.star[s], ax, ay);
        __syncthreads();   // the next 64 overwrite the stars
    }
    __syncthreads();       // the coefficients, when the leaf has no near star
    far_field<R>(dx, dy, li, S.d, p, ax, ay, ax_out, ay_out);
}

// leaf containing (x, y): down from the root through the children, the
// quadrant of (x, y) one level down picking one (a divided node has all four,
// at child0 + quadrant in Morton order), squares clamped to the root like the
// star keys; -1 if the point lies in no leaf of the tree
__device__ inline int64_t find_leaf(double x, double y, int nlevels, double L0, int L0_exp,
                                    const int32_t *__restrict__ child0, const int32_t *__restrict__ leaf,
                                    const int32_t *__restrict__ node_leaf)
{
    int64_t node = 0;
    for (int lev = 0; lev < nlevels; ++lev) {
        if (leaf[node]) return node_leaf[node];
        const int32_t c0 = child0[node];
        if (c0 < 0) return -1;
        const double scale = ldexp(1.0, lev + 1 - L0_exp);
        const int64_t i = level_cell(x, L0, scale, lev + 1), j = level_cell(y, L0, scale, lev + 1);
        node = (int64_t)c0 + ((i & 1) | ((j & 1) << 1));
    }
    return -1;
}

}  // namespace mlm
