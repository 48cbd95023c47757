// Inverse polygon mapping (sec. 3.2): every grid cell is split into two
// triangles; each mapped triangle's image-plane area is apportioned among the
// source pixels it covers, in proportion to (triangle n pixel) / triangle.
//
// Pixel areas come from closed forms instead of explicit polygon clipping:
// inside a strip of pixel rows (or columns) the triangle's area on one side of
// a line across the strip is a sum over its edges clipped to the strip of
// (signed extent) x (integral of a clamped linear function), and the area of
// a pixel is the difference of two such sums.
//
// A triangle inside one pixel is one deposit; one inside a 2 x 2 pixel box
// is apportioned in place from the areas of the corner triangles that the
// pixel lines cut off; other ordinary triangles go by pixel columns, one work
// item per (triangle, column).  Triangles next to a star map to huge
// triangles (the linear interpolation of a singular mapping), covering up to
// millions of pixels; their cost is made proportional to their perimeter:
// they are binned by bands of pixel rows and apportioned through per-row
// column differences.
//
// Every geometric helper is templated on its arithmetic type R: FP64, or FP32
// in the mixed-precision mode, where coordinates are first made local to the
// triangle in FP64 and the sums are kept in FP64.
#include <algorithm>

#include "colarea.hpp"
#include "dev.hpp"

namespace mlm {

namespace {

// Part of segment P->Q with lo <= coordinate <= hi (AXIS 0: u, 1: v).  The
// segment lies on a line whose other coordinate changes by `slope` per unit of
// the clipping coordinate, so a crossing is one multiply-add.
template <int AXIS, class R>
__device__ inline bool clip_seg(Pt<R> P, Pt<R> Q, R lo, R hi, R slope, Pt<R> &E, Pt<R> &X)
{
    const R p = AXIS ? P.v : P.u, q = AXIS ? Q.v : Q.u;
    const R po = AXIS ? P.u : P.v;
    auto at = [&](R c) { return AXIS ? Pt<R>{po + (c - p) * slope, c} : Pt<R>{c, po + (c - p) * slope}; };
    if (p == q) {
        if (p < lo || p > hi) return false;
        E = P;
        X = Q;
        return true;
    }
    if (q > p) {
        if (q < lo || p > hi) return false;
        E = p < lo ? at(lo) : P;
        X = q > hi ? at(hi) : Q;
    } else {
        if (p < lo || q > hi) return false;
        E = p > hi ? at(hi) : P;
        X = q < lo ? at(lo) : Q;
    }
    return true;
}

// integral over t in [0, 1] of max(ua + t (ub - ua), 0); inv = 1 / |ub - ua|
// (unused when ua and ub have the same sign)
template <class R>
__device__ inline R clamp_integral(R ua, R ub, R inv)
{
    const R m = fmax(ua, ub);
    const R cross = R(0.5) * m * m * inv;
    return (ua >= R(0) && ub >= R(0)) ? R(0.5) * (ua + ub) : ((ua <= R(0) && ub <= R(0)) ? R(0) : cross);
}

// Pixel areas from the triangle's edges clipped to one strip.  For a strip of
// pixel rows [v0, v0 + 1] and a polygon traversed counter-clockwise, the area
// left of the line u = c is  G(c) = -sum_e dv_e * I(c - ua_e, c - ub_e), I the
// clamp integral above; for a strip of columns and the line v = r, the area
// below it is  H(r) = sum_e du_e * I(r - va_e, r - vb_e).  A pixel's area is
// then a difference of two such sums.  (Clockwise triangles give the negated
// area, matching the sign of their signed area.)
template <class R> struct SegsT {
    R a[3], b[3];       // coordinate across the strip at both ends (u for rows, v for columns)
    R d[3];             // signed extent along the strip (dv for rows, du for columns)
    R inv[3];           // 1 / |b - a| (0 if equal)
};
using Segs = SegsT<double>;

template <int AXIS, class R>
__device__ inline void strip_segments(const Pt<R> (&T)[3], const R (&slope)[3], R lo, R hi, SegsT<R> &S)
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        Pt<R> E, X;
        if (clip_seg<AXIS>(T[k], T[(k + 1) % 3], lo, hi, slope[k], E, X)) {
            S.a[k] = AXIS ? E.u : E.v;
            S.b[k] = AXIS ? X.u : X.v;
            S.d[k] = AXIS ? X.v - E.v : X.u - E.u;
        } else {
            S.a[k] = S.b[k] = S.d[k] = R(0);
        }
        const R w = fabs(S.b[k] - S.a[k]);
        S.inv[k] = w > R(0) ? qdiv(R(1), w) : R(0);
    }
}

// sum_e d_e * I(c - a_e, c - b_e)
template <class R>
__device__ inline R strip_cumulative(const SegsT<R> &S, R c)
{
    R s = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) s += S.d[k] * clamp_integral(c - S.a[k], c - S.b[k], S.inv[k]);
    return s;
}

// Largest ratio of squared extent to twice the area that the FP32 geometry
// of the mixed mode accepts: its relative area error is about FP32's unit
// round-off times this ratio (below 2e-5 here).  Thinner triangles, the ones
// folded across a caustic, are apportioned in FP64.
constexpr double MIXED_MAX_COND = 256.0;

__device__ inline void deposit(double *map, const MapGeom &g, int i, int j, double val)
{
    // the map is global memory (also when its pointer was read from a batch
    // descriptor, where the compiler could not tell): a global, not a flat, atomic
    auto *gm = (__attribute__((address_space(1))) double *)map;
    __hip_atomic_fetch_add(gm + (int64_t)j * g.n1 + i, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// pixel window of a workgroup in LDS: deposits inside it are summed there and
// added to the map once per pixel at the end; the rest go straight to the map.
// Its side N is 48 pixels (wide enough for most tiles' images at a few cells
// per pixel; 18 KiB, so more cell-pass workgroups share a CU with the band
// pass beside it than at 64), or 16 where a tile's cells cover far less than
// a pixel each (a highly magnified map), so that clearing and flushing the
// window does not cost more than the tile's deposits.
constexpr int WIN = 48;        // window side in pixels (WIN x WIN doubles)
constexpr int WIN_FINE = 16;   // the side for maps of many cells per pixel

template <int N> struct Window {
    double *acc;          // N x N, row-major
    int i0, j0;           // map pixel of acc[0]
};

template <int N>
__device__ inline void deposit_w(const Window<N> &w, double *map, const MapGeom &g, int i, int j, double val)
{
    const int di = i - w.i0, dj = j - w.j0;
    if ((unsigned)di < (unsigned)N && (unsigned)dj < (unsigned)N)
        // workgroup scope: kept apart from the device-scope map deposit, so the
        // two are not merged into one generic (flat) atomic and this one stays
        // an LDS atomic
        __hip_atomic_fetch_add(w.acc + dj * N + di, val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    else
        deposit(map, g, i, j, val);
}

// Classification of one mapped triangle (pixel coordinates) for the cell pass.
//   kind 0: nothing to deposit (outside the map, or skipped as non-finite)
//   kind 1: one deposit (single pixel, or zero area -> its centroid's pixel)
//   kind 2: within a 2 x 2 pixel box (`small`), apportioned in place; else
//           `cols` pixel columns, each one work item of the column pass
//   kind 3: large: goes to the row-parallel pass
struct TriClass {
    int kind;
    int cols;
    bool small;           // kind 2 within a 2 x 2 pixel box: apportioned in place, no work items
    int i0;               // first column inside the map
    int pi, pj;           // pixel of a kind-1 deposit (or -1: outside)
};

// twice the signed area of (A, B, C) in coordinates relative to (ou, ov),
// evaluated as written so every kernel gets the same value
__device__ inline double twice_area(P2 A, P2 B, P2 C, double ou, double ov)
{
#pragma clang fp contract(off)
    const double au = A.u - ou, av = A.v - ov;
    return ((B.u - ou) - au) * ((C.v - ov) - av) - ((C.u - ou) - au) * ((B.v - ov) - av);
}

__device__ inline TriClass classify(P2 A, P2 B, P2 C, const MapGeom &g)
{
    TriClass c{0, 0, false, 0, -1, -1};
    if (!(isfinite(A.u) && isfinite(A.v) && isfinite(B.u) && isfinite(B.v) && isfinite(C.u) && isfinite(C.v)))
        return c;
    const double umin = fmin(A.u, fmin(B.u, C.u)), umax = fmax(A.u, fmax(B.u, C.u));
    const double vmin = fmin(A.v, fmin(B.v, C.v)), vmax = fmax(A.v, fmax(B.v, C.v));
    const double fu0 = floor(umin), fu1 = floor(umax), fv0 = floor(vmin), fv1 = floor(vmax);
    if (fu1 < 0.0 || fv1 < 0.0 || fu0 > (double)(g.n1 - 1) || fv0 > (double)(g.n2 - 1)) return c;
    if (fu0 == fu1 && fv0 == fv1) {
        c.kind = 1;
        c.pi = (int)fu0;
        c.pj = (int)fv0;
        return c;
    }
    if (twice_area(A, B, C, fu0, fv0) == 0.0) {
        // no source-plane area: the whole image area goes to the centroid's pixel
        const double fi = floor((A.u + B.u + C.u) / 3.0), fj = floor((A.v + B.v + C.v) / 3.0);
        c.kind = 1;
        if (fi >= 0.0 && fj >= 0.0 && fi <= (double)(g.n1 - 1) && fj <= (double)(g.n2 - 1)) {
            c.pi = (int)fi;
            c.pj = (int)fj;
        }
        return c;
    }
    const int i0 = (int)fmax(fu0, 0.0), i1 = (int)fmin(fu1, (double)(g.n1 - 1));
    const int j0 = (int)fmax(fv0, 0.0), j1 = (int)fmin(fv1, (double)(g.n2 - 1));
    if ((int64_t)(i1 - i0 + 1) * (j1 - j0 + 1) > (int64_t)g.big_px) {   // large: by row bands
        c.kind = 3;
        return c;
    }
    c.kind = 2;
    c.cols = (int)(i1 - i0 + 1);
    c.small = fu1 - fu0 <= 1.0 && fv1 - fv0 <= 1.0;
    c.i0 = i0;
    return c;
}

// Area (signed like S, the triangle's signed area) of the part of a triangle
// with coordinates a, b, c along one axis that lies below the line x = 1.  A
// line leaving one vertex x0 alone on its side cuts off the corner triangle at
// that vertex; along each edge from x0 the line sits at the fraction
// t = (1 - x0) / (x - x0), so the corner's area is S t1 t2.
__device__ inline double part_below(double a, double b, double c, double S)
{
    const bool la = a < 1.0, lb = b < 1.0, lc = c < 1.0;
    const int n = (int)la + (int)lb + (int)lc;
    const bool split = n == 1 || n == 2;
    const double x0 = lb == lc ? a : (la == lc ? b : c);   // the lone vertex
    const double x1 = lb == lc ? b : (la == lc ? c : a);
    const double x2 = lb == lc ? c : (la == lc ? a : b);
    const double den = split ? (x1 - x0) * (x2 - x0) : 1.0;
    const double corner = S * ((1.0 - x0) * (1.0 - x0) / den);
    return n == 0 ? 0.0 : (n == 3 ? S : (n == 1 ? corner : S - corner));
}

template <int N>
__device__ inline void put_pixel(const Window<N> &w, double *map, const MapGeom &g, int i, int j, double val)
{
    if (val != 0.0 && i >= 0 && j >= 0 && i < g.n1 && j < g.n2) deposit_w(w, map, g, i, j, val);
}

// A triangle inside a 2 x 2 pixel box (first pixel (fu0, fv0)), apportioned
// in place: with local coordinates at most the lines u = 1 and v = 1 cross
// it, and its four pieces follow from the part left of u = 1 (GL), the part
// below v = 1 (HB) and the part in both (Q).  Q is the corner triangle that
// u = 1 cuts off, clipped below v = 1 (or HB minus it, when the corner is the
// right-hand part).  Local coordinates are exact: a double minus a nearby
// integer.
template <int N>
__device__ inline void small_triangle(P2 A, P2 B, P2 C, double fu0, double fv0, const MapGeom &g, double *map,
                                      const Window<N> &w)
{
    const P2 a{A.u - fu0, A.v - fv0}, b{B.u - fu0, B.v - fv0}, c{C.u - fu0, C.v - fv0};
    const double S = 0.5 * twice_area(A, B, C, fu0, fv0);   // never 0: those go to one pixel
    const double inv = g.tri_weight / S;
    const bool cu = fmax(a.u, fmax(b.u, c.u)) >= 1.0, cv = fmax(a.v, fmax(b.v, c.v)) >= 1.0;
    const double HB = cv ? part_below(a.v, b.v, c.v, S) : S;
    double GL = S, Q = HB;
    if (cu) {
        const bool la = a.u < 1.0, lb = b.u < 1.0, lc = c.u < 1.0;
        const P2 p0 = lb == lc ? a : (la == lc ? b : c);   // alone on its side of u = 1
        const P2 p1 = lb == lc ? b : (la == lc ? c : a);
        const P2 p2 = lb == lc ? c : (la == lc ? a : b);
        const double t1 = (1.0 - p0.u) / (p1.u - p0.u), t2 = (1.0 - p0.u) / (p2.u - p0.u);
        const double corner = S * t1 * t2;
        const bool left = p0.u < 1.0;
        GL = left ? corner : S - corner;
        Q = GL;
        if (cv) {
            const double q = part_below(p0.v, p0.v + t1 * (p1.v - p0.v), p0.v + t2 * (p2.v - p0.v), corner);
            Q = left ? q : HB - q;
        }
    }
    const int i = (int)fu0, j = (int)fv0;   // at least -1: the box meets the map
    put_pixel(w, map, g, i, j, Q * inv);
    if (cu) put_pixel(w, map, g, i + 1, j, (HB - Q) * inv);
    if (cv) put_pixel(w, map, g, i, j + 1, (GL - Q) * inv);
    if (cu && cv) put_pixel(w, map, g, i + 1, j + 1, ((S - GL) - (HB - Q)) * inv);
}

// the corners of the cell in column a of vertex row r (counted in `verts`);
// the vertices are global memory (also when their pointer was read from a
// batch descriptor)
__device__ inline void load_cell_at(const double2 *verts, int64_t nr1, int64_t r, int64_t a, P2 &v00, P2 &v10,
                                    P2 &v11, P2 &v01)
{
    using GD = const __attribute__((address_space(1))) double;
    GD *r0 = (GD *)verts + 2 * (r * nr1 + a), *r1 = r0 + 2 * nr1;
    v00 = P2{r0[0], r0[1]};
    v10 = P2{r0[2], r0[3]};
    v11 = P2{r1[2], r1[3]};
    v01 = P2{r1[0], r1[1]};
}

__device__ inline bool cell_in_one_pixel(P2 v00, P2 v10, P2 v11, P2 v01, const MapGeom &g, int &pi, int &pj)
{
    const double fu = floor(v00.u), fv = floor(v00.v);
    if (!(floor(v10.u) == fu && floor(v11.u) == fu && floor(v01.u) == fu && floor(v10.v) == fv &&
          floor(v11.v) == fv && floor(v01.v) == fv))
        return false;
    pi = pj = -1;
    if (fu >= 0.0 && fv >= 0.0 && fu <= (double)(g.n1 - 1) && fv <= (double)(g.n2 - 1)) {
        pi = (int)fu;
        pj = (int)fv;
    }
    return true;
}

// pixel pieces of one column of a triangle: T in coordinates local to the
// integer point (fu0, fv0) (formed in FP64), cl = column - fu0; each piece is
// a difference of the column's cumulative edge sum H at two row lines
template <class R, int N>
__device__ inline int column_pieces(const P2 (&Td)[3], const double (&svd)[3], const double (&sud)[3], double cl, double fv0, int i, int j0, int j1,
                                     double scale, const MapGeom &g, double *map, const Window<N> &w)
{
    const Pt<R> T[3] = {Pt<R>{(R)Td[0].u, (R)Td[0].v}, Pt<R>{(R)Td[1].u, (R)Td[1].v}, Pt<R>{(R)Td[2].u, (R)Td[2].v}};
    const R sv[3] = {(R)svd[0], (R)svd[1], (R)svd[2]};
    const R su[3] = {(R)sud[0], (R)sud[1], (R)sud[2]};
    ColSegs<R> S;
    col_segments(T, sv, su, (R)cl, (R)(cl + 1.0), S);
    const R big = sizeof(R) == 4 ? R(3e38f) : R(1e300);
    R cvmin = big, cvmax = -big;
    col_range(S.e0, cvmin, cvmax);
    col_range(S.e1, cvmin, cvmax);
    col_range(S.e2, cvmin, cvmax);
    if (cvmin > cvmax) return 0;
    // area below v = r inside the column; a piece is the difference of two
    // rows of the column's pieces, clamped to the triangle's in-map rows
    const int ja = (int)fmin(fmax(floor((double)cvmin) + fv0, (double)j0), (double)j1 + 1.0);
    const int jb = (int)fmax(fmin(floor((double)cvmax) + fv0, (double)j1), (double)j0 - 1.0);
    R rj = (R)((double)ja - fv0);   // row line j local to fv0 (an integer: exact, also in FP32)
    R h0 = col_cumulative(S, rj);
    for (int j = ja; j <= jb; ++j) {
        rj += R(1);
        const R h1 = col_cumulative(S, rj);
        const double a2 = 2.0 * ((double)h1 - (double)h0);   // twice the piece area, signed like the triangle
        h0 = h1;
        if (a2 != 0.0) deposit_w(w, map, g, i, j, scale * a2);
    }
    return jb >= ja ? jb - ja + 1 : 0;
}

// What a pixel column of a medium triangle needs, computed once per triangle
// by the thread that classified it and read by the threads that take its
// columns (through cross-lane reads, so no cell is loaded twice).
struct ColSetup {
    P2 T[3];              // vertices local to (fu0, fv0)
    double sv[3];         // edge slopes dv/du
    double su[3];         // and du/dv
    double scale;         // tri_weight / (twice the signed area)
    double fu0, fv0;      // floor of the box's lower-left corner
    int i0, j0, j1;       // first in-map column; in-map rows
    int fp32;             // mixed mode: conditioned well enough for FP32 geometry
};

__device__ inline ColSetup col_setup(P2 A, P2 B, P2 C, int i0, const MapGeom &g, bool mixed)
{
    ColSetup c;
    const double umin = fmin(A.u, fmin(B.u, C.u)), vmin = fmin(A.v, fmin(B.v, C.v));
    const double umax = fmax(A.u, fmax(B.u, C.u)), vmax = fmax(A.v, fmax(B.v, C.v));
    c.fu0 = floor(umin);
    c.fv0 = floor(vmin);
    c.T[0] = P2{A.u - c.fu0, A.v - c.fv0};
    c.T[1] = P2{B.u - c.fu0, B.v - c.fv0};
    c.T[2] = P2{C.u - c.fu0, C.v - c.fv0};
    tri_slopes(c.T, c.sv, c.su);
    const double S2 = twice_area(A, B, C, c.fu0, c.fv0);
    c.scale = fdiv(g.tri_weight, S2);
    c.i0 = (int)i0;
    c.j0 = (int)fmax(c.fv0, 0.0);
    c.j1 = (int)fmin(floor(vmax), (double)(g.n2 - 1));
    const double eu = umax - umin, ev = vmax - vmin;
    c.fp32 = mixed && eu * eu + ev * ev <= MIXED_MAX_COND * fabs(S2);
    return c;
}

__device__ inline ColSetup shfl_setup(const ColSetup &s, int L)
{
    ColSetup c;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c.T[k].u = __shfl(s.T[k].u, L, 64);
        c.T[k].v = __shfl(s.T[k].v, L, 64);
        c.sv[k] = __shfl(s.sv[k], L, 64);
        c.su[k] = __shfl(s.su[k], L, 64);
    }
    c.scale = __shfl(s.scale, L, 64);
    c.fu0 = __shfl(s.fu0, L, 64);
    c.fv0 = __shfl(s.fv0, L, 64);
    c.i0 = __shfl(s.i0, L, 64);
    c.j0 = __shfl(s.j0, L, 64);
    c.j1 = __shfl(s.j1, L, 64);
    c.fp32 = __shfl(s.fp32, L, 64);
    return c;
}

// pixel column i0 + r of the triangle set up in `c`
template <bool MIXED, int N>
__device__ inline int setup_column(const ColSetup &c, int r, const MapGeom &g, double *map, const Window<N> &w)
{
    const int i = c.i0 + r;
    const double cl = (double)i - c.fu0;
    if (MIXED && c.fp32) return column_pieces<float>(c.T, c.sv, c.su, cl, c.fv0, i, c.j0, c.j1, c.scale, g, map, w);
    return column_pieces<double>(c.T, c.sv, c.su, cl, c.fv0, i, c.j0, c.j1, c.scale, g, map, w);
}

// IPM of the ordinary triangles.  A workgroup takes a tile of 16 x 16 cells
// (each wavefront 16 x 4): one thread per cell deposits single-pixel
// triangles and classifies the rest (cell (a, b) splits along v00-v11 into
// T1 = (v00, v10, v11) and T2 = (v00, v11, v01)); then each wavefront spreads
// its triangles' pixel columns evenly over its lanes.  A tile of cells maps to
// a compact patch of the source plane, so deposits are summed in an LDS
// window around the tile's image first.  Large triangles are only counted:
// one total per tile, for the gather pass.
constexpr int CT = 16;   // cells per tile side

// cell tile `tile` of a strip (a whole workgroup of 256 threads; acc is its
// N x N LDS window)
template <bool MIXED, int N>
__device__ __forceinline__ void ipm_tile(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0, int64_t nrows,
                                int64_t vb0, const MapGeom &g, double *__restrict__ map,
                                unsigned long long *__restrict__ counters, int32_t *__restrict__ tile_big, int64_t tile,
                                double *acc, unsigned long long *__restrict__ work)
{
    const int64_t ncol = nr1 - 1;
    const int64_t tiles_a = (ncol + CT - 1) / CT;
    const int64_t ta = tile % tiles_a, tb = tile / tiles_a;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t a = ta * CT + (lane & (CT - 1));
    const int64_t brow = tb * CT + wave * 4 + (lane >> 4);   // cell row within the strip
    for (int k = threadIdx.x; k < N * N; k += blockDim.x) acc[k] = 0.0;
    // window anchored on the image of the tile's centre vertex
    Window<N> w;
    w.acc = acc;
    {
        const int64_t ca = min(ta * CT + CT / 2, ncol), cb = min(tb * CT + CT / 2, nrows);
        const double2 c = verts[(cb0 + cb - vb0) * nr1 + ca];
        const double fu = isfinite(c.x) ? fmin(fmax(floor(c.x), -1e9), 1e9) : 0.0;
        const double fv = isfinite(c.y) ? fmin(fmax(floor(c.y), -1e9), 1e9) : 0.0;
        w.i0 = (int)fu - N / 2;
        w.j0 = (int)fv - N / 2;
    }
    __syncthreads();
    unsigned n_small = 0, n_items = 0, n_pieces = 0;   // work counts (statistics)
    int mcols[2] = {0, 0};      // pixel columns of each medium triangle of the cell (0: none)
    int mi0[2] = {0, 0};
    P2 v00{0.0, 0.0}, v10{0.0, 0.0}, v11{0.0, 0.0}, v01{0.0, 0.0};
    int nb = 0;   // large triangles of the cell
    if (a < ncol && brow < nrows) {
        load_cell_at(verts, nr1, cb0 + brow - vb0, a, v00, v10, v11, v01);
        int pi, pj;
        if (cell_in_one_pixel(v00, v10, v11, v01, g, pi, pj)) {
            if (pi >= 0) deposit_w(w, map, g, pi, pj, 2.0 * g.tri_weight);
        } else {
            const P2 tri[2][3] = {{v00, v10, v11}, {v00, v11, v01}};
#pragma unroll
            for (int k = 0; k < 2; ++k) {
                const P2 A = tri[k][0], B = tri[k][1], C = tri[k][2];
                const TriClass c = classify(A, B, C, g);
                if (c.kind == 0) {
                    if (!(isfinite(A.u) && isfinite(A.v) && isfinite(B.u) && isfinite(B.v) && isfinite(C.u) &&
                          isfinite(C.v)))
                        atomicAdd(counters, 1ull);
                } else if (c.kind == 1) {
                    if (c.pi >= 0) deposit_w(w, map, g, c.pi, c.pj, g.tri_weight);
                } else if (c.kind == 2) {
                    if (c.small) {
                        const double fu0 = floor(fmin(A.u, fmin(B.u, C.u))), fv0 = floor(fmin(A.v, fmin(B.v, C.v)));
                        small_triangle(A, B, C, fu0, fv0, g, map, w);
                        ++n_small;
                    } else {
                        mcols[k] = c.cols;
                        mi0[k] = c.i0;
                    }
                } else {
                    ++nb;
                }
            }
        }
    }
    if (tile_big) {   // the tile's count of large triangles (tile_big is zeroed beforehand)
        int s = nb;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0 && s) atomicAdd(tile_big + tile, s);
    }
    // the medium triangles' pixel columns, spread evenly over the wavefront's
    // lanes: first triangle of every cell, then the second
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        int total;
        const int excl = wave_excl_scan(mcols[k], lane, total);
        if (total == 0) continue;
        ColSetup own{};
        if (mcols[k] > 0) own = k == 0 ? col_setup(v00, v10, v11, mi0[k], g, MIXED) : col_setup(v00, v11, v01, mi0[k], g, MIXED);
        for (int base = 0; base < total; base += 64) {
            const int item = base + lane;
            const int L = wave_find(excl, item);
            const int r = item - __shfl(excl, L, 64);
            const ColSetup c = shfl_setup(own, L);
            if (item < total) {
                n_pieces += (unsigned)setup_column<MIXED>(c, r, g, map, w);
                ++n_items;
            }
        }
    }
    if (work) {   // one sum per wavefront and count, spread over WORK_SLOTS slots per count
        unsigned v[3] = {n_small, n_items, n_pieces};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
            if (lane == 0 && v[k]) atomicAdd(work + k * WORK_SLOTS + (tile & (WORK_SLOTS - 1)), (unsigned long long)v[k]);
        }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < N * N; k += blockDim.x) {
        const double v = acc[k];
        if (v != 0.0) {
            const int i = w.i0 + (k % N), j = w.j0 + (k / N);
            deposit(map, g, i, j, v);   // inside the map: only in-map pixels were deposited
        }
    }
    __syncthreads();   // the window may be reused by the workgroup's next tile
}

// Registers capped at 128 per lane (four waves per SIMD, no spills): the
// compiler's free choice (132) holds three, and the cell pass gains more from
// the fourth wave hiding its LDS and cross-lane latency than it loses.
template <bool MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ipm(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0,
                                             int64_t nrows, int64_t vb0, MapGeom g, double *__restrict__ map,
                                             unsigned long long *__restrict__ counters, int32_t *__restrict__ tile_big,
                                             unsigned long long *__restrict__ work)
{
    __shared__ double acc[WIN * WIN];
    ipm_tile<MIXED, WIN>(verts, nr1, cb0, nrows, vb0, g, map, counters, tile_big, blockIdx.x, acc, work);
}

// the same with the 16 x 16 window
template <bool MIXED>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_ipm_fine(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0,
                                             int64_t nrows, int64_t vb0, MapGeom g, double *__restrict__ map,
                                             unsigned long long *__restrict__ counters, int32_t *__restrict__ tile_big,
                                             unsigned long long *__restrict__ work)
{
    __shared__ double acc[WIN_FINE * WIN_FINE];
    ipm_tile<MIXED, WIN_FINE>(verts, nr1, cb0, nrows, vb0, g, map, counters, tile_big, blockIdx.x, acc, work);
}

// every cell tile of every map of a fused batch in one launch (one
// workgroup per tile of the concatenated tile list)
__global__ __launch_bounds__(256) void k_ipm_batch(const BatchMap *__restrict__ maps, int32_t nmaps,
                                                   int64_t ntiles, int32_t *__restrict__ tile_big)
{
    __shared__ double acc[WIN * WIN];
    {
        const int64_t t = blockIdx.x;
        const int32_t m = batch_find(maps, nmaps, t, &BatchMap::ctile_lo);
        const BatchMap &d = maps[m];
        if (d.mixed)
            ipm_tile<true, WIN>(d.verts, d.nr1, 0, d.nrows, 0, d.g, d.map, d.counters, tile_big + d.ctile_lo, t - d.ctile_lo,
                           acc, nullptr);
        else
            ipm_tile<false, WIN>(d.verts, d.nr1, 0, d.nrows, 0, d.g, d.map, d.counters, tile_big + d.ctile_lo, t - d.ctile_lo,
                            acc, nullptr);
    }
}

// which of the cell's two triangles are large (bit k: triangle k), with the
// cell pass's classification: none if the cell lies in one pixel
__device__ inline int cell_big_mask(P2 v00, P2 v10, P2 v11, P2 v01, const MapGeom &g)
{
    int pi, pj;
    if (cell_in_one_pixel(v00, v10, v11, v01, g, pi, pj)) return 0;
    return (classify(v00, v10, v11, g).kind == 3 ? 1 : 0) | (classify(v00, v11, v01, g).kind == 3 ? 2 : 0);
}

// set-up of the cell's large triangles (`mask`), written to slots [slot,
// end): integer local origin (inside or at the edge of the map, so nearby
// pixel boundaries are exact), counter-clockwise local vertices, edge slopes,
// the deposit scale, and the pixel rows it covers (their count in rows[], the
// first in row0[]: compact copies for the binning passes, which need nothing
// else)
__device__ inline void gather_cell(P2 v00, P2 v10, P2 v11, P2 v01, int mask, int64_t slot, int64_t end,
                                   const MapGeom &g, BigPrep *__restrict__ prep, int64_t *__restrict__ rows,
                                   int32_t *__restrict__ row0)
{
    const P2 tri[2][3] = {{v00, v10, v11}, {v00, v11, v01}};
    for (int k = 0; k < 2 && slot < end; ++k) {
        if (!(mask >> k & 1)) continue;
        const P2 A = tri[k][0], B = tri[k][1], C = tri[k][2];
        const double umin = fmin(A.u, fmin(B.u, C.u));
        const double vmin = fmin(A.v, fmin(B.v, C.v)), vmax = fmax(A.v, fmax(B.v, C.v));
        const double ou = fmax(floor(umin), 0.0), ov = fmax(floor(vmin), 0.0);
        P2 T[3] = {P2{A.u - ou, A.v - ov}, P2{B.u - ou, B.v - ov}, P2{C.u - ou, C.v - ov}};
        double S2 = twice_area(A, B, C, ou, ov);
        if (S2 < 0.0) {   // counter-clockwise: the interior is left of every edge
            const P2 tmp = T[1];
            T[1] = T[2];
            T[2] = tmp;
            S2 = -S2;
        }
        BigPrep bp;
        double sv[3], su[3];
        tri_slopes(T, sv, su);
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            bp.u[m] = T[m].u;
            bp.v[m] = T[m].v;
            bp.su[m] = su[m];
        }
        bp.ou = ou;
        bp.ov = ov;
        bp.scale = g.tri_weight / S2;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const double dv = T[m == 2 ? 0 : m + 1].v - T[m].v;
            bp.kc[m] = dv > 0.0 ? -bp.scale * fabs(sv[m]) : (dv < 0.0 ? bp.scale * fabs(sv[m]) : 0.0);
        }
        prep[slot] = bp;
        const double j1 = fmin(floor(vmax), (double)(g.n2 - 1));
        rows[slot] = j1 >= ov ? (int64_t)(j1 - ov) + 1 : 0;
        row0[slot] = (int32_t)ov;
        ++slot;
    }
}

// The large triangles of one cell tile (one workgroup of 256 threads, the
// cells over the threads as in the cell pass), written in thread order to
// [lo, hi), the tile's range from the scan of the cell pass's per-tile counts.
// Slots of that range this pass does not fill (none, as both passes classify
// alike) are left as triangles without rows.
__device__ inline void gather_tile(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0, int64_t nrows,
                                   int64_t vb0, const MapGeom &g, int64_t tile, int64_t lo, int64_t hi,
                                   BigPrep *__restrict__ prep, int64_t *__restrict__ rows,
                                   int32_t *__restrict__ row0, int32_t *wsum)
{
    const int64_t ncol = nr1 - 1;
    const int64_t tiles_a = (ncol + CT - 1) / CT;
    const int64_t ta = tile % tiles_a, tb = tile / tiles_a;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t a = ta * CT + (lane & (CT - 1));
    const int64_t brow = tb * CT + wave * 4 + (lane >> 4);
    P2 v00{0.0, 0.0}, v10{0.0, 0.0}, v11{0.0, 0.0}, v01{0.0, 0.0};
    int mask = 0;
    if (a < ncol && brow < nrows) {
        load_cell_at(verts, nr1, cb0 + brow - vb0, a, v00, v10, v11, v01);
        mask = cell_big_mask(v00, v10, v11, v01, g);
    }
    const int nb = (mask & 1) + (mask >> 1);
    int total;
    const int excl = wave_excl_scan(nb, lane, total);
    if (lane == 0) wsum[wave] = total;
    __syncthreads();
    int64_t slot = lo + excl, found = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) slot += wsum[w];
        found += wsum[w];
    }
    if (mask) gather_cell(v00, v10, v11, v01, mask, slot, min(slot + nb, hi), g, prep, rows, row0);
    for (int64_t s = lo + found + threadIdx.x; s < hi; s += blockDim.x) {
        rows[s] = 0;
        row0[s] = 0;
    }
}

// The number of large triangles of every cell tile (the cell pass's
// classification, cells over the threads as there), stored per tile: what the
// gather needs, without the cell pass, so the large-triangle passes can run
// beside it.
__global__ __launch_bounds__(256) void k_big_count(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0,
                                                   int64_t nrows, int64_t vb0, MapGeom g, int32_t *__restrict__ tile_big)
{
    __shared__ int32_t wsum[4];
    const int64_t tile = blockIdx.x;
    const int64_t ncol = nr1 - 1;
    const int64_t tiles_a = (ncol + CT - 1) / CT;
    const int64_t ta = tile % tiles_a, tb = tile / tiles_a;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t a = ta * CT + (lane & (CT - 1));
    const int64_t brow = tb * CT + wave * 4 + (lane >> 4);
    int nb = 0;
    if (a < ncol && brow < nrows) {
        P2 v00, v10, v11, v01;
        load_cell_at(verts, nr1, cb0 + brow - vb0, a, v00, v10, v11, v01);
        const int mask = cell_big_mask(v00, v10, v11, v01, g);
        nb = (mask & 1) + (mask >> 1);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) nb += __shfl_xor(nb, o, 64);
    if (lane == 0) wsum[wave] = nb;
    __syncthreads();
    if (threadIdx.x == 0) tile_big[tile] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

__global__ __launch_bounds__(256) void k_big_gather(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0,
                                                    int64_t nrows, int64_t vb0, MapGeom g,
                                                    const int64_t *__restrict__ tile_off, BigPrep *__restrict__ prep,
                                                    int64_t *__restrict__ rows, int32_t *__restrict__ row0)
{
    __shared__ int32_t wsum[4];
    const int64_t t = blockIdx.x, lo = tile_off[t], hi = tile_off[t + 1];
    if (lo == hi) return;   // the whole workgroup
    gather_tile(verts, nr1, cb0, nrows, vb0, g, t, lo, hi, prep, rows, row0, wsum);
}

// Calls f(t) for the tiles t < tiles that hold large triangles (tile_off[t] <
// tile_off[t + 1]), with the workgroup in step.  A resident grid strides over
// the tiles; each workgroup reads the offsets of its next 256 tiles at once
// (one per thread) and lists the ones that hold any, so that an empty tile
// costs one load and no workgroup.
template <class F>
__device__ inline void for_big_tiles(int64_t tiles, const int64_t *__restrict__ tile_off, F &&f)
{
    __shared__ int64_t todo[256];
    __shared__ int32_t nwave[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t G = gridDim.x;
    for (int64_t base = blockIdx.x; base < tiles; base += G * 256) {
        const int64_t t = base + (int64_t)threadIdx.x * G;
        const bool has = t < tiles && tile_off[t] != tile_off[t + 1];
        const unsigned long long m = __ballot(has);
        if (lane == 0) nwave[wave] = __popcll(m);
        __syncthreads();
        int off = 0, n = 0;
        for (int k = 0; k < 4; ++k) {
            if (k < wave) off += nwave[k];
            n += nwave[k];
        }
        if (has) todo[off + __popcll(m & ((1ull << lane) - 1ull))] = t;
        __syncthreads();
        for (int k = 0; k < n; ++k) {
            f(todo[k]);
            __syncthreads();   // the tile's LDS may be reused by the next
        }
    }
}

// The gather where most tiles hold no large triangle (a highly magnified
// map, whose cells are far smaller than a pixel): a resident grid that skips
// the empty tiles, instead of a workgroup per tile.
__global__ __launch_bounds__(256) void k_big_gather_sparse(const double2 *__restrict__ verts, int64_t nr1,
                                                           int64_t cb0, int64_t nrows, int64_t vb0, MapGeom g,
                                                           int64_t tiles, const int64_t *__restrict__ tile_off,
                                                           BigPrep *__restrict__ prep, int64_t *__restrict__ rows,
                                                           int32_t *__restrict__ row0)
{
    __shared__ int32_t wsum[4];
    for_big_tiles(tiles, tile_off, [&](int64_t t) {
        gather_tile(verts, nr1, cb0, nrows, vb0, g, t, tile_off[t], tile_off[t + 1], prep, rows, row0, wsum);
    });
}

// the batch's cell tiles: tile_off is the scan over all maps' tiles
__global__ __launch_bounds__(256) void k_big_gather_batch(const BatchMap *__restrict__ maps, int32_t nmaps,
                                                          const int64_t *__restrict__ tile_off,
                                                          BigPrep *__restrict__ prep, int64_t *__restrict__ rows,
                                                          int32_t *__restrict__ row0)
{
    __shared__ int32_t wsum[4];
    const int64_t t = blockIdx.x, lo = tile_off[t], hi = tile_off[t + 1];
    if (lo == hi) return;   // the whole workgroup
    const BatchMap &d = maps[batch_find(maps, nmaps, t, &BatchMap::ctile_lo)];
    gather_tile(d.verts, d.nr1, 0, d.nrows, 0, d.g, t - d.ctile_lo, lo, hi, prep, rows, row0, wsum);
}

// The edges of a large triangle clipped to pixel row j (local coordinates),
// the row's column range [ga, gb] inside the map and the run [pa, pb] of
// pixels fully inside the triangle (local column indices; pa > pb: none);
// false if the row holds nothing
struct RowInfo {
    Segs S;
    double rl;
    int64_t ga, gb, pa, pb;
};

__device__ inline bool row_info(const BigPrep &bp, int64_t j, const MapGeom &g, RowInfo &ri)
{
    const P2 T[3] = {P2{bp.u[0], bp.v[0]}, P2{bp.u[1], bp.v[1]}, P2{bp.u[2], bp.v[2]}};
    const double su[3] = {bp.su[0], bp.su[1], bp.su[2]};
    ri.rl = (double)j - bp.ov;
    const double rl = ri.rl;
    strip_segments<1>(T, su, rl, rl + 1.0, ri.S);
    double rumin = 1e300, rumax = -1e300;
#pragma unroll
    for (int k = 0; k < 3; ++k)
        if (ri.S.d[k] != 0.0 || ri.S.a[k] != ri.S.b[k]) {
            rumin = fmin(rumin, fmin(ri.S.a[k], ri.S.b[k]));
            rumax = fmax(rumax, fmax(ri.S.a[k], ri.S.b[k]));
        }
    if (rumin > rumax) return false;
    const double ga = fmax(floor(rumin), -bp.ou), gb = fmin(floor(rumax), (double)(g.n1 - 1) - bp.ou);
    if (ga > gb) return false;
    // a pixel is fully inside when every corner is on the inner side of each edge
    double fa = -1e300, fb = 1e300;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const P2 P = T[m], Q = T[(m + 1) % 3];
        const double dx = Q.u - P.u, dy = Q.v - P.v;
        const double vc = dx > 0.0 ? rl : rl + 1.0;
        const double off = (vc - P.v) * su[m];   // dx (vc - P.v) / dy
        if (dy > 0.0) fb = fmin(fb, floor(P.u - 1.0 + off));
        else if (dy < 0.0) fa = fmax(fa, ceil(P.u + off));
        else if (dx * (vc - P.v) < 0.0) fa = 1e300;
    }
    fa = fmax(fa, ga);
    fb = fmin(fb, gb);
    ri.ga = (int64_t)ga;
    ri.gb = (int64_t)gb;
    if (fa <= fb) {
        ri.pa = (int64_t)fa;
        ri.pb = (int64_t)fb;
    } else {
        ri.pa = ri.gb + 1;
        ri.pb = ri.gb;
    }
    return true;
}

// IPM of the large triangles: a wavefront owns 64 of them; their pixel rows
// are spread over its lanes (fully covered runs go to the difference buffer),
// then the boundary pixels of those 64 rows, whose row polygons the lanes
// share through the wavefront's slots in LDS
struct RowSlot {
    Segs S;
    double ou, scale;
    int64_t j, ga, pa, pb, gb;
};

__global__ __launch_bounds__(256) void k_big(int64_t nbig, const BigPrep *__restrict__ prep,
                                             const int64_t *__restrict__ rows, MapGeom g, double *__restrict__ map,
                                             double *__restrict__ diff)
{
    __shared__ RowSlot slots[256];
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63);
    const int64_t k = wave0 + lane;
    RowSlot *ws = slots + (threadIdx.x & ~63);
    const int nrow = k < nbig ? (int)rows[k] : 0;
    int rtotal;
    const int rexcl = wave_excl_scan(nrow, lane, rtotal);
    for (int rbase = 0; rbase < rtotal; rbase += 64) {
        const int ritem = rbase + lane;
        const int L = wave_find(rexcl, ritem);
        const int rr = ritem - __shfl(rexcl, L, 64);
        int np = 0;
        if (ritem < rtotal) {
            const BigPrep bp = prep[wave0 + L];
            const int64_t j = (int64_t)bp.ov + rr;
            RowInfo ri;
            if (row_info(bp, j, g, ri)) {
                const bool full = ri.pa <= ri.pb;
                np = (int)(full ? (ri.pa - ri.ga) + (ri.gb - ri.pb) : ri.gb - ri.ga + 1);
                if (full) {
                    double *dr = diff + j * (int64_t)(g.n1 + 1) + (int64_t)bp.ou;
                    unsafeAtomicAdd(dr + ri.pa, 2.0 * bp.scale);
                    unsafeAtomicAdd(dr + ri.pb + 1, -2.0 * bp.scale);
                }
                RowSlot &sl = ws[lane];
                sl.S = ri.S;
                sl.ou = bp.ou;
                sl.scale = bp.scale;
                sl.j = j;
                sl.ga = ri.ga;
                sl.pa = ri.pa;
                sl.pb = ri.pb;
                sl.gb = ri.gb;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        int ptotal;
        const int pexcl = wave_excl_scan(np, lane, ptotal);
        for (int pbase = 0; pbase < ptotal; pbase += 64) {
            const int pitem = pbase + lane;
            const int M = wave_find(pexcl, pitem);
            const int64_t r = pitem - __shfl(pexcl, M, 64);
            if (pitem < ptotal) {
                const RowSlot &sl = ws[M];
                int64_t i;
                if (sl.pa <= sl.pb) i = (r < sl.pa - sl.ga) ? sl.ga + r : sl.pb + 1 + (r - (sl.pa - sl.ga));
                else i = sl.ga + r;
                if (i >= sl.ga && i <= sl.gb) {
                    const Segs S = sl.S;
                    // twice the area: 2 (G(i + 1) - G(i)), G(c) = -sum dv I(c - ua, c - ub)
                    const double a2 = 2.0 * (strip_cumulative(S, (double)i) - strip_cumulative(S, (double)(i + 1)));
                    if (a2 != 0.0) deposit(map, g, (int)(i + (int64_t)sl.ou), (int)sl.j, sl.scale * a2);   // in the map
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---------------------------------------------------------------------------
// Large triangles by pixel bands.  Every pixel receives hundreds of boundary
// deposits from the large triangles around star images, and device-wide
// atomics are the limit, so the work is binned instead: the map's rows are cut
// into bands of BH full-width rows, each large triangle is listed in every
// band its rows cross, and one workgroup per band accumulates the column
// differences of its rows in LDS from the triangles' edges, prefix-sums its
// own rows and adds them to the map.
// ---------------------------------------------------------------------------
// Two band workgroups share a compute unit's LDS; 768 threads each with at
// most 80 registers per lane (a few bytes spilled) keep six waves per SIMD,
// where 512 threads left four.
constexpr int BAND_THREADS = 768;
constexpr int64_t BAND_LDS_DOUBLES = 8192;    // band difference rows (64 KiB)

__device__ inline void band_range(int64_t j0, int64_t rows, int bh, int64_t &b0, int64_t &b1)
{
    b0 = j0 / bh;
    b1 = (j0 + rows - 1) / bh;
}

// Per-band counts of a workgroup's triangles from their band ranges [b0, b1]:
// each adds +1 at b0 and -1 past b1 in `hist` (nb + 1 entries, zeroed), and
// a prefix sum over the bands turns that in place into the counts (O(1)
// updates per triangle instead of one per band).  The sum runs over
// contiguous chunks of bands, one per thread, chained by a scan of the chunk
// totals (`part`: one entry per wavefront).  Called by the whole workgroup;
// synchronises before and after.
__device__ inline void band_diff_to_counts(int32_t *hist, int32_t nb, int32_t *part)
{
    __syncthreads();
    const int nt = (int)blockDim.x, t = (int)threadIdx.x, lane = t & 63, wave = t >> 6;
    const int chunk = (nb + nt - 1) / nt, c0 = min(t * chunk, (int)nb), c1 = min(c0 + chunk, (int)nb);
    int sum = 0;
    for (int b = c0; b < c1; ++b) sum += hist[b];
    int total;
    const int excl = wave_excl_scan(sum, lane, total);
    if (lane == 0) part[wave] = total;
    __syncthreads();
    int run = excl;
    for (int w = 0; w < wave; ++w) run += part[w];
    for (int b = c0; b < c1; ++b) {
        run += hist[b];
        hist[b] = run;
    }
    __syncthreads();
}

// LDS words of a band histogram with its scan totals (256 threads), rounded
// up to whole 8-byte words
__host__ __device__ inline size_t band_hist_words(int64_t nb) { return (size_t)((nb + 1 + 4 + 1) & ~1); }

// Binning of the large triangles into bands.  A workgroup takes BIN_TRIS
// consecutive ones, [lo, hi) of one map, so that each device-wide update of a
// band's total or cursor serves many triangles (with one triangle per thread
// those updates, all on the few hundred band entries, were the cost).
// bin_count adds the workgroup's per-band counts to count[] (hist: LDS of
// band_hist_words(nb) words).
__device__ inline void bin_count(int64_t lo, int64_t hi, const int32_t *__restrict__ row0,
                                 const int64_t *__restrict__ rows, int bh, int32_t nb, int32_t *hist,
                                 int32_t *__restrict__ count)
{
    for (int32_t b = threadIdx.x; b <= nb; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        const int64_t n = rows[k];
        if (n <= 0) continue;
        int64_t b0, b1;
        band_range(row0[k], n, bh, b0, b1);
        atomicAdd(&hist[b0], 1);
        atomicAdd(&hist[b1 + 1], -1);
    }
    band_diff_to_counts(hist, nb, hist + nb + 1);
    for (int32_t b = threadIdx.x; b < nb; b += blockDim.x)
        if (hist[b]) atomicAdd(count + b, hist[b]);
}

// triangle indices into their bands' lists: the workgroup reserves one range
// per band from cursor[] and hands out slots inside it from LDS (sh:
// band_hist_words(nb) words, then nb 8-byte range starts)
__device__ inline void bin_scatter(int64_t lo, int64_t hi, const int32_t *__restrict__ row0,
                                   const int64_t *__restrict__ rows, int bh, int32_t nb, int32_t *sh,
                                   unsigned long long *__restrict__ cursor, int32_t *__restrict__ list)
{
    int32_t *hist = sh;
    unsigned long long *base = reinterpret_cast<unsigned long long *>(sh + band_hist_words(nb));
    for (int32_t b = threadIdx.x; b <= nb; b += blockDim.x) hist[b] = 0;
    __syncthreads();
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        const int64_t n = rows[k];
        if (n <= 0) continue;
        int64_t b0, b1;
        band_range(row0[k], n, bh, b0, b1);
        atomicAdd(&hist[b0], 1);
        atomicAdd(&hist[b1 + 1], -1);
    }
    band_diff_to_counts(hist, nb, hist + nb + 1);
    for (int32_t b = threadIdx.x; b < nb; b += blockDim.x) {
        if (hist[b]) base[b] = atomicAdd(cursor + b, (unsigned long long)hist[b]);
        hist[b] = 0;
    }
    __syncthreads();
    for (int64_t k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        const int64_t n = rows[k];
        if (n <= 0) continue;
        int64_t b0, b1;
        band_range(row0[k], n, bh, b0, b1);
        for (int64_t b = b0; b <= b1; ++b) {
            const int32_t o = atomicAdd(&hist[b], 1);
            list[base[b] + o] = (int32_t)k;
        }
    }
}

__global__ __launch_bounds__(256) void k_band_count(int64_t nbig, const int32_t *__restrict__ row0,
                                                    const int64_t *__restrict__ rows, int bh, int32_t nbands,
                                                    int32_t *__restrict__ count)
{
    extern __shared__ int32_t hist[];
    const int64_t lo = (int64_t)blockIdx.x * BIN_TRIS;
    bin_count(lo, min(lo + BIN_TRIS, nbig), row0, rows, bh, nbands, hist, count);
}

__global__ __launch_bounds__(256) void k_band_scatter(int64_t nbig, const int32_t *__restrict__ row0,
                                                      const int64_t *__restrict__ rows, int bh, int32_t nbands,
                                                      unsigned long long *__restrict__ cursor,
                                                      int32_t *__restrict__ list)
{
    extern __shared__ int32_t sh[];
    const int64_t lo = (int64_t)blockIdx.x * BIN_TRIS;
    bin_scatter(lo, min(lo + BIN_TRIS, nbig), row0, rows, bh, nbands, sh, cursor, list);
}

// A workgroup takes a band of bh pixel rows (or a slice of its list); a
// thread takes one (listed triangle, band row) item at a time.  Within a pixel row the triangle's area
// left of u = c is G(c) = -sum_e dv_e J_e(c), J_e(c) = I(c - ua_e, c - ub_e)
// over the edges clipped to the row, so pixel i receives
// sum_e delta_e(i), delta_e(i) = -dv_e (J_e(i + 1) - J_e(i)).  delta_e is zero
// left of the edge, equal to -dv_e right of it and varies only over the
// columns the edge crosses; so the band keeps differences
// D(i) = delta(i) - delta(i - 1), which an edge changes only at those columns
// and the one after, and a prefix sum along the row gives the pixel areas
// (the covered interior costs nothing).  Columns left of the map fold into
// column 0, those right of it are dropped.  The differences live in LDS, so
// no device-wide atomic is needed per deposit; the rows are added to the map
// once per band (atomically when the band is shared or the cell pass runs
// beside it).

// edge P->Q clipped to the pixel row rl <= v <= rl + 1 (su = du/dv, finite):
// the u of its ends and its extent dv; false if it has none in the row (an
// edge with P.v = Q.v included).  Ends inside the row keep their exact u (for
// P the clip's product is then an exact zero).
__device__ inline bool row_clip(P2 P, P2 Q, double rl, double su, double &ua, double &ub, double &dv)
{
    const double ev = fmin(fmax(P.v, rl), rl + 1.0), xv = fmin(fmax(Q.v, rl), rl + 1.0);
    ua = fma(ev - P.v, su, P.u);
    ub = xv == Q.v ? Q.u : P.u + (xv - P.v) * su;
    dv = xv - ev;
    return dv != 0.0;
}

// band `band` of one map: its listed triangles are list[r0, r1); bdiff is
// the workgroup's LDS (bh x n1 doubles), wsum two LDS counters
__device__ inline void band_rows(int64_t band, int64_t r0, int64_t r1, const int32_t *__restrict__ list,
                                 const BigPrep *__restrict__ prep, const int64_t *__restrict__ rows, int bh,
                                 const MapGeom &g, double *__restrict__ map, unsigned long long *__restrict__ work,
                                 double *bdiff, unsigned long long *wsum, bool atomic_flush)
{
    if (threadIdx.x < 2) wsum[threadIdx.x] = 0;
    unsigned long long my_rows = 0, my_pieces = 0;
    const int64_t n1 = g.n1;
    const int64_t jb0 = band * bh;
    const int nrow = (int)min((int64_t)bh, (int64_t)g.n2 - jb0);
    for (int64_t t = threadIdx.x; t < (int64_t)bh * n1; t += blockDim.x) bdiff[t] = 0.0;
    __syncthreads();
    // items (listed triangle, row of the band); bh is a power of two that
    // divides the workgroup, so a thread keeps its row
    const int lg = __builtin_ctz((unsigned)bh);
    const int rr = (int)threadIdx.x & (bh - 1);
    const int nlist = (int)(r1 - r0);
    for (int li = (int)threadIdx.x >> lg; li < nlist; li += (int)blockDim.x >> lg) {
        if (rr >= nrow) break;
        const int64_t k = list[r0 + li];
        const BigPrep bp = prep[k];
        const int j = (int)jb0 + rr, ov = (int)bp.ov;   // ov in [0, n2)
        if (j < ov || j - ov >= rows[k]) continue;
        ++my_rows;
        const double rl = (double)(j - ov);
        const int ou = (int)bp.ou;             // in [0, n1]
        double *drow = bdiff + rr * n1 + ou;   // indexed by local column
        const int cmin = -ou, cmax = (int)n1 - 1 - ou;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            const P2 P{bp.u[m], bp.v[m]}, Q{bp.u[(m + 1) % 3], bp.v[(m + 1) % 3]};
            double ua, ub, dv;
            if (!row_clip(P, Q, rl, bp.su[m], ua, ub, dv)) continue;
            // first and last column of the clipped edge, clamped to one
            // column beyond the map on either side (which changes nothing
            // below) so they fit 32 bits
            const double lo = (double)cmin - 1.0, hi = (double)cmax + 1.0;
            const int x0 = (int)fmin(fmax(floor(fmin(ua, ub)), lo), hi);
            const int x1 = (int)fmin(fmax(floor(fmax(ua, ub)), lo), hi);
            const double f = -2.0 * bp.scale * dv;   // deposit for a fully covered difference
            const int is = max(x0, cmin);
            if (is > x1) {   // the segment lies left of the map
                atomicAdd(drow + cmin, f);
                ++my_pieces;
                continue;
            }
            // f J(x) at column boundaries x, J the clamp integral over the
            // clipped edge of width w: 0 up to x0, the crossing form
            // f (x - umin)^2 / (2 w) = kc (x - umin)^2 up to x1 (f / w is
            // fixed along the edge), the linear form at x1 + 1 (past the
            // edge), so the walk needs neither case tests nor a division
            const double umin = fmin(ua, ub), kc = bp.kc[m];
            auto cross = [&](int x) {
                const double t = (double)x - umin;
                return kc * t * t;
            };
            double Jc = is > x0 ? cross(is) : 0.0, prev = 0.0;
            const int iend = min(x1 - 1, cmax);
            if (is <= iend) {
                // differences of the crossing form, cur(i) = J(i + 1) - J(i),
                // are kc (2 (i - umin) + 1) past the edge's first column, so
                // consecutive ones differ by the constant 2 kc: all the
                // columns past the first two receive
                const double J1 = cross(is + 1);
                prev = J1 - Jc;
                atomicAdd(drow + is, prev);
                if (is + 1 <= iend) {
                    const double d2 = 2.0 * kc;
                    const double c1 = kc * (2.0 * ((double)(is + 1) - umin) + 1.0);
                    atomicAdd(drow + is + 1, c1 - prev);
                    for (int i = is + 2; i <= iend; ++i) atomicAdd(drow + i, d2);
                    prev = kc * (2.0 * ((double)iend - umin) + 1.0);
                }
                Jc = cross(iend + 1);
            }
            if (x1 <= cmax) {
                const double Jn = f * (0.5 * (((double)(x1 + 1) - ua) + ((double)(x1 + 1) - ub)));
                const double cur = Jn - Jc;
                atomicAdd(drow + x1, cur - prev);
                prev = cur;
                if (x1 + 1 <= cmax) atomicAdd(drow + x1 + 1, f - prev);
            }
            my_pieces += (unsigned long long)(max(min(x1, cmax) - is + 1, 0) + (x1 + 1 <= cmax ? 1 : 0));
        }
    }
    __syncthreads();
    // per row: prefix sum of the differences, added to the map
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int rr = wave; rr < nrow; rr += BAND_THREADS / 64) {
        const double *dr = bdiff + rr * n1;
        double *mr = map + (jb0 + rr) * n1;
        double carry = 0.0;
        for (int64_t c = 0; c < n1; c += 64) {
            const int64_t i = c + lane;
            double v = i < n1 ? dr[i] : 0.0;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const double o = __shfl_up(v, d, 64);
                if (lane >= d) v += o;
            }
            v += carry;
            carry = __shfl(v, 63, 64);
            if (i < n1 && v != 0.0) {
                if (atomic_flush) unsafeAtomicAdd(mr + i, v);   // the cell pass may be adding to these rows
                else mr[i] += v;
            }
        }
    }
    if (work) {   // work counts for statistics: row items and difference deposits
        atomicAdd(&wsum[0], my_rows);
        atomicAdd(&wsum[1], my_pieces);
        __syncthreads();
        if (threadIdx.x < 2 && wsum[threadIdx.x]) atomicAdd(work + threadIdx.x, wsum[threadIdx.x]);
    }
    __syncthreads();   // the LDS may be reused for the workgroup's next band
}

// The next work item of a persistent band pass for this workgroup, or -1 when
// every range is drained: its XCD's range first, then the others in turn.
// `visited` (thread 0's own) counts the ranges found empty, so each counter is
// pushed past its range at most once per workgroup and the loop ends.
__device__ inline int64_t next_item(unsigned long long *queue, const ItemParts &parts, int &visited)
{
    const int home = (int)(blockIdx.x % NXCD);
    while (visited < NXCD) {
        const int x = (home + visited) % NXCD;
        const int64_t k = (int64_t)atomicAdd(queue + (size_t)x * QUEUE_STRIDE, 1ull);
        if (parts.lo[x] + k < parts.lo[x + 1]) return parts.lo[x] + k;
        ++visited;
    }
    return -1;
}

// The batch's band pass as one persistent launch: a grid the device holds at
// once pulls work items from device-wide counters until none are left.  An
// item is a slice of one band's list (BandItem), so a heavy band is shared by
// several workgroups instead of holding one while the others idle; a band
// split into several items adds its rows to the map atomically.
__global__ __launch_bounds__(BAND_THREADS) __attribute__((amdgpu_waves_per_eu(6))) void k_band_queue(const BatchMap *__restrict__ maps, int32_t nmaps,
                                                             const BandItem *__restrict__ items, ItemParts parts,
                                                             unsigned long long *__restrict__ queue,
                                                             const int32_t *__restrict__ list,
                                                             const BigPrep *__restrict__ prep,
                                                             const int64_t *__restrict__ rows)
{
    extern __shared__ double bdiff[];
    __shared__ unsigned long long wsum[2];
    __shared__ int64_t cur;
    int visited = 0;
    for (;;) {
        if (threadIdx.x == 0) cur = next_item(queue, parts, visited);
        __syncthreads();
        const int64_t i = cur;
        __syncthreads();   // every thread has read cur before the next item overwrites it
        if (i < 0) break;   // the same for the whole workgroup
        const BandItem it = items[i];
        const int32_t m = batch_find(maps, nmaps, it.gband, &BatchMap::band_lo);
        const BatchMap &d = maps[m];
        band_rows(it.gband - d.band_lo, it.lo, it.hi, list, prep, rows, d.bh, d.g, d.map, nullptr, bdiff, wsum,
                  it.shared != 0);
    }
}

// The same for one map: items over its bands (BandItem.gband is the band);
// with `atomic_all` every band's rows are added atomically (the cell pass
// runs beside it).
__global__ __launch_bounds__(BAND_THREADS) __attribute__((amdgpu_waves_per_eu(6))) void k_band_queue1(const BandItem *__restrict__ items, ItemParts parts,
                                                              unsigned long long *__restrict__ queue,
                                                              const int32_t *__restrict__ list,
                                                              const BigPrep *__restrict__ prep,
                                                              const int64_t *__restrict__ rows, int bh, MapGeom g,
                                                              double *__restrict__ map,
                                                              unsigned long long *__restrict__ work, int atomic_all)
{
    extern __shared__ double bdiff[];
    __shared__ unsigned long long wsum[2];
    __shared__ int64_t cur;
    int visited = 0;
    for (;;) {
        if (threadIdx.x == 0) cur = next_item(queue, parts, visited);
        __syncthreads();
        const int64_t i = cur;
        __syncthreads();
        if (i < 0) break;
        const BandItem it = items[i];
        band_rows(it.gband, it.lo, it.hi, list, prep, rows, bh, g, map, work, bdiff, wsum,
                  atomic_all != 0 || it.shared != 0);
    }
}

// band binning of a batch's large triangles.  The triangles of map m are
// the contiguous range [big_lo, big_hi) of its BatchMap (they were gathered
// in cell order); slice s of the launch holds up to BIN_TRIS of them and lies
// inside one map (`slice_map`, `slice_lo`), so a workgroup histograms that
// map's bands in LDS and issues one device-wide atomic per band it touches.
__global__ __launch_bounds__(256) void k_band_count_batch(const BatchMap *__restrict__ maps,
                                                          const int32_t *__restrict__ slice_map,
                                                          const int64_t *__restrict__ slice_lo,
                                                          const int32_t *__restrict__ row0,
                                                          const int64_t *__restrict__ rows,
                                                          int32_t *__restrict__ count)
{
    extern __shared__ int32_t hist[];
    const BatchMap &d = maps[slice_map[blockIdx.x]];
    const int64_t lo = slice_lo[blockIdx.x];
    bin_count(lo, min(lo + BIN_TRIS, d.big_hi), row0, rows, d.bh, (int32_t)d.nbands, hist, count + d.band_lo);
}

__global__ __launch_bounds__(256) void k_band_scatter_batch(const BatchMap *__restrict__ maps,
                                                            const int32_t *__restrict__ slice_map,
                                                            const int64_t *__restrict__ slice_lo,
                                                            const int32_t *__restrict__ row0,
                                                            const int64_t *__restrict__ rows,
                                                            unsigned long long *__restrict__ cursor,
                                                            int32_t *__restrict__ list)
{
    extern __shared__ int32_t sh[];
    const BatchMap &d = maps[slice_map[blockIdx.x]];
    const int64_t lo = slice_lo[blockIdx.x];
    bin_scatter(lo, min(lo + BIN_TRIS, d.big_hi), row0, rows, d.bh, (int32_t)d.nbands, sh, cursor + d.band_lo, list);
}

// map[j][i] += sum_{k <= i} diff[j][k]; one wavefront per pixel row
__global__ __launch_bounds__(64) void k_diff_rows(MapGeom g, const double *__restrict__ diff, double *__restrict__ map)
{
    const int64_t j = blockIdx.x;
    const int lane = threadIdx.x;
    const double *dr = diff + j * (int64_t)(g.n1 + 1);
    double *mr = map + j * (int64_t)g.n1;
    double carry = 0.0;
    for (int64_t c = 0; c < g.n1; c += 64) {
        const int64_t i = c + lane;
        double v = i < g.n1 ? dr[i] : 0.0;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const double o = __shfl_up(v, d, 64);
            if (lane >= d) v += o;
        }
        v += carry;
        if (i < g.n1 && v != 0.0) mr[i] += v;
        carry = __shfl(v, 63, 64);
    }
}


// Statistics only (maps with timing 2): the (triangle, pixel) pairs of cell
// rows [cb0, cb0 + ncells / (nr1 - 1)) that meet inside the map -- the pieces
// the apportioning deposits, whatever path a triangle takes.  The part of a
// triangle inside one pixel row is a convex polygon spanning [umin, umax], so
// it meets the columns floor(umin) .. ceil(umax) - 1 of that row.  A
// zero-area triangle is one piece (its centroid's pixel); one with a
// non-finite vertex none.
__device__ inline int64_t tri_pieces(double2 A, double2 B, double2 C, const MapGeom &g)
{
    if (!isfinite(A.x) || !isfinite(A.y) || !isfinite(B.x) || !isfinite(B.y) || !isfinite(C.x) || !isfinite(C.y))
        return 0;
    const double s2 = (B.x - A.x) * (C.y - A.y) - (C.x - A.x) * (B.y - A.y);
    if (s2 == 0.0) {
        const double cu = floor((A.x + B.x + C.x) / 3.0), cv = floor((A.y + B.y + C.y) / 3.0);
        return (cu >= 0.0 && cv >= 0.0 && cu < (double)g.n1 && cv < (double)g.n2) ? 1 : 0;
    }
    const double2 P[3] = {A, B, C};
    const double vlo = fmin(A.y, fmin(B.y, C.y)), vhi = fmax(A.y, fmax(B.y, C.y));
    const double j0 = fmax(floor(vlo), 0.0), j1 = fmin(ceil(vhi) - 1.0, (double)g.n2 - 1.0);
    int64_t n = 0;
    for (double j = j0; j <= j1; j += 1.0) {
        double lo = INFINITY, hi = -INFINITY;
        for (int k = 0; k < 3; ++k) {
            const double2 p = P[k], q = P[(k + 1) % 3];
            if (p.y >= j && p.y <= j + 1.0) {
                lo = fmin(lo, p.x);
                hi = fmax(hi, p.x);
            }
            for (int e = 0; e < 2; ++e) {   // crossings of v = j and v = j + 1
                const double r = j + (double)e;
                if ((p.y - r) * (q.y - r) < 0.0) {
                    const double x = p.x + (r - p.y) * (q.x - p.x) / (q.y - p.y);
                    lo = fmin(lo, x);
                    hi = fmax(hi, x);
                }
            }
        }
        if (!(lo <= hi)) continue;
        const double i0 = fmax(floor(lo), 0.0), i1 = fmin(ceil(hi) - 1.0, (double)g.n1 - 1.0);
        if (i1 >= i0) n += (int64_t)(i1 - i0) + 1;
    }
    return n;
}

__global__ __launch_bounds__(256) void k_count_pieces(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0,
                                                      int64_t ncells, int64_t vb0, MapGeom g,
                                                      unsigned long long *__restrict__ out)
{
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long n = 0;
    if (c < ncells) {
        const int64_t a = c % (nr1 - 1), b = cb0 + c / (nr1 - 1);
        const double2 *r0 = verts + (b - vb0) * nr1, *r1 = r0 + nr1;
        n = (unsigned long long)(tri_pieces(r0[a], r0[a + 1], r1[a + 1], g) + tri_pieces(r0[a], r1[a + 1], r1[a], g));
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) n += __shfl_xor(n, o, 64);
    if ((threadIdx.x & 63) == 0 && n) atomicAdd(out, n);
}

}  // namespace

void launch_ipm(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                double *map, unsigned long long *counters, int32_t *tile_big, bool mixed, bool fine,
                unsigned long long *work, hipStream_t st)
{
    const int64_t nrows = cb1 - cb0, tiles = ipm_tile_count(nr1, nrows);
    if (tiles <= 0) return;
    auto *k = fine ? (mixed ? k_ipm_fine<true> : k_ipm_fine<false>) : (mixed ? k_ipm<true> : k_ipm<false>);
    hipLaunchKernelGGL(k, dim3((unsigned)tiles), dim3(256), 0, st, verts, nr1, cb0, nrows, vb0, g, map, counters,
                       tile_big, work);
}

// grid of a persistent kernel: the workgroups of `threads` threads of `kernel`
// the device holds at once with `shmem` bytes of LDS, or fewer for few items
// (a multiple of NXCD, so that every XCD's range has workgroups of its own)
static int64_t resident_grid(const void *kernel, int threads, size_t shmem, int64_t nitems)
{
    int dev = 0, cus = 0, per_cu = 0;
    MLM_HIP(hipGetDevice(&dev));
    MLM_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    MLM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, shmem));
    const int64_t full = (int64_t)std::max(cus, 1) * std::max(per_cu, 1);
    return std::min(full, (nitems + NXCD - 1) / NXCD * NXCD);
}

int64_t ipm_tile_count(int64_t nr1, int64_t nrows)
{
    const int64_t ncol = nr1 - 1;
    if (ncol <= 0 || nrows <= 0) return 0;
    return ((ncol + CT - 1) / CT) * ((nrows + CT - 1) / CT);
}

void launch_big_gather(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                       int64_t nbig, const int64_t *tile_off, BigPrep *prep, int64_t *rows, int32_t *row0,
                       hipStream_t st)
{
    const int64_t tiles = ipm_tile_count(nr1, cb1 - cb0);
    if (tiles <= 0) return;
    if (nbig < tiles) {   // fewer large triangles than tiles: most tiles are empty
        const int64_t grid = resident_grid(reinterpret_cast<const void *>(&k_big_gather_sparse), 256, 0, tiles);
        hipLaunchKernelGGL(k_big_gather_sparse, dim3((unsigned)grid), dim3(256), 0, st, verts, nr1, cb0, cb1 - cb0,
                           vb0, g, tiles, tile_off, prep, rows, row0);
    } else {
        hipLaunchKernelGGL(k_big_gather, dim3((unsigned)tiles), dim3(256), 0, st, verts, nr1, cb0, cb1 - cb0, vb0, g,
                           tile_off, prep, rows, row0);
    }
}

void launch_big_count(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                      int32_t *tile_big, hipStream_t st)
{
    const int64_t tiles = ipm_tile_count(nr1, cb1 - cb0);
    if (tiles > 0)
        hipLaunchKernelGGL(k_big_count, dim3((unsigned)tiles), dim3(256), 0, st, verts, nr1, cb0, cb1 - cb0, vb0, g,
                           tile_big);
}

void launch_big(int64_t nbig, const BigPrep *prep, const int64_t *rows, const MapGeom &g, double *map, double *diff,
                hipStream_t st)
{
    if (nbig > 0)
        hipLaunchKernelGGL(k_big, dim3((unsigned)((nbig + 255) / 256)), dim3(256), 0, st, nbig, prep, rows, g, map, diff);
}

// LDS bytes of the scatter pass's workgroup for nb bands (the largest of the
// binning passes): the histogram with its scan totals, then one 8-byte range
// start per band
static size_t bin_lds_bytes(int64_t nb) { return band_hist_words(nb) * sizeof(int32_t) + (size_t)nb * 8; }

// the LDS a workgroup may be given on the current device (64 KiB if the
// device does not say)
static size_t lds_per_workgroup()
{
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v <= 0)
        v = 65536;
    return (size_t)v;
}

int band_height(int32_t n1, int32_t n2)
{
    // a power of two (at most 16, so it divides the workgroup), as many rows
    // of the map as the LDS holds
    int64_t bh = 16;
    while (bh > 0 && bh * n1 > BAND_LDS_DOUBLES) bh >>= 1;
    // 0: the map is too wide for one band per workgroup, or has too many bands
    // for the binning histograms in LDS
    static const size_t lds = lds_per_workgroup();
    if (bh > 0 && bin_lds_bytes((n2 + bh - 1) / bh) > lds) bh = 0;
    return (int)bh;
}

void launch_band_count(int64_t nbig, const int32_t *row0, const int64_t *rows, int bh, int32_t nbands, int32_t *count,
                       hipStream_t st)
{
    (void)hipGetLastError();   // clear what earlier calls left, so the check below sees this launch
    if (nbig > 0)
        hipLaunchKernelGGL(k_band_count, dim3((unsigned)((nbig + BIN_TRIS - 1) / BIN_TRIS)), dim3(256),
                           band_hist_words(nbands) * sizeof(int32_t), st, nbig, row0, rows, bh, nbands, count);
    MLM_HIP(hipGetLastError());   // a refused launch leaves the band lists unset: fail here
}

void launch_band_scatter(int64_t nbig, const int32_t *row0, const int64_t *rows, int bh, int32_t nbands,
                         unsigned long long *cursor, int32_t *list, hipStream_t st)
{
    const size_t shmem = bin_lds_bytes(nbands);
    (void)hipGetLastError();   // clear what earlier calls left, so the check below sees this launch
    if (nbig > 0)
        hipLaunchKernelGGL(k_band_scatter, dim3((unsigned)((nbig + BIN_TRIS - 1) / BIN_TRIS)), dim3(256), shmem, st, nbig, row0, rows,
                           bh, nbands, cursor, list);
    MLM_HIP(hipGetLastError());
}


void launch_ipm_batch(const BatchMap *maps, int32_t nmaps, int64_t nctiles, int32_t *tile_big, hipStream_t st)
{
    if (nctiles <= 0) return;
    if (nctiles > (int64_t)UINT32_MAX) fail(MLM_ERANGE, "too many cell tiles in one batch chunk");
    hipLaunchKernelGGL(k_ipm_batch, dim3((unsigned)nctiles), dim3(256), 0, st, maps, nmaps, nctiles, tile_big);
}

void launch_big_gather_batch(const BatchMap *maps, int32_t nmaps, int64_t nctiles, const int64_t *tile_off,
                             BigPrep *prep, int64_t *rows, int32_t *row0, hipStream_t st)
{
    if (nctiles > 0)
        hipLaunchKernelGGL(k_big_gather_batch, dim3((unsigned)nctiles), dim3(256), 0, st, maps, nmaps, tile_off, prep,
                           rows, row0);
}

static __global__ void k_zero_queue(unsigned long long *q)
{
    if (threadIdx.x < NXCD) q[(size_t)threadIdx.x * QUEUE_STRIDE] = 0ull;
}

ItemParts split_items(const BandItem *items, int64_t n)
{
    // cut points at equal shares of the total list length
    int64_t total = 0;
    for (int64_t i = 0; i < n; ++i) total += items[i].hi - items[i].lo;
    ItemParts p{};
    int x = 1;
    int64_t acc = 0;
    for (int64_t i = 0; i < n && x < NXCD; ++i) {
        acc += items[i].hi - items[i].lo;
        while (x < NXCD && acc * NXCD >= total * x) p.lo[x++] = i + 1;
    }
    for (; x <= NXCD; ++x) p.lo[x] = n;
    return p;
}

void launch_band_queue(const BatchMap *maps, int32_t nmaps, const BandItem *items, int64_t nitems,
                       const ItemParts &parts, unsigned long long *queue, const int32_t *list, const BigPrep *prep,
                       const int64_t *rows, int64_t lds_doubles, hipStream_t st)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band_queue),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)(BAND_LDS_DOUBLES * sizeof(double)));
    MLM_HIP(attr);
    if (lds_doubles > BAND_LDS_DOUBLES) fail(MLM_EINVAL, "band of %lld doubles exceeds LDS", (long long)lds_doubles);
    if (nitems <= 0) return;
    if (parts.lo[0] != 0 || parts.lo[NXCD] != nitems) fail(MLM_EINVAL, "band item ranges do not cover the items");
    const size_t shmem = (size_t)lds_doubles * sizeof(double);
    // as many workgroups as the device holds at once at this LDS size
    const int64_t grid = resident_grid(reinterpret_cast<const void *>(&k_band_queue), BAND_THREADS, shmem, nitems);
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, queue);
    hipLaunchKernelGGL(k_band_queue, dim3((unsigned)grid), dim3(BAND_THREADS), shmem, st, maps, nmaps, items, parts,
                       queue, list, prep, rows);
}

void launch_band_queue1(const BandItem *items, int64_t nitems, const ItemParts &parts, unsigned long long *queue,
                        const int32_t *list, const BigPrep *prep, const int64_t *rows, int bh, const MapGeom &g,
                        double *map, unsigned long long *work, bool atomic_all, hipStream_t st)
{
    static const hipError_t attr = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_band_queue1),
                                                       hipFuncAttributeMaxDynamicSharedMemorySize,
                                                       (int)(BAND_LDS_DOUBLES * sizeof(double)));
    MLM_HIP(attr);
    if (nitems <= 0) return;
    if (parts.lo[0] != 0 || parts.lo[NXCD] != nitems) fail(MLM_EINVAL, "band item ranges do not cover the items");
    const size_t shmem = (size_t)bh * (size_t)g.n1 * sizeof(double);
    const int64_t grid = resident_grid(reinterpret_cast<const void *>(&k_band_queue1), BAND_THREADS, shmem, nitems);
    hipLaunchKernelGGL(k_zero_queue, dim3(1), dim3(64), 0, st, queue);
    hipLaunchKernelGGL(k_band_queue1, dim3((unsigned)grid), dim3(BAND_THREADS), shmem, st, items, parts, queue, list,
                       prep, rows, bh, g, map, work, atomic_all ? 1 : 0);
}

void launch_band_count_batch(const BatchMap *maps, int64_t nslices, const int32_t *slice_map, const int64_t *slice_lo,
                             int32_t max_bands, const int32_t *row0, const int64_t *rows, int32_t *count,
                             hipStream_t st)
{
    (void)hipGetLastError();   // clear what earlier calls left, so the check below sees this launch
    if (nslices > 0)
        hipLaunchKernelGGL(k_band_count_batch, dim3((unsigned)nslices), dim3(256),
                           band_hist_words(max_bands) * sizeof(int32_t), st, maps, slice_map, slice_lo, row0, rows,
                           count);
    MLM_HIP(hipGetLastError());
}

void launch_band_scatter_batch(const BatchMap *maps, int64_t nslices, const int32_t *slice_map,
                               const int64_t *slice_lo, int32_t max_bands, const int32_t *row0, const int64_t *rows,
                               unsigned long long *cursor, int32_t *list, hipStream_t st)
{
    const size_t shmem = bin_lds_bytes(max_bands);
    (void)hipGetLastError();   // clear what earlier calls left, so the check below sees this launch
    if (nslices > 0)
        hipLaunchKernelGGL(k_band_scatter_batch, dim3((unsigned)nslices), dim3(256), shmem, st, maps, slice_map,
                           slice_lo, row0, rows, cursor, list);
    MLM_HIP(hipGetLastError());
}


void launch_count_pieces(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                         unsigned long long *out, hipStream_t st)
{
    const int64_t ncells = (nr1 - 1) * (cb1 - cb0);
    if (ncells > 0)
        hipLaunchKernelGGL(k_count_pieces, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, st, verts, nr1, cb0,
                           ncells, vb0, g, out);
}

void launch_diff_rows(const MapGeom &g, const double *diff, double *map, hipStream_t st)
{
    hipLaunchKernelGGL(k_diff_rows, dim3((unsigned)g.n2), dim3(64), 0, st, g, diff, map);
}

}  // namespace mlm
