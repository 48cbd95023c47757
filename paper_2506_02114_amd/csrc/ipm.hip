// Inverse polygon mapping (sec. 3.2): every grid cell is split into two
// triangles; each mapped triangle's image-plane area is apportioned among the
// source pixels it covers, in proportion to (triangle n pixel) / triangle.
//
// A triangle is cut along pixel columns, and each column piece along pixel
// rows, as in the paper's column-then-row clipping.  The clipping keeps a
// fixed number of vertex slots: each polygon edge is clipped to the strip by
// its parameter interval (Liang-Barsky), and an edge entirely outside the
// strip is replaced by a repeat of the previous exit point.  For a convex
// polygon the gaps so closed run along the strip's boundary lines, so the
// slots trace exactly the clipped polygon, with every index known at compile
// time (no dynamically indexed arrays, nothing spilled to scratch).
//
// Triangles next to a star map to huge triangles (the linear interpolation
// of a singular mapping), covering up to millions of pixels.  Their cost is
// made proportional to their perimeter instead of their area: they are queued
// and processed one (triangle, pixel row) per thread; in each row only the
// pixels on the triangle's boundary are clipped, and the run of fully covered
// pixels between them is recorded as two entries of a per-row difference
// buffer, whose prefix sums are added to the map at the end.
#include "dev.hpp"

namespace mlm {

namespace {

struct P2 {
    double u, v;
};

constexpr int64_t BIG_PIXELS = 48;   // bounding-box pixels above which a triangle is queued

struct BigQueue {
    BigTri *tri;
    unsigned long long *count;
    unsigned long long cap;
};

__device__ inline P2 lerp2(P2 P, P2 Q, double t)
{
    if (t == 0.0) return P;
    if (t == 1.0) return Q;
    return P2{P.u + t * (Q.u - P.u), P.v + t * (Q.v - P.v)};
}

// part of segment P->Q with lo <= coordinate <= hi (AXIS 0: u, 1: v)
template <int AXIS>
__device__ inline bool clip_seg(P2 P, P2 Q, double lo, double hi, P2 &E, P2 &X)
{
    const double p = AXIS ? P.v : P.u, q = AXIS ? Q.v : Q.u;
    if (p == q) {
        if (p < lo || p > hi) return false;
        E = P;
        X = Q;
        return true;
    }
    const double inv = 1.0 / (q - p);
    const double ta = (lo - p) * inv, tb = (hi - p) * inv;
    double tin, tout, bin, bout;
    if (q > p) {
        tin = ta; bin = lo; tout = tb; bout = hi;
    } else {
        tin = tb; bin = hi; tout = ta; bout = lo;
    }
    const bool cut_in = tin > 0.0, cut_out = tout < 1.0;
    if (!cut_in) tin = 0.0;
    if (!cut_out) tout = 1.0;
    if (tin > tout) return false;
    E = lerp2(P, Q, tin);
    X = lerp2(P, Q, tout);
    if (cut_in) { if (AXIS) E.v = bin; else E.u = bin; }
    if (cut_out) { if (AXIS) X.v = bout; else X.u = bout; }
    return true;
}

// polygon of N slots clipped to a strip -> 2N slots; false if empty
template <int AXIS, int N>
__device__ inline bool clip_poly(const P2 (&in)[N], double lo, double hi, P2 (&out)[2 * N])
{
    P2 E[N], X[N];
    bool ok[N];
    bool any = false;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        ok[k] = clip_seg<AXIS>(in[k], in[(k + 1) % N], lo, hi, E[k], X[k]);
        any = any || ok[k];
    }
    if (!any) return false;
    P2 carry = in[0];
#pragma unroll
    for (int k = 0; k < N; ++k)
        if (ok[k]) carry = X[k];     // exit point of the last non-empty edge
#pragma unroll
    for (int k = 0; k < N; ++k) {
        if (ok[k]) {
            out[2 * k] = E[k];
            out[2 * k + 1] = X[k];
            carry = X[k];
        } else {
            out[2 * k] = carry;
            out[2 * k + 1] = carry;
        }
    }
    return true;
}

// twice the signed area (shoelace), coordinates taken relative to (ou, ov)
template <int N>
__device__ inline double shoelace2(const P2 (&p)[N], double ou, double ov)
{
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        const double x1 = p[k].u - ou, y1 = p[k].v - ov;
        const double x2 = p[(k + 1) % N].u - ou, y2 = p[(k + 1) % N].v - ov;
        s += x1 * y2 - x2 * y1;
    }
    return s;
}

__device__ inline void deposit(double *map, const MapGeom &g, int64_t i, int64_t j, double val)
{
    unsafeAtomicAdd(map + j * (int64_t)g.n1 + i, val);
}

// apportion one triangle (pixel coordinates); weight = its image area / pixel area.
// Triangles whose bounding box within the map exceeds BIG_PIXELS go to the
// big-triangle queue (unless it is full).
__device__ void apportion(P2 A, P2 B, P2 C, double weight, const MapGeom &g, double *map,
                          unsigned long long *counters, BigQueue q)
{
    if (!(isfinite(A.u) && isfinite(A.v) && isfinite(B.u) && isfinite(B.v) && isfinite(C.u) && isfinite(C.v))) {
        atomicAdd(counters, 1ull);
        return;
    }
    const double umin = fmin(A.u, fmin(B.u, C.u)), umax = fmax(A.u, fmax(B.u, C.u));
    const double vmin = fmin(A.v, fmin(B.v, C.v)), vmax = fmax(A.v, fmax(B.v, C.v));
    const double fu0 = floor(umin), fu1 = floor(umax), fv0 = floor(vmin), fv1 = floor(vmax);
    // entirely outside the map
    if (fu1 < 0.0 || fv1 < 0.0 || fu0 > (double)(g.n1 - 1) || fv0 > (double)(g.n2 - 1)) return;
    if (fu0 == fu1 && fv0 == fv1) {
        deposit(map, g, (int64_t)fu0, (int64_t)fv0, weight);
        return;
    }
    // local coordinates relative to the bounding box's lower-left pixel corner
    const P2 T[3] = {P2{A.u - fu0, A.v - fv0}, P2{B.u - fu0, B.v - fv0}, P2{C.u - fu0, C.v - fv0}};
    const double S2 = (T[1].u - T[0].u) * (T[2].v - T[0].v) - (T[2].u - T[0].u) * (T[1].v - T[0].v);
    if (S2 == 0.0) {
        // no source-plane area: the whole image area goes to the centroid's pixel
        const double cu = (A.u + B.u + C.u) / 3.0, cv = (A.v + B.v + C.v) / 3.0;
        const double fi = floor(cu), fj = floor(cv);
        if (fi >= 0.0 && fj >= 0.0 && fi <= (double)(g.n1 - 1) && fj <= (double)(g.n2 - 1))
            deposit(map, g, (int64_t)fi, (int64_t)fj, weight);
        return;
    }
    const double scale = weight / S2;
    const int64_t i0 = (int64_t)fmax(fu0, 0.0), i1 = (int64_t)fmin(fu1, (double)(g.n1 - 1));
    const int64_t j0 = (int64_t)fmax(fv0, 0.0), j1 = (int64_t)fmin(fv1, (double)(g.n2 - 1));
    if ((i1 - i0 + 1) * (j1 - j0 + 1) > BIG_PIXELS) {
        unsigned long long k = atomicAdd(q.count, 1ull);
        if (k < q.cap) {
            q.tri[k] = BigTri{A.u, A.v, B.u, B.v, C.u, C.v};
            return;
        }
        atomicAdd(counters + 3, 1ull);   // queue full: apportion here
    }
    for (int64_t i = i0; i <= i1; ++i) {
        const double cl = (double)i - fu0;
        P2 col[6];
        if (!clip_poly<0, 3>(T, cl, cl + 1.0, col)) continue;
        double cvmin = col[0].v, cvmax = col[0].v;
#pragma unroll
        for (int k = 1; k < 6; ++k) {
            cvmin = fmin(cvmin, col[k].v);
            cvmax = fmax(cvmax, col[k].v);
        }
        const double gj0 = floor(cvmin), gj1 = floor(cvmax);
        if (gj0 == gj1) {
            const int64_t j = (int64_t)gj0 + (int64_t)fv0;
            if (j >= j0 && j <= j1) deposit(map, g, i, j, scale * shoelace2(col, cl, gj0));
            continue;
        }
        const int64_t ja = (int64_t)fmax(gj0 + fv0, (double)j0), jb = (int64_t)fmin(gj1 + fv0, (double)j1);
        for (int64_t j = ja; j <= jb; ++j) {
            const double rl = (double)j - fv0;
            P2 piece[12];
            if (!clip_poly<1, 6>(col, rl, rl + 1.0, piece)) continue;
            const double a2 = shoelace2(piece, cl, rl);
            if (a2 != 0.0) deposit(map, g, i, j, scale * a2);
        }
    }
}

// one thread per grid cell of cell rows [cb0, cb1)
__global__ __launch_bounds__(256) void k_ipm(const double2 *__restrict__ verts, int64_t nr1, int64_t cb0,
                                             int64_t ncells, int64_t vb0, MapGeom g, double *__restrict__ map,
                                             unsigned long long *__restrict__ counters, BigQueue q)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncells) return;
    const int64_t ncol = nr1 - 1;
    const int64_t a = t % ncol, b = cb0 + t / ncol;
    const double2 *r0 = verts + (b - vb0) * nr1, *r1 = r0 + nr1;
    const double2 q00 = r0[a], q10 = r0[a + 1], q01 = r1[a], q11 = r1[a + 1];
    const P2 v00{q00.x, q00.y}, v10{q10.x, q10.y}, v11{q11.x, q11.y}, v01{q01.x, q01.y};
    // both triangles inside one pixel: one deposit for the cell
    const double fu = floor(v00.u), fv = floor(v00.v);
    if (floor(v10.u) == fu && floor(v11.u) == fu && floor(v01.u) == fu && floor(v10.v) == fv &&
        floor(v11.v) == fv && floor(v01.v) == fv) {
        if (fu >= 0.0 && fv >= 0.0 && fu <= (double)(g.n1 - 1) && fv <= (double)(g.n2 - 1))
            deposit(map, g, (int64_t)fu, (int64_t)fv, 2.0 * g.tri_weight);
        return;
    }
    // T1 = (v00, v10, v11), T2 = (v00, v11, v01): split along v00-v11
    apportion(v00, v10, v11, g.tri_weight, g, map, counters, q);
    apportion(v00, v11, v01, g.tri_weight, g, map, counters, q);
}

// pixel rows of each queued triangle inside the map
__global__ void k_big_rows(int64_t nq, const BigTri *__restrict__ tri, MapGeom g, int64_t *__restrict__ rows)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nq) return;
    const BigTri t = tri[k];
    const double vmin = fmin(t.v0, fmin(t.v1, t.v2)), vmax = fmax(t.v0, fmax(t.v1, t.v2));
    const double j0 = fmax(floor(vmin), 0.0), j1 = fmin(floor(vmax), (double)(g.n2 - 1));
    rows[k] = j1 >= j0 ? (int64_t)(j1 - j0) + 1 : 0;
}

// one (queued triangle, pixel row) per thread
__global__ __launch_bounds__(256) void k_big_apportion(int64_t total, int64_t nq, const int64_t *__restrict__ row_off,
                                                       const BigTri *__restrict__ tri, MapGeom g,
                                                       double *__restrict__ map, double *__restrict__ diff)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= total) return;
    const int64_t k = upper_bound_i64<int64_t>(row_off, nq, t) - 1;
    const BigTri bt = tri[k];
    const double umin = fmin(bt.u0, fmin(bt.u1, bt.u2)), vmin = fmin(bt.v0, fmin(bt.v1, bt.v2));
    // integer local origin inside or at the edge of the map: exact pixel boundaries nearby
    const double ou = fmax(floor(umin), 0.0), ov = fmax(floor(vmin), 0.0);
    const int64_t j = (int64_t)ov + (t - row_off[k]);
    P2 T[3] = {P2{bt.u0 - ou, bt.v0 - ov}, P2{bt.u1 - ou, bt.v1 - ov}, P2{bt.u2 - ou, bt.v2 - ov}};
    double S2 = (T[1].u - T[0].u) * (T[2].v - T[0].v) - (T[2].u - T[0].u) * (T[1].v - T[0].v);
    if (S2 < 0.0) {   // counter-clockwise order: interior to the left of every edge
        const P2 tmp = T[1];
        T[1] = T[2];
        T[2] = tmp;
        S2 = -S2;
    }
    const double scale = g.tri_weight / S2;   // deposit = scale * (twice the piece area)
    const double rl = (double)j - ov;
    P2 row[6];
    if (!clip_poly<1, 3>(T, rl, rl + 1.0, row)) return;
    double rumin = row[0].u, rumax = row[0].u;
#pragma unroll
    for (int m = 1; m < 6; ++m) {
        rumin = fmin(rumin, row[m].u);
        rumax = fmax(rumax, row[m].u);
    }
    const double ga = fmax(floor(rumin), -ou), gb = fmin(floor(rumax), (double)(g.n1 - 1) - ou);
    if (ga > gb) return;
    // pixels of this row fully inside the triangle: every corner on the inner
    // side of each edge (local pixel indices)
    double fa = -1e300, fb = 1e300;
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        const P2 P = T[m], Q = T[(m + 1) % 3];
        const double dx = Q.u - P.u, dy = Q.v - P.v;
        const double vc = dx > 0.0 ? rl : rl + 1.0;
        const double base = dx * (vc - P.v);
        if (dy > 0.0) fb = fmin(fb, floor(P.u - 1.0 + base / dy));
        else if (dy < 0.0) fa = fmax(fa, ceil(P.u - base / (-dy)));
        else if (base < 0.0) fa = 1e300;
    }
    fa = fmax(fa, ga);
    fb = fmin(fb, gb);
    const bool has_full = fa <= fb;
    const int64_t ia = (int64_t)ga, ib = (int64_t)gb;
    const int64_t pa = has_full ? (int64_t)fa : ib + 1, pb = has_full ? (int64_t)fb : ib;
    // boundary pixels: exact clip of the row polygon to the pixel column
    for (int64_t i = ia; i <= ib; ++i) {
        if (i == pa && has_full) {
            i = pb;
            continue;
        }
        const double cl = (double)i;
        P2 piece[12];
        if (!clip_poly<0, 6>(row, cl, cl + 1.0, piece)) continue;
        const double a2 = shoelace2(piece, cl, rl);
        if (a2 != 0.0) deposit(map, g, i + (int64_t)ou, j, scale * a2);
    }
    if (has_full) {
        double *dr = diff + j * (int64_t)(g.n1 + 1) + (int64_t)ou;
        unsafeAtomicAdd(dr + pa, 2.0 * scale);
        unsafeAtomicAdd(dr + pb + 1, -2.0 * scale);
    }
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

}  // namespace

void launch_ipm(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                double *map, unsigned long long *counters, BigTri *queue, int64_t queue_cap, hipStream_t st)
{
    int64_t ncells = (nr1 - 1) * (cb1 - cb0);
    if (ncells <= 0) return;
    BigQueue q{queue, counters + 4, (unsigned long long)queue_cap};
    hipLaunchKernelGGL(k_ipm, dim3((unsigned)((ncells + 255) / 256)), dim3(256), 0, st, verts, nr1, cb0, ncells, vb0,
                       g, map, counters, q);
}

void launch_big_rows(int64_t nq, const BigTri *tri, const MapGeom &g, int64_t *rows, hipStream_t st)
{
    if (nq > 0) hipLaunchKernelGGL(k_big_rows, dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, st, nq, tri, g, rows);
}

void launch_big_apportion(int64_t total_rows, int64_t nq, const int64_t *row_off, const BigTri *tri, const MapGeom &g,
                          double *map, double *diff, hipStream_t st)
{
    if (total_rows > 0)
        hipLaunchKernelGGL(k_big_apportion, dim3((unsigned)((total_rows + 255) / 256)), dim3(256), 0, st, total_rows,
                           nq, row_off, tri, g, map, diff);
}

void launch_diff_rows(const MapGeom &g, const double *diff, double *map, hipStream_t st)
{
    hipLaunchKernelGGL(k_diff_rows, dim3((unsigned)g.n2), dim3(64), 0, st, g, diff, map);
}

}  // namespace mlm
