// Cell refinement and the network that predicts it.
//
// The paper apportions each ray-grid cell as two triangles (sec. 3.2); where
// the mapping is strongly curved (next to a star, across a caustic) that
// linear interpolation is coarse.  Plain refinement: a (sub)cell is refined
// if its mapped ears disagree in orientation (a critical curve crosses it) or
// if splitting it 2 x 2 changes its in-map deposits by more than tau times
// its image area (L1 over pixels); a refined cell is replaced by its four
// children, which are tested again down to `max_depth` levels; cells whose
// triangles span more than `window` pixels are left alone.  The map changes
// by (deposits of the leaves - deposits of the cell).
//
// The learned variant runs the test only on the cells a small network
// (12 -> 64 -> 64 -> 1, BF16 weights, FP32 accumulation on the matrix cores)
// flags from each cell's mapped corners and ear signs, plus every folded cell.
#include <algorithm>
#include <vector>

#include "cellfeat.hpp"
#include "colarea.hpp"
#include "shoot_dev.hpp"

namespace mlm {

namespace {

constexpr int RBLK = 64;

// A triangle of the refinement in coordinates local to (ou, ov), an integer
// point at or below its box (so the subtraction is exact): vertices, edge
// slopes and its deposit per unit of covered area, w / S (S its signed
// area; f = 0 for a degenerate or non-finite one, which deposits nothing).
// Its pixel areas are column sums (colarea.hpp): in pixel column i the area
// between rows j and j + 1 is H(j + 1 - ov) - H(j - ov), signed like S.
struct RTri {
    P2 T[3];
    double sv[3], su[3];
    double f;
};

__device__ inline RTri rtri(double u0, double v0, double u1, double v1, double u2, double v2, double ou, double ov,
                            double w)
{
    RTri t;
    const double S = 0.5 * area2(u0, v0, u1, v1, u2, v2);
    t.f = (S != 0.0 && isfinite(S)) ? w / S : 0.0;
    if (t.f == 0.0) return t;
    t.T[0] = P2{u0 - ou, v0 - ov};
    t.T[1] = P2{u1 - ou, v1 - ov};
    t.T[2] = P2{u2 - ou, v2 - ov};
    tri_slopes(t.T, t.sv, t.su);
    return t;
}

// rows per pass of a column's sums (registers hold one pass)
constexpr int RCH = 10;

// adds the deposits of triangle t in pixel column i, rows jc .. jc + nr - 1,
// to acc[0 .. nr)
__device__ inline void column_deposits(const RTri &t, int64_t i, int64_t jc, int nr, double ou, double ov,
                                       double (&acc)[RCH])
{
    if (t.f == 0.0) return;
    ColSegs<double> S;
    const double cl = (double)i - ou;
    col_segments(t.T, t.sv, t.su, cl, cl + 1.0, S);
    double h0 = col_cumulative(S, (double)jc - ov);
#pragma unroll
    for (int k = 0; k < RCH; ++k) {
        if (k < nr) {
            const double h1 = col_cumulative(S, (double)(jc + k + 1) - ov);
            acc[k] += t.f * (h1 - h0);
            h0 = h1;
        }
    }
}



struct RefineArgs {
    double x0, y0, d1, d2;
    LensConst lc;
    MapGeom g;
    int nlevels, L0_exp, p;
    double L0;
    const int32_t *child0, *leaf, *node_leaf;
    const LeafInfo *leaves;
    const double4 *near;
    const double2 *deriv;
    double tau;
    int max_depth, window;
};

// source position (pixel units) of image point (x0 + A d1, y0 + B d2)
__device__ inline void shoot_uv(const RefineArgs &ra, double A, double B, double &u, double &v)
{
    double x, y;
    {
#pragma clang fp contract(off)
        x = ra.x0 + A * ra.d1;
        y = ra.y0 + B * ra.d2;
    }
    const int64_t lf = find_leaf(x, y, ra.nlevels, ra.L0, ra.L0_exp, ra.child0, ra.leaf, ra.node_leaf);
    if (lf < 0) {
        u = v = nan("");
        return;
    }
    const LeafInfo li = ra.leaves[lf];
    double ax, ay;
    leaf_alpha<double>(x - li.cx, y - li.cy, li, ra.near + li.near_off, ra.deriv + lf * ra.p, ra.p, ax, ay);
    double w1, w2;
    double2 uv;
    finish_vertex(ra.lc, ra.g, x, y, ax, ay, w1, w2, uv);
    u = uv.x;
    v = uv.y;
}

// deposits of a (sub)cell's two triangles, times `sign`, into the map
__device__ inline void add_cell(const RefineArgs &ra, double *map, double w, const double *u4, const double *v4,
                                double sign)
{
#pragma unroll 1
    for (int k = 0; k < 2; ++k) {
        // triangle k of the cell: corners (0, 1, 2) or (0, 2, 3)
        const double tu[3] = {u4[0], k ? u4[2] : u4[1], k ? u4[3] : u4[2]};
        const double tv[3] = {v4[0], k ? v4[2] : v4[1], k ? v4[3] : v4[2]};
        bool ok = true;
#pragma unroll
        for (int m = 0; m < 3; ++m) ok = ok && isfinite(tu[m]) && isfinite(tv[m]);
        if (!ok) continue;
        const double fu = floor(fmin(tu[0], fmin(tu[1], tu[2]))), fv = floor(fmin(tv[0], fmin(tv[1], tv[2])));
        const int64_t i0 = max((int64_t)fu, (int64_t)0);
        const int64_t i1 = min((int64_t)floor(fmax(tu[0], fmax(tu[1], tu[2]))), (int64_t)ra.g.n1 - 1);
        const int64_t j0 = max((int64_t)fv, (int64_t)0);
        const int64_t j1 = min((int64_t)floor(fmax(tv[0], fmax(tv[1], tv[2]))), (int64_t)ra.g.n2 - 1);
        if (i0 > i1 || j0 > j1) continue;
        const RTri tri = rtri(tu[0], tv[0], tu[1], tv[1], tu[2], tv[2], fu, fv, sign * w);
        for (int64_t jc = j0; jc <= j1; jc += RCH) {
            const int nr = (int)min((int64_t)RCH, j1 - jc + 1);
            for (int64_t i = i0; i <= i1; ++i) {
                double d[RCH];
#pragma unroll
                for (int r = 0; r < RCH; ++r) d[r] = 0.0;
                column_deposits(tri, i, jc, nr, fu, fv, d);
#pragma unroll
                for (int r = 0; r < RCH; ++r)
                    if (r < nr && d[r] != 0.0) unsafeAtomicAdd(map + (jc + r) * (int64_t)ra.g.n1 + i, d[r]);
            }
        }
    }
}

struct SubCell {
    double A0, B0, h;
    int d;
    double u[4], v[4];
};

// The test of one subcell; fills its 3 x 3 grid of source points (corners
// from the subcell, five new rays) and returns whether it is refined.
// the subcell's 3 x 3 grid of source points: its corners and five new rays
__device__ inline void fill_grid(const RefineArgs &ra, const SubCell &c, double (&gu)[3][3], double (&gv)[3][3])
{
    gu[0][0] = c.u[0]; gv[0][0] = c.v[0];
    gu[0][2] = c.u[1]; gv[0][2] = c.v[1];
    gu[2][2] = c.u[2]; gv[2][2] = c.v[2];
    gu[2][0] = c.u[3]; gv[2][0] = c.v[3];
    const double hh = 0.5 * c.h;
    shoot_uv(ra, c.A0 + hh, c.B0, gu[0][1], gv[0][1]);
    shoot_uv(ra, c.A0, c.B0 + hh, gu[1][0], gv[1][0]);
    shoot_uv(ra, c.A0 + hh, c.B0 + hh, gu[1][1], gv[1][1]);
    shoot_uv(ra, c.A0 + c.h, c.B0 + hh, gu[1][2], gv[1][2]);
    shoot_uv(ra, c.A0 + hh, c.B0 + c.h, gu[2][1], gv[2][1]);
}

// triangle t of a refinement test: t = 0, 1 the (sub)cell's two, t = 2 ..
// 9 its four children's two each (child (r, s) of the 3 x 3 grid, t = 2 +
// 2 (2 r + s) + k), corners in the cell pass's order
__device__ inline void test_triangle(int t, const SubCell &c, const double (&gu)[3][3], const double (&gv)[3][3],
                                     double &a0, double &b0, double &a1, double &b1, double &a2, double &b2)
{
    switch (t) {
#define MLM_TRI(T, U0, V0, U1, V1, U2, V2) \
    case T: a0 = U0; b0 = V0; a1 = U1; b1 = V1; a2 = U2; b2 = V2; return;
        MLM_TRI(0, c.u[0], c.v[0], c.u[1], c.v[1], c.u[2], c.v[2])
        MLM_TRI(1, c.u[0], c.v[0], c.u[2], c.v[2], c.u[3], c.v[3])
        MLM_TRI(2, gu[0][0], gv[0][0], gu[0][1], gv[0][1], gu[1][1], gv[1][1])
        MLM_TRI(3, gu[0][0], gv[0][0], gu[1][1], gv[1][1], gu[1][0], gv[1][0])
        MLM_TRI(4, gu[0][1], gv[0][1], gu[0][2], gv[0][2], gu[1][2], gv[1][2])
        MLM_TRI(5, gu[0][1], gv[0][1], gu[1][2], gv[1][2], gu[1][1], gv[1][1])
        MLM_TRI(6, gu[1][0], gv[1][0], gu[1][1], gv[1][1], gu[2][1], gv[2][1])
        MLM_TRI(7, gu[1][0], gv[1][0], gu[2][1], gv[2][1], gu[2][0], gv[2][0])
        MLM_TRI(8, gu[1][1], gv[1][1], gu[1][2], gv[1][2], gu[2][2], gv[2][2])
        default: MLM_TRI(9, gu[1][1], gv[1][1], gu[2][2], gv[2][2], gu[2][1], gv[2][1])
#undef MLM_TRI
    }
}

__device__ inline bool refine_test(const RefineArgs &ra, const SubCell &c, double (&gu)[3][3], double (&gv)[3][3],
                                   int &too_large)
{
    fill_grid(ra, c, gu, gv);
    double umin = 1e300, umax = -1e300, vmin = 1e300, vmax = -1e300;
    bool finite = true;
    for (int r = 0; r < 3; ++r)
        for (int s = 0; s < 3; ++s) {
            finite = finite && isfinite(gu[r][s]) && isfinite(gv[r][s]);
            umin = fmin(umin, gu[r][s]);
            umax = fmax(umax, gu[r][s]);
            vmin = fmin(vmin, gv[r][s]);
            vmax = fmax(vmax, gv[r][s]);
        }
    if (!finite || !(umax - umin <= ra.window && vmax - vmin <= ra.window)) {
        too_large = 1;
        return false;
    }
    float f[12];
    cell_features(c.u, c.v, f);
    if (folded(f)) return true;
    const double w = ra.g.tri_weight * c.h * c.h;   // parent triangle weight
    const double ou = floor(umin), ov = floor(vmin);
    const int64_t i0 = max((int64_t)ou, (int64_t)0), i1 = min((int64_t)floor(umax), (int64_t)ra.g.n1 - 1);
    const int64_t j0 = max((int64_t)ov, (int64_t)0), j1 = min((int64_t)floor(vmax), (int64_t)ra.g.n2 - 1);
    // L1 over the in-map pixels of (children's deposits - the cell's): pixel
    // column by column, a pass of RCH rows at a time, one triangle after the
    // other (t uniform across the wavefront, so the vertex choice is a scalar
    // branch and only one triangle's column state is live)
    double l1 = 0.0;
    for (int64_t jc = j0; jc <= j1; jc += RCH) {
        const int nr = (int)min((int64_t)RCH, j1 - jc + 1);
        for (int64_t i = i0; i <= i1; ++i) {
            double diff[RCH];
#pragma unroll
            for (int k = 0; k < RCH; ++k) diff[k] = 0.0;
#pragma unroll 1
            for (int t = 0; t < 10; ++t) {
                double a0, b0, a1, b1, a2, b2;
                test_triangle(t, c, gu, gv, a0, b0, a1, b1, a2, b2);
                column_deposits(rtri(a0, b0, a1, b1, a2, b2, ou, ov, t < 2 ? -w : 0.25 * w), i, jc, nr, ou, ov,
                                diff);
            }
#pragma unroll
            for (int k = 0; k < RCH; ++k)
                if (k < nr) l1 += fabs(diff[k]);
        }
    }
    return l1 > ra.tau * 2.0 * w;
}

// Refinement level by level (breadth first): every (sub)cell of a level is
// one thread of k_refine_test, which only decides; the few refined ones are
// numbered by a scan and expanded by k_refine_expand, which moves their
// deposits to their four children and lists the children for the next
// level.  Lanes of a wavefront so do equal work, where one thread walking a
// cell's whole subtree kept the other lanes waiting.
//
// A level's items are either candidate cells (cand: a + (nr1 - 1) b, corners
// from the strip's vertices) or a list of subcells.
__device__ inline SubCell level_item(int64_t t, const int64_t *__restrict__ cand, const SubCell *__restrict__ list,
                                     int64_t nr1, int64_t vb0, const double2 *__restrict__ verts)
{
    if (list) return list[t];
    SubCell c;
    const int64_t cell = cand[t];
    const int64_t a = cell % (nr1 - 1), b = cell / (nr1 - 1);
    c.A0 = (double)a;
    c.B0 = (double)b;
    c.h = 1.0;
    c.d = 0;
    const double2 *r0 = verts + (b - vb0) * nr1, *r1 = r0 + nr1;
    const double2 q[4] = {r0[a], r0[a + 1], r1[a + 1], r1[a]};
    for (int m = 0; m < 4; ++m) {
        c.u[m] = q[m].x;
        c.v[m] = q[m].y;
    }
    return c;
}

// flag[t] = the item is refined (and label[t] too, for candidate cells);
// stats: [0] tested, [1] refined, [2] too large (one atomic per wavefront each)
// (at most 168 registers, three waves per SIMD, a few bytes spilled: the
// compiler's 173 held two, and the test is latency-bound on its rays' loads)
__global__ __launch_bounds__(RBLK) __attribute__((amdgpu_waves_per_eu(3))) void k_refine_test(RefineArgs ra, int64_t n, const int64_t *__restrict__ cand,
                                                      const SubCell *__restrict__ list, int64_t nr1, int64_t vb0,
                                                      const double2 *__restrict__ verts, int32_t *__restrict__ flag,
                                                      uint8_t *__restrict__ label,
                                                      unsigned long long *__restrict__ stats)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int refine = 0, large = 0, tested = 0;
    if (t < n) {
        const SubCell c = level_item(t, cand, list, nr1, vb0, verts);
        double gu[3][3], gv[3][3];
        refine = refine_test(ra, c, gu, gv, large) ? 1 : 0;
        tested = 1;
        flag[t] = refine;
        if (label) label[t] = (uint8_t)refine;
    }
    if (stats) {
        int v[3] = {tested, refine, large};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
            if ((threadIdx.x & 63) == 0 && v[k]) atomicAdd(stats + k, (unsigned long long)v[k]);
        }
    }
}

// the refined items (flag[t]; pos: exclusive scan of the flags): the map
// loses the item's deposits and gains its four children's, and the children
// are written to out[4 pos[t] .. 4 pos[t] + 3]
__global__ __launch_bounds__(RBLK) void k_refine_expand(RefineArgs ra, int64_t n, const int64_t *__restrict__ cand,
                                                        const SubCell *__restrict__ list, int64_t nr1, int64_t vb0,
                                                        const double2 *__restrict__ verts,
                                                        const int32_t *__restrict__ flag,
                                                        const int64_t *__restrict__ pos, double *__restrict__ map,
                                                        SubCell *__restrict__ out)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n || !flag[t]) return;
    const SubCell c = level_item(t, cand, list, nr1, vb0, verts);
    double gu[3][3], gv[3][3];
    fill_grid(ra, c, gu, gv);
    const double w = ra.g.tri_weight * c.h * c.h;
    if (map) add_cell(ra, map, w, c.u, c.v, -1.0);
    const double hh = 0.5 * c.h;
    SubCell *dst = out + 4 * pos[t];
#pragma unroll
    for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
            SubCell ch;
            ch.A0 = c.A0 + s * hh;
            ch.B0 = c.B0 + r * hh;
            ch.h = hh;
            ch.d = c.d + 1;
            const double cu[4] = {gu[r][s], gu[r][s + 1], gu[r + 1][s + 1], gu[r + 1][s]};
            const double cv[4] = {gv[r][s], gv[r][s + 1], gv[r + 1][s + 1], gv[r + 1][s]};
            for (int m = 0; m < 4; ++m) {
                ch.u[m] = cu[m];
                ch.v[m] = cv[m];
            }
            if (map) add_cell(ra, map, 0.25 * w, ch.u, ch.v, +1.0);   // a refined child takes it back itself
            dst[2 * r + s] = ch;
        }
}

// features of arbitrary cells, corners shot on the spot
__global__ __launch_bounds__(RBLK) void k_sample_features(RefineArgs ra, int64_t n, const int64_t *__restrict__ ab,
                                                          float *__restrict__ feats)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const double A = (double)ab[2 * t], B = (double)ab[2 * t + 1];
    double u4[4], v4[4];
    shoot_uv(ra, A, B, u4[0], v4[0]);
    shoot_uv(ra, A + 1.0, B, u4[1], v4[1]);
    shoot_uv(ra, A + 1.0, B + 1.0, u4[2], v4[2]);
    shoot_uv(ra, A, B + 1.0, u4[3], v4[3]);
    float f[12];
    cell_features(u4, v4, f);
    for (int m = 0; m < 12; ++m) feats[t * 12 + m] = isfinite(f[m]) ? f[m] : 0.0f;
}

// the refinement test at depth 0 of arbitrary cells (labels only)
__global__ __launch_bounds__(RBLK) __attribute__((amdgpu_waves_per_eu(3))) void k_sample_labels(RefineArgs ra, int64_t n, const int64_t *__restrict__ ab,
                                                        uint8_t *__restrict__ label)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    SubCell c;
    c.A0 = (double)ab[2 * t];
    c.B0 = (double)ab[2 * t + 1];
    c.h = 1.0;
    c.d = 0;
    shoot_uv(ra, c.A0, c.B0, c.u[0], c.v[0]);
    shoot_uv(ra, c.A0 + 1.0, c.B0, c.u[1], c.v[1]);
    shoot_uv(ra, c.A0 + 1.0, c.B0 + 1.0, c.u[2], c.v[2]);
    shoot_uv(ra, c.A0, c.B0 + 1.0, c.u[3], c.v[3]);
    double gu[3][3], gv[3][3];
    int large = 0;
    label[t] = refine_test(ra, c, gu, gv, large) ? 1 : 0;
}

// cand[pos[t]] = base + t for flagged t (pos: exclusive scan of the flags,
// pos[t + 1] - pos[t] = flag[t]); with flag == NULL every t
__global__ __launch_bounds__(256) void k_compact(int64_t n, const int32_t *__restrict__ flag,
                                                 const int64_t *__restrict__ pos, int64_t base,
                                                 int64_t *__restrict__ cand)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    if (!flag) cand[t] = base + t;
    else if (flag[t]) cand[pos[t]] = base + t;
}

}  // namespace

RefineArgs make_refine_args(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau,
                            int max_depth, int window)
{
    RefineArgs ra{};
    ra.x0 = R.x0;
    ra.y0 = R.y0;
    ra.d1 = R.d1;
    ra.d2 = R.d2;
    ra.lc = lc;
    ra.g = g;
    ra.nlevels = T.nlevels;
    ra.L0_exp = T.L0_exp;
    ra.p = T.p;
    ra.L0 = T.L0;
    ra.child0 = T.child0;
    ra.leaf = T.leaf;
    ra.node_leaf = T.node_leaf;
    ra.leaves = T.leaves;
    ra.near = T.near;
    ra.deriv = T.deriv;
    ra.tau = tau;
    ra.max_depth = max_depth;
    ra.window = window;
    return ra;
}

size_t refine_subcell_bytes() { return sizeof(SubCell); }

void launch_refine_test(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau, int depth,
                        int window, int64_t n, const int64_t *cand, const void *list, int64_t nr1, int64_t vb0,
                        const double2 *verts, int32_t *flag, uint8_t *label, unsigned long long *stats, hipStream_t st)
{
    if (n <= 0) return;
    const RefineArgs ra = make_refine_args(T, R, lc, g, tau, depth, window);
    hipLaunchKernelGGL(k_refine_test, dim3((unsigned)((n + RBLK - 1) / RBLK)), dim3(RBLK), 0, st, ra, n, cand,
                       static_cast<const SubCell *>(list), nr1, vb0, verts, flag, label, stats);
}

void launch_refine_expand(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau, int depth,
                          int window, int64_t n, const int64_t *cand, const void *list, int64_t nr1, int64_t vb0,
                          const double2 *verts, const int32_t *flag, const int64_t *pos, double *map, void *out,
                          hipStream_t st)
{
    if (n <= 0) return;
    const RefineArgs ra = make_refine_args(T, R, lc, g, tau, depth, window);
    hipLaunchKernelGGL(k_refine_expand, dim3((unsigned)((n + RBLK - 1) / RBLK)), dim3(RBLK), 0, st, ra, n, cand,
                       static_cast<const SubCell *>(list), nr1, vb0, verts, flag, pos, map,
                       static_cast<SubCell *>(out));
}

void launch_sample_features(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, int64_t n,
                            const int64_t *ab, float *feats, hipStream_t st)
{
    if (n <= 0) return;
    const RefineArgs ra = make_refine_args(T, R, lc, g, 0.0, 1, 1);
    hipLaunchKernelGGL(k_sample_features, dim3((unsigned)((n + RBLK - 1) / RBLK)), dim3(RBLK), 0, st, ra, n, ab,
                       feats);
}

void launch_sample_labels(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau,
                          int window, int64_t n, const int64_t *ab, uint8_t *label, hipStream_t st)
{
    if (n <= 0) return;
    const RefineArgs ra = make_refine_args(T, R, lc, g, tau, 1, window);
    hipLaunchKernelGGL(k_sample_labels, dim3((unsigned)((n + RBLK - 1) / RBLK)), dim3(RBLK), 0, st, ra, n, ab, label);
}

void launch_compact(int64_t n, const int32_t *flag, const int64_t *pos, int64_t base, int64_t *cand, hipStream_t st)
{
    if (n > 0)
        hipLaunchKernelGGL(k_compact, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n, flag, pos, base, cand);
}

}  // namespace mlm
