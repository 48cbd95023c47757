// Ray shooting (sec. 2.2, 3.3): the source position of every ray-grid vertex,
//   w = (1-kappa) z + gamma conj(z) - a_*(z) - a_s(z),
// with a_* = (near field summed directly over the stars of the vertex's leaf
// and its neighbours) + conj(d/dz of the leaf's Taylor series).
//
// Work is leaf-major: the grid vertices inside each leaf form a rectangle,
// cut into 8 x 8 tiles; one 64-lane wavefront shoots one tile.  All lanes of a
// wavefront share the leaf, so the near stars and the Taylor coefficients are
// wavefront-uniform and are read through the scalar cache into SGPRs.
#include <algorithm>

#include "shoot_dev.hpp"

namespace mlm {

int64_t scan_total_public(mlm_lens *lens, const int32_t *in, int32_t *out, int64_t n, hipStream_t st);

namespace {

constexpr int BLK = 256;
inline unsigned nblocks(int64_t n, int b = BLK) { return (unsigned)((n + b - 1) / b); }

// first a in [lo, hi) whose lattice point lies in square index >= target at level lev
__device__ inline int64_t first_in_cell(double x0, double d, double h, int64_t lo, int64_t hi, double L0,
                                        double scale_lev, int lev, int64_t target)
{
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (level_cell(grid_pos(x0, d, mid, h), L0, scale_lev, lev) < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// lattice columns and rows (within rows [vb0, vb1)) inside each leaf
__global__ void k_tile_counts(int64_t nleaves, const int32_t *__restrict__ leaf_node,
                              const uint64_t *__restrict__ code, const int32_t *__restrict__ level, double L0,
                              int L0_exp, double x0, double d1, int64_t nr1, double y0, double d2, int64_t vb0,
                              int64_t vb1, double h, LeafInfo *__restrict__ info, int32_t *__restrict__ cnt)
{
    int64_t lf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves) return;
    int32_t q = leaf_node[lf];
    int lev = level[q];
    uint64_t c = code[q];
    int64_t i = compact_bits(c), j = compact_bits(c >> 1);
    double scale = ldexp(1.0, lev - L0_exp);   // 2^lev / (2 L0)
    int64_t a0 = first_in_cell(x0, d1, h, 0, nr1, L0, scale, lev, i);
    int64_t a1 = first_in_cell(x0, d1, h, a0, nr1, L0, scale, lev, i + 1);
    int64_t b0 = first_in_cell(y0, d2, h, vb0, vb1, L0, scale, lev, j);
    int64_t b1 = first_in_cell(y0, d2, h, b0, vb1, L0, scale, lev, j + 1);
    LeafInfo &li = info[lf];
    li.a_lo = (int32_t)a0;
    li.na = (int32_t)(a1 - a0);
    li.b_lo = (int32_t)b0;
    li.nb = (int32_t)(b1 - b0);
    li.ntx = (li.na + TILE - 1) / TILE;
    int32_t nty = (li.nb + TILE - 1) / TILE;
    cnt[lf] = (li.na > 0 && li.nb > 0) ? li.ntx * nty : 0;
}

__global__ void k_tile_leaf(int64_t ntiles, int64_t nleaves, const int32_t *__restrict__ tile_off,
                            int32_t *__restrict__ tile_leaf)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ntiles) return;
    tile_leaf[t] = (int32_t)(upper_bound_i64<int32_t>(tile_off, nleaves, (int32_t)t) - 1);
}


// the lattice point of tile t's lane: its leaf and position, and whether it
// exists (the tile may overhang the leaf's rectangle)
struct TilePoint {
    int32_t lf;
    int64_t a, b;
    double x, y;
    bool valid;
};

__device__ inline TilePoint tile_point(const ShootArgs &sa, const int32_t *__restrict__ tile_leaf,
                                       const int32_t *__restrict__ tile_off, const LeafInfo &li, int32_t lf,
                                       int64_t t, int lane)
{
    const int32_t local = (int32_t)t - tile_off[lf];
    const int32_t ty = local / li.ntx, tx = local - ty * li.ntx;
    const int32_t ia = tx * TILE + (lane & (TILE - 1)), ib = ty * TILE + (lane >> 3);
    TilePoint pt;
    pt.lf = lf;
    pt.valid = ia < li.na && ib < li.nb;
    pt.a = li.a_lo + ia;
    pt.b = li.b_lo + ib;
    pt.x = grid_pos(sa.x0, sa.d1, pt.a, sa.h);
    pt.y = grid_pos(sa.y0, sa.d2, pt.b, sa.h);
    return pt;
}

// inverse ray shooting of tile t (one wavefront per 8 x 8 tile of cell
// centres): every ray counted in its pixel
template <class R>
__global__ __launch_bounds__(64) void k_shoot_irs(ShootArgs sa, LensConst lc, MapGeom g,
                                                  const int32_t *__restrict__ tile_leaf,
                                                  const int32_t *__restrict__ tile_off,
                                                  const LeafInfo *__restrict__ leaves,
                                                  const double4 *__restrict__ near,
                                                  const typename Cx<R>::c2 *__restrict__ deriv,
                                                  unsigned long long *__restrict__ counts)
{
    const int64_t t = blockIdx.x;
    const int32_t lf = tile_leaf[t];
    const LeafInfo li = leaves[lf];
    const TilePoint pt = tile_point(sa, tile_leaf, tile_off, li, lf, t, threadIdx.x);
    double ax, ay;
    leaf_alpha<R>(pt.x - li.cx, pt.y - li.cy, li, near + li.near_off, deriv + (int64_t)lf * sa.p, sa.p, ax, ay);
    double w1, w2;
    double2 uv;
    finish_vertex(lc, g, pt.x, pt.y, ax, ay, w1, w2, uv);
    irs_count(pt.valid, uv, g, counts);
}

// shoot tile t of a map (one 64-lane wavefront per 8 x 8 tile, a workgroup
// of its own); STAGED: the leaf's near stars and coefficients through LDS
// (leaf_alpha_tile), else through the scalar cache
template <class R, bool STAGED = false>
__device__ inline void shoot_tile(const ShootArgs &sa, const LensConst &lc, const MapGeom &g,
                                  const int32_t *__restrict__ tile_leaf, const int32_t *__restrict__ tile_off,
                                  const LeafInfo *__restrict__ leaves, const double4 *__restrict__ near,
                                  const typename Cx<R>::c2 *__restrict__ deriv, double2 *__restrict__ verts,
                                  double2 *__restrict__ w_out, int64_t t, int lane)
{
    const int32_t lf = tile_leaf[t];
    const LeafInfo li = leaves[lf];
    const int32_t local = (int32_t)t - tile_off[lf];
    const int32_t ty = local / li.ntx, tx = local - ty * li.ntx;
    const int32_t ia = tx * TILE + (lane & (TILE - 1)), ib = ty * TILE + (lane >> 3);
    const bool valid = ia < li.na && ib < li.nb;
    const int64_t a = li.a_lo + ia, b = li.b_lo + ib;
    const double x = grid_pos(sa.x0, sa.d1, a), y = grid_pos(sa.y0, sa.d2, b);
    double ax, ay;
    if constexpr (STAGED) {
        __shared__ LeafLds<R> S;   // the workgroup is this one wavefront
        leaf_alpha_tile<R>(x - li.cx, y - li.cy, li, near + li.near_off, deriv + (int64_t)lf * sa.p, sa.p, ax, ay, S);
    } else {
        leaf_alpha<R>(x - li.cx, y - li.cy, li, near + li.near_off, deriv + (int64_t)lf * sa.p, sa.p, ax, ay);
    }
    double w1, w2;
    double2 uv;
    finish_vertex(lc, g, x, y, ax, ay, w1, w2, uv);
    if (valid) {
        const int64_t o = (b - sa.vb0) * sa.nr1 + a;
        verts[o] = uv;
        if (w_out) w_out[o] = make_double2(w1, w2);
    }
}

template <class R>
__global__ __launch_bounds__(64) void k_shoot(ShootArgs sa, LensConst lc, MapGeom g,
                                              const int32_t *__restrict__ tile_leaf,
                                              const int32_t *__restrict__ tile_off,
                                              const LeafInfo *__restrict__ leaves,
                                              const double4 *__restrict__ near,
                                              const typename Cx<R>::c2 *__restrict__ deriv,
                                              double2 *__restrict__ verts, double2 *__restrict__ w_out)
{
    shoot_tile<R>(sa, lc, g, tile_leaf, tile_off, leaves, near, deriv, verts, w_out, blockIdx.x, threadIdx.x);
}

// the same with the leaf's stars and coefficients staged through LDS, for
// maps of few tiles per leaf: there a tile's scalar loads of its leaf's stars
// mostly miss the scalar cache, and waiting on them a few stars at a time
// cost more than one vector load of 64 (on the 1e5-star map: shooting
// 1.11 -> 0.81 ms); where a leaf has thousands of tiles they hit, and the
// scalar path is the faster
template <class R>
__global__ __launch_bounds__(64) void k_shoot_staged(ShootArgs sa, LensConst lc, MapGeom g,
                                                     const int32_t *__restrict__ tile_leaf,
                                                     const int32_t *__restrict__ tile_off,
                                                     const LeafInfo *__restrict__ leaves,
                                                     const double4 *__restrict__ near,
                                                     const typename Cx<R>::c2 *__restrict__ deriv,
                                                     double2 *__restrict__ verts, double2 *__restrict__ w_out)
{
    shoot_tile<R, true>(sa, lc, g, tile_leaf, tile_off, leaves, near, deriv, verts, w_out, blockIdx.x, threadIdx.x);
}

// the maps of a fused batch: every tile of every map in one launch (one
// wavefront per tile of the concatenated tile list)
__global__ __launch_bounds__(64) void k_shoot_batch(const BatchMap *__restrict__ maps, int32_t nmaps,
                                                    int64_t ntiles)
{
    {
        const int64_t t = blockIdx.x;
        const int32_t m = batch_find(maps, nmaps, t, &BatchMap::tile_lo);
        const BatchMap &d = maps[m];
        const ShootArgs sa{d.x0, d.y0, d.d1, d.d2, d.nr1, 0, d.p, 0, 0.0};
        // (the branches are uniform over the workgroup: one tile of one map)
        if (d.mixed) {
            if (d.staged)
                shoot_tile<float, true>(sa, d.lc, d.g, d.tile_leaf, d.tile_off, d.leaves, d.near,
                                        static_cast<const float2 *>(d.deriv), d.verts, nullptr, t - d.tile_lo,
                                        threadIdx.x);
            else
                shoot_tile<float>(sa, d.lc, d.g, d.tile_leaf, d.tile_off, d.leaves, d.near,
                                  static_cast<const float2 *>(d.deriv), d.verts, nullptr, t - d.tile_lo, threadIdx.x);
        } else {
            if (d.staged)
                shoot_tile<double, true>(sa, d.lc, d.g, d.tile_leaf, d.tile_off, d.leaves, d.near,
                                         static_cast<const double2 *>(d.deriv), d.verts, nullptr, t - d.tile_lo,
                                         threadIdx.x);
            else
                shoot_tile<double>(sa, d.lc, d.g, d.tile_leaf, d.tile_off, d.leaves, d.near,
                                   static_cast<const double2 *>(d.deriv), d.verts, nullptr, t - d.tile_lo, threadIdx.x);
        }
    }
}

// direct summation over every star (no FMM): one thread per vertex, stars
// staged through LDS in tiles; with counts, the points are the cell centres
// and each is counted in its pixel (inverse ray shooting) instead of stored
constexpr int DTILE = 256;
__global__ __launch_bounds__(256) void k_shoot_direct(ShootArgs sa, LensConst lc, MapGeom g, int64_t nverts,
                                                      const double *__restrict__ sx, const double *__restrict__ sy,
                                                      const double *__restrict__ sm, int32_t n,
                                                      double2 *__restrict__ verts, double2 *__restrict__ w_out,
                                                      unsigned long long *__restrict__ counts)
{
    __shared__ double3 tile[DTILE];
    int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t a = v % sa.nr1, b = sa.vb0 + v / sa.nr1;
    double x = grid_pos(sa.x0, sa.d1, a, sa.h), y = grid_pos(sa.y0, sa.d2, b, sa.h);
    double ax = 0.0, ay = 0.0;
    for (int32_t s0 = 0; s0 < n; s0 += DTILE) {
        int32_t s = s0 + threadIdx.x;
        __syncthreads();
        if (s < n) tile[threadIdx.x] = make_double3(sx[s], sy[s], sm[s]);
        __syncthreads();
        int32_t cnt = min(DTILE, n - s0);
        for (int32_t k = 0; k < cnt; ++k) {
            double3 st = tile[k];
            double ex = x - st.x, ey = y - st.y;
            double f = st.z / (ex * ex + ey * ey);
            ax += f * ex;
            ay += f * ey;
        }
    }
    double w1, w2;
    double2 uv;
    finish_vertex(lc, g, x, y, ax, ay, w1, w2, uv);
    if (counts) {
        irs_count(v < nverts, uv, g, counts);
        return;
    }
    if (v >= nverts) return;
    verts[v] = uv;
    if (w_out) w_out[v] = make_double2(w1, w2);
}

__global__ void k_irs_mu(const unsigned long long *__restrict__ counts, int64_t npix, double w,
                         double *__restrict__ map)
{
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < npix) map[k] = (double)counts[k] * w;
}

// w at arbitrary points: leaf by descending the tree, then as k_shoot
template <class R>
__global__ void k_deflect_points(int64_t npts, const double2 *__restrict__ z, int nlevels, double L0, int L0_exp,
                                 const int32_t *__restrict__ child0, const int32_t *__restrict__ leaf,
                                 const int32_t *__restrict__ node_leaf,
                                 const LeafInfo *__restrict__ leaves, const double4 *__restrict__ near,
                                 const typename Cx<R>::c2 *__restrict__ deriv, int p, LensConst lc,
                                 double2 *__restrict__ w)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    double x = z[t].x, y = z[t].y;
    const int64_t lf = find_leaf(x, y, nlevels, L0, L0_exp, child0, leaf, node_leaf);
    if (lf < 0) {
        w[t] = make_double2(nan(""), nan(""));
        return;
    }
    const LeafInfo li = leaves[lf];
    double ax, ay;
    leaf_alpha<R>(x - li.cx, y - li.cy, li, near + li.near_off, deriv + lf * p, p, ax, ay);
    MapGeom g{0, 0, 1, 1, 1, 1, 0};
    double w1, w2;
    double2 uv;
    finish_vertex(lc, g, x, y, ax, ay, w1, w2, uv);
    w[t] = make_double2(w1, w2);
}

__global__ void k_deflect_direct(int64_t npts, const double2 *__restrict__ z, const double *__restrict__ sx,
                                 const double *__restrict__ sy, const double *__restrict__ sm, int32_t n,
                                 LensConst lc, double2 *__restrict__ w)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= npts) return;
    double x = z[t].x, y = z[t].y, ax = 0.0, ay = 0.0;
    for (int32_t s = 0; s < n; ++s) {
        double ex = x - sx[s], ey = y - sy[s];
        double f = sm[s] / (ex * ex + ey * ey);
        ax += f * ex;
        ay += f * ey;
    }
    MapGeom g{0, 0, 1, 1, 1, 1, 0};
    double w1, w2;
    double2 uv;
    finish_vertex(lc, g, x, y, ax, ay, w1, w2, uv);
    w[t] = make_double2(w1, w2);
}

}  // namespace

LensConst lens_const(const mlm_lens *lens, const Region &R)
{
    LensConst lc;
    lc.lam1 = R.lam1;
    lc.lam2 = R.lam2;
    lc.kappa_star = lens->params.kappa_star;
    lc.r_star2 = lens->r_star * lens->r_star;
    lc.c1 = lens->ext1;
    lc.c2 = lens->ext2;
    lc.sheet = lens->n == 0 ? 0 : lens->params.sheet == MLM_SHEET_CIRCLE ? 1 : lens->params.sheet == MLM_SHEET_RECT ? 2 : 0;
    for (int k = 0; k < 4; ++k) lc.psi3[k] = lens->params.psi3[k];
    lc.cubic = has_psi3(lens->params) ? 1 : 0;
    return lc;
}

int64_t plan_tiles(mlm_lens *lens, Tree &T, const Region &R, int64_t vb0, int64_t vb1, hipStream_t st, bool centres)
{
    Workspace &ws = lens->ws;
    int64_t nl = T.nleaves;
    const int64_t ncols = centres ? R.nr1 - 1 : R.nr1;
    const double h = centres ? 0.5 : 0.0;
    // every lattice point lies in exactly one leaf and every tile holds at
    // least one point, so the tiles number at most the points: bounding those
    // keeps the int32 counts and their scan from overflowing
    if ((vb1 - vb0) * ncols > (int64_t)INT32_MAX) fail(MLM_ERANGE, "more than 2^31 rays in one shooting plan");
    int32_t *cnt = static_cast<int32_t *>(ws.flags.reserve(nl * 4));
    int32_t *off = static_cast<int32_t *>(ws.tile_off.reserve(nl * 4));
    hipLaunchKernelGGL(k_tile_counts, dim3(nblocks(nl)), dim3(BLK), 0, st, nl, T.leaf_node, T.code, T.level, T.L0,
                       T.L0_exp, R.x0, R.d1, ncols, R.y0, R.d2, vb0, vb1, h, T.leaves, cnt);
    int64_t ntiles = scan_total_public(lens, cnt, off, nl, st);
    if (ntiles > 0) {
        int32_t *tl = static_cast<int32_t *>(ws.tile_leaf.reserve(ntiles * 4));
        hipLaunchKernelGGL(k_tile_leaf, dim3(nblocks(ntiles)), dim3(BLK), 0, st, ntiles, nl, off, tl);
    }
    return ntiles;
}

constexpr double STAGED_TILES_PER_LEAF = 256.0;

bool shoot_staged(const Region &R, const Tree &T)
{
    return (double)R.nr1 * (double)R.nr2 < STAGED_TILES_PER_LEAF * 64.0 * (double)std::max<int64_t>(T.nleaves, 1);
}

void launch_shoot(mlm_lens *lens, const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g,
                  int64_t ntiles, int64_t vb0, double2 *verts, double *w_out, hipStream_t st)
{
    if (ntiles <= 0) return;
    Workspace &ws = lens->ws;
    ShootArgs sa{R.x0, R.y0, R.d1, R.d2, R.nr1, vb0, T.p, 0, 0.0};
    const bool staged = shoot_staged(R, T);
    if (T.mixed)
        hipLaunchKernelGGL(staged ? k_shoot_staged<float> : k_shoot<float>, dim3((unsigned)ntiles), dim3(64), 0, st, sa,
                           lc, g, ws.tile_leaf.as<int32_t>(), ws.tile_off.as<int32_t>(), T.leaves, T.near, T.deriv_f,
                           verts, reinterpret_cast<double2 *>(w_out));
    else
        hipLaunchKernelGGL(staged ? k_shoot_staged<double> : k_shoot<double>, dim3((unsigned)ntiles), dim3(64), 0, st,
                           sa, lc, g, ws.tile_leaf.as<int32_t>(), ws.tile_off.as<int32_t>(), T.leaves, T.near, T.deriv,
                           verts, reinterpret_cast<double2 *>(w_out));
}

void launch_shoot_direct(mlm_lens *lens, const Region &R, const LensConst &lc, const MapGeom &g, int64_t vb0,
                         int64_t vb1, double2 *verts, double *w_out, hipStream_t st)
{
    int64_t nv = (vb1 - vb0) * R.nr1;
    if (nv <= 0) return;
    ShootArgs sa{R.x0, R.y0, R.d1, R.d2, R.nr1, vb0, 0, 0, 0.0};
    hipLaunchKernelGGL(k_shoot_direct, dim3(nblocks(nv)), dim3(256), 0, st, sa, lc, g, nv, lens->d_x, lens->d_y,
                       lens->d_m, (int32_t)lens->n, verts, reinterpret_cast<double2 *>(w_out), nullptr);
}

void launch_shoot_irs(mlm_lens *lens, const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g,
                      int64_t ntiles, int64_t cb0, unsigned long long *counts, hipStream_t st)
{
    if (ntiles <= 0) return;
    Workspace &ws = lens->ws;
    ShootArgs sa{R.x0, R.y0, R.d1, R.d2, R.nr1 - 1, cb0, T.p, 0, 0.5};
    if (T.mixed)
        hipLaunchKernelGGL(k_shoot_irs<float>, dim3((unsigned)ntiles), dim3(64), 0, st, sa, lc, g,
                           ws.tile_leaf.as<int32_t>(), ws.tile_off.as<int32_t>(), T.leaves, T.near, T.deriv_f, counts);
    else
        hipLaunchKernelGGL(k_shoot_irs<double>, dim3((unsigned)ntiles), dim3(64), 0, st, sa, lc, g,
                           ws.tile_leaf.as<int32_t>(), ws.tile_off.as<int32_t>(), T.leaves, T.near, T.deriv, counts);
}

void launch_shoot_irs_direct(mlm_lens *lens, const Region &R, const LensConst &lc, const MapGeom &g, int64_t cb0,
                             int64_t cb1, unsigned long long *counts, hipStream_t st)
{
    const int64_t nv = (cb1 - cb0) * (R.nr1 - 1);
    if (nv <= 0) return;
    ShootArgs sa{R.x0, R.y0, R.d1, R.d2, R.nr1 - 1, cb0, 0, 0, 0.5};
    hipLaunchKernelGGL(k_shoot_direct, dim3(nblocks(nv)), dim3(256), 0, st, sa, lc, g, nv, lens->d_x, lens->d_y,
                       lens->d_m, (int32_t)lens->n, nullptr, nullptr, counts);
}

void launch_irs_mu(const unsigned long long *counts, int64_t npix, double w, double *map, hipStream_t st)
{
    if (npix > 0) hipLaunchKernelGGL(k_irs_mu, dim3(nblocks(npix)), dim3(BLK), 0, st, counts, npix, w, map);
}

void launch_shoot_batch(const BatchMap *maps, int32_t nmaps, int64_t ntiles, hipStream_t st)
{
    if (ntiles <= 0) return;
    if (ntiles > (int64_t)UINT32_MAX) fail(MLM_ERANGE, "too many ray tiles in one batch chunk");
    hipLaunchKernelGGL(k_shoot_batch, dim3((unsigned)ntiles), dim3(64), 0, st, maps, nmaps, ntiles);
}

void launch_deflect_points(mlm_lens *lens, const Tree *T, const LensConst &lc, const double *z, int64_t n,
                           double *w, hipStream_t st)
{
    if (n <= 0) return;
    const double2 *z2 = reinterpret_cast<const double2 *>(z);
    double2 *w2 = reinterpret_cast<double2 *>(w);
    if (!T) {
        hipLaunchKernelGGL(k_deflect_direct, dim3(nblocks(n)), dim3(BLK), 0, st, n, z2, lens->d_x, lens->d_y,
                           lens->d_m, (int32_t)lens->n, lc, w2);
        return;
    }
    if (T->mixed)
        hipLaunchKernelGGL(k_deflect_points<float>, dim3(nblocks(n)), dim3(BLK), 0, st, n, z2, T->nlevels, T->L0,
                           T->L0_exp, T->child0, T->leaf, T->node_leaf, T->leaves, T->near, T->deriv_f, T->p, lc, w2);
    else
        hipLaunchKernelGGL(k_deflect_points<double>, dim3(nblocks(n)), dim3(BLK), 0, st, n, z2, T->nlevels, T->L0,
                           T->L0_exp, T->child0, T->leaf, T->node_leaf, T->leaves, T->near, T->deriv, T->p, lc, w2);
}

}  // namespace mlm
