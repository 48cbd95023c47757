// Internal declarations of the MI355X magnification-map library.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>
#include <vector>

#include "mlmap.h"

namespace mlm {

// ---------------------------------------------------------------------------
// errors: thrown inside the library, turned into mlm_status at the C ABI
// ---------------------------------------------------------------------------
struct Error {
    mlm_status status;
    std::string msg;
};

[[noreturn]] void fail(mlm_status st, const char *fmt, ...);

#define MLM_HIP(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            ::mlm::fail(e_ == hipErrorOutOfMemory ? MLM_ENOMEM : MLM_EDEVICE, "%s: %s", \
                        #call, hipGetErrorString(e_));                                 \
    } while (0)

// ---------------------------------------------------------------------------
// device buffers that grow on demand and are reused across calls
// ---------------------------------------------------------------------------
struct DevBuf {
    void *p = nullptr;
    size_t cap = 0;
    void *reserve(size_t bytes);  // contents are not preserved when it grows
    // grows keeping the first `keep` bytes (copied on `st`)
    void *grow_keep(size_t keep, size_t bytes, hipStream_t st);
    void release();
    ~DevBuf() { release(); }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// Scratch arena of the entry point that allocates nothing.  While one is
// installed on the calling thread, DevBuf::reserve and grow_keep hand out
// slices of it instead of device allocations (a slice is reused while it is
// large enough; nothing is freed), and every buffer it replaced is put back
// when the arena is removed.  Exhausting it is MLM_ERANGE.
struct Arena {
    static constexpr int MAX_BUFS = 128;
    char *base = nullptr;
    size_t cap = 0, used = 0;
    struct Saved {
        DevBuf *buf;
        void *p;
        size_t cap;
    } saved[MAX_BUFS];
    int nsaved = 0;
    bool owns(const void *q) const
    {
        return q && static_cast<const char *>(q) >= base && static_cast<const char *>(q) < base + cap;
    }
    void *take(size_t bytes);
    void *reserve(DevBuf &b, size_t bytes);
    void restore();
};
// the arena installed on this thread, or nullptr
Arena *&thread_arena();

// ---------------------------------------------------------------------------
// constants of the tree
// ---------------------------------------------------------------------------
constexpr int KEY_BITS = 24;     // square index bits per axis at the finest level
constexpr int MAX_ORDER = 31;    // expansion order limit (32 coefficients)
constexpr int NLIST = 27;        // interaction squares per node
constexpr int TILE = 8;          // ray tiles are TILE x TILE grid vertices

// interaction entry of a node: an M2L source node, or the stars of a square
// lying inside a coarser leaf (P2L), or nothing
struct IEntry {
    int32_t src;   // >= 0: source node;  -1: P2L from stars [slo, shi);  -2: empty
    int32_t off;   // offset index (dx + 3) + 7 (dy + 3) of the source square
    int32_t slo, shi;
};

// per-leaf data used by the ray kernels
struct LeafInfo {
    double cx, cy;        // centre
    double L, invL;       // half-length and its inverse
    int32_t near_off;     // first near star in the near-star array
    int32_t near_cnt;     // stars in the leaf's 3x3 block of same-level squares
    int32_t a_lo, na;     // grid columns [a_lo, a_lo + na) inside the leaf
    int32_t b_lo, nb;     // grid rows [b_lo, b_lo + nb) inside the leaf
    int32_t ntx, pad;     // tiles per tile-row
    double f0x, f0y;      // far field at the centre, d_0 = c_1 / L (FP64 in both modes)
};

// shooting region and ray grid
struct Region {
    double kappa, lam1, lam2, mu_macro;
    double mean_m, mean_m2, border;
    double X1, X2, dX1, dX2;
    double pix1, pix2;
    int64_t nr1, nr2;
    double d1, d2, x0, y0;
    double L0;
    int32_t L0_exp;       // L0 = 2^(L0_exp - 1)
};

// the lens equation's constant terms, passed by value to kernels
struct LensConst {
    double lam1, lam2;      // 1 - kappa + gamma, 1 - kappa - gamma
    double kappa_star;
    double r_star2;         // R_*^2
    double c1, c2;          // corner of the star rectangle (rectangular sheet)
    double psi3[4];         // third derivatives of the macro potential (app. D)
    int32_t sheet;          // 0: none, 1: circular sheet, 2: rectangular sheet
    int32_t cubic;          // psi3 has a nonzero entry
};

// per-triangle data of the row-parallel IPM: counter-clockwise vertices
// relative to the integer origin (ou, ov), edge slopes su = du/dv, the
// deposit per unit of twice the piece area, and per edge the factor of the
// squared distance past the edge's first column in its row term,
// -scale sign(dv) |dv/du| (0 for edges with du = 0) (120 bytes)
struct BigPrep {
    double u[3], v[3];
    double su[3];
    double ou, ov, scale;
    double kc[3];
};

// ray-grid geometry of a shooting launch: points (x0 + (a + h) d1,
// y0 + (b + h) d2), a < nr1, rows b from vb0 (h = 0: the grid's vertices;
// h = 1/2: the centres of its cells, for inverse ray shooting)
struct ShootArgs {
    double x0, y0, d1, d2;
    int64_t nr1, vb0;
    int p;
    int pad;
    double h;
};

// map geometry for the IPM, in pixel units
struct MapGeom {
    double ylo1, ylo2;      // lower-left corner of the map
    double pix1, pix2;
    int32_t n1, n2;
    double tri_weight;      // image area of a triangle / pixel area
    int32_t big_px;         // IPM: triangles whose bounding box covers more pixels go by row bands
    int32_t pad;
};

// the band threshold of a request (bounding-box pixels), default 64
inline int32_t big_pixels_of(const mlm_map_request &q) { return q.big_pixels > 0 ? q.big_pixels : 64; }

// one map of a fused batch, as the batch kernels see it (device array, in
// the order of the maps; the *_lo fields are non-decreasing prefix offsets)
struct BatchMap {
    double x0, y0, d1, d2;            // ray grid
    int64_t nr1, nrows;               // vertices per grid row, cell rows
    LensConst lc;
    MapGeom g;
    const int32_t *tile_leaf, *tile_off;
    const LeafInfo *leaves;
    const double4 *near;
    const void *deriv;                // double2, or float2 if mixed
    double2 *verts;                   // vertex rows 0 .. nrows of this map
    double *map;                      // n2 x n1, accumulated into
    unsigned long long *counters;     // [0] skipped triangles of this map
    int64_t tile_lo, ctile_lo, cell_lo, band_lo;   // first shoot tile, cell tile, cell, band
    int64_t big_lo, big_hi;           // this map's large triangles in the gathered list
    int32_t bh, nbands, p, mixed;
    int32_t staged, pad;              // staged: shoot with the leaf's stars through LDS (shoot_staged)
};

// one work item of the batch's persistent band pass: a slice [lo, hi) of the
// list of band `gband` (numbered over the batch's maps); `shared`: the band
// is split over several items, so its rows are added to the map atomically
struct BandItem {
    int64_t gband;
    int64_t lo, hi;
    int32_t shared, pad;
};

// The persistent band passes keep one work counter per XCD: the item list
// (in band order) is cut into NXCD contiguous ranges of about equal list
// length, and a workgroup first drains the range of the XCD it runs on, so
// the triangles a run of neighbouring bands shares are fetched into one L2
// (workgroups are dispatched to the XCDs round-robin, so workgroup i runs on
// XCD i mod NXCD); then it helps the other ranges.  The counters sit
// QUEUE_STRIDE u64 apart, each on its own cache line.
constexpr int NXCD = 8;
constexpr int QUEUE_STRIDE = 32;
constexpr size_t QUEUE_BYTES = (size_t)NXCD * QUEUE_STRIDE * sizeof(unsigned long long);
struct ItemParts {
    int64_t lo[NXCD + 1];   // range x is items [lo[x], lo[x + 1])
};
ItemParts split_items(const BandItem *items, int64_t n);

// index of the map whose range [lo, next lo) holds item x (maps with empty
// ranges are skipped: the last map whose lo <= x)
template <class T>
__device__ inline int32_t batch_find(const BatchMap *maps, int32_t nmaps, int64_t x, T BatchMap::*lo)
{
    int32_t a = 0, b = nmaps - 1;
    while (a < b) {
        const int32_t mid = (a + b + 1) >> 1;
        if (maps[mid].*lo <= x) a = mid;
        else b = mid - 1;
    }
    return a;
}

// FMM tree with coefficients (device arrays) and host metadata
struct Tree {
    double L0 = 0;
    int L0_exp = 0;
    int nmax = 32, lmax = KEY_BITS, p = 0;
    int64_t n = 0;                       // stars
    int nlevels = 0;
    std::vector<int64_t> level_lo, level_hi;
    int64_t nnodes = 0, nleaves = 0, near_total = 0;
    // stars in Morton order
    uint64_t *keys = nullptr;
    double *x = nullptr, *y = nullptr, *m = nullptr;
    // nodes
    uint64_t *code = nullptr;
    int32_t *level = nullptr, *leaf = nullptr, *slo = nullptr, *shi = nullptr, *block = nullptr;
    int32_t *parent = nullptr, *child0 = nullptr, *node_leaf = nullptr;
    int32_t *leaf_node = nullptr;
    IEntry *ilist = nullptr;
    bool mixed = false;                  // FP32 Taylor evaluation (deriv_f) and near field
    double2 *mult = nullptr, *local = nullptr;   // FP64 in both modes
    // leaf tables
    LeafInfo *leaves = nullptr;
    double4 *near = nullptr;             // (dx, dy, m, 0) relative to the leaf centre (both modes)
    double2 *deriv = nullptr;            // [nleaves][p]: (l+1) c_{l+1} / L
    float2 *deriv_f = nullptr;           // the same rounded to FP32 (mixed mode; entry 0 unused:
                                         // the leaf's f0x, f0y carry it in FP64)
};

struct Workspace {
    DevBuf keys_in, keys, idx_in, idx, sx, sy, sm, scan_tmp;
    DevBuf code, level, leaf, slo, shi, block, parent, child0, coll, node_leaf, leaf_node, flags, offs;
    DevBuf ilist, mult, local, ops_m2m, ops_m2l, ops_l2l;
    DevBuf leaves, near, deriv, near_offs;
    DevBuf tile_off, tile_leaf, verts, map, wbuf, pts, counters, items, itemoff, tbig, tbigoff, bigprep, bigrows, bigrow0, rowoff, nbnd, nbndoff, diff, bandcnt, bandoff,
        bandcur, bandlist, rfeat, rflag, rpos, rcand, rlabel, rstats, irs_counts, rtflag, rtpos, rsub0, rsub1, bitems, bqueue, tune_map;
    hipStream_t side = nullptr;           // second stream of a map: the large-triangle passes beside the cell pass
    hipEvent_t fork = nullptr, join = nullptr;
    void *pinned = nullptr;               // small pinned host buffer for read-backs
    size_t pinned_cap = 0;
    int64_t *spin = nullptr;              // coherent pinned slot of scan totals: {total, sequence}
    int64_t spin_seq = 0;                 // sequence number of the last total asked for
    int ops_p = -1;                       // expansion order of the operator tables
    ~Workspace();
};

}  // namespace mlm

struct mlm_lens {
    mlm_lens_params params{};
    int64_t n = 0;
    int device = 0;
    double *d_x = nullptr, *d_y = nullptr, *d_m = nullptr;
    double mass_sum = 0, mass2_sum = 0, max_abs = 0, r_star = 0;
    double ext1 = 0, ext2 = 0;            // star region: (R_*, R_*) or the rectangle's (c1, c2)
    mlm::Workspace ws;
    std::mutex mu;
};

// refinement network: FP32 master weights, Adam moments, gradient (+ loss),
// bf16 copies in the kernels' layouts, staging
struct mlm_refiner {
    mlm::DevBuf P, M, V, G, W1b, W2b, xbuf, gpart, idx, feats, labels, logits;
    mlm::DevBuf tstep;     // Adam steps taken (int64, on the device: read by the step kernels)
    mlm::DevBuf lacc;      // loss summed over an epoch's rows (double)
    hipStream_t gst = nullptr;   // training stream (graph capture needs a stream of its own)
    std::mutex mu;
    ~mlm_refiner()
    {
        if (gst) (void)hipStreamDestroy(gst);
    }
};

namespace mlm {

// region.cpp (host arithmetic, compiled without floating-point contraction)
mlm_status setup_region(const mlm_lens *lens, const mlm_map_request *req, Region *R);
int auto_order(double mean_m, double mean_m2, double L, double eps);

// field.cpp (host arithmetic, compiled without floating-point contraction)
void field_moments(const mlm_field_params &F, double &mean_m, double &mean_m2);
int64_t field_count(const mlm_field_params &F);
void field_extent(int shape, double kappa_star, double mass_sum, double aspect, double &e1, double &e2);
int64_t field_sample(const mlm_field_params &F, std::vector<double> &x, std::vector<double> &y,
                     std::vector<double> &m, double &e1, double &e2);
// the shooting region's centre and half-sizes (sec. 2.3, app. A) for given
// mass moments; (ext1, ext2): half-sizes of the star region's bounding box,
// searched for the images of the map when the lens has third-order terms
void shooting_region(const mlm_lens_params &P, double mean_m, double mean_m2, double ext1, double ext2,
                     const mlm_map_request &q, double &X1, double &X2, double &dX1, double &dX2);
bool has_psi3(const mlm_lens_params &P);

// tree.hip
void build_tree(mlm_lens *lens, const Region &R, const mlm_map_request &req, Tree &T,
                hipStream_t st);

// fmm.hip
void run_fmm(mlm_lens *lens, Tree &T, int p, hipStream_t st);
void build_leaf_tables(mlm_lens *lens, Tree &T, hipStream_t st);

// shoot.hip
LensConst lens_const(const mlm_lens *lens, const Region &R);
// ray tiles of the grid vertices of rows [vb0, vb1), or (centres) of the
// cell centres of cell rows [vb0, vb1)
int64_t plan_tiles(mlm_lens *lens, Tree &T, const Region &R, int64_t vb0, int64_t vb1,
                   hipStream_t st, bool centres = false);
// inverse ray shooting of the cell centres of cell rows [cb0, cb1): counts
// per pixel (n2 x n1) are added to `counts`
void launch_shoot_irs(mlm_lens *lens, const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g,
                      int64_t ntiles, int64_t cb0, unsigned long long *counts, hipStream_t st);
void launch_shoot_irs_direct(mlm_lens *lens, const Region &R, const LensConst &lc, const MapGeom &g, int64_t cb0,
                             int64_t cb1, unsigned long long *counts, hipStream_t st);
// map = counts * w
void launch_irs_mu(const unsigned long long *counts, int64_t npix, double w, double *map, hipStream_t st);
// whether a map's shooting stages each leaf's near stars through LDS: the
// grid has few ray tiles (64 rays) per leaf, so the scalar cache would miss
bool shoot_staged(const Region &R, const Tree &T);
void launch_shoot(mlm_lens *lens, const Tree &T, const Region &R, const LensConst &lc,
                  const MapGeom &g, int64_t ntiles, int64_t vb0, double2 *verts, double *w_out,
                  hipStream_t st);
void launch_shoot_direct(mlm_lens *lens, const Region &R, const LensConst &lc, const MapGeom &g,
                         int64_t vb0, int64_t vb1, double2 *verts, double *w_out,
                         hipStream_t st);
void launch_shoot_batch(const BatchMap *maps, int32_t nmaps, int64_t ntiles, hipStream_t st);
void launch_deflect_points(mlm_lens *lens, const Tree *T, const LensConst &lc, const double *z,
                           int64_t n, double *w, hipStream_t st);

// ipm.hip
// work counts of the per-cell IPM kernel (statistics): WORK_SLOTS partial sums
// per count, so that the wavefronts' additions rarely meet at one address
constexpr int WORK_SLOTS = 256;
// large triangles per workgroup of the band binning passes (and per slice of
// a batch map's list of them)
constexpr int64_t BIN_TRIS = 2048;
// cell tiles of the cell pass over cell rows [cb0, cb0 + nrows): one workgroup and one
// large-triangle count each
int64_t ipm_tile_count(int64_t nr1, int64_t nrows);
// (fine: the 16 x 16 pixel LDS window, for maps of many cells per pixel)
void launch_ipm(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                double *map, unsigned long long *counters, int32_t *tile_big, bool mixed, bool fine,
                unsigned long long *work, hipStream_t st);
// the large triangles of the tiles into prep/rows/row0 at the tiles' offsets
// tile_off (nbig in all; with fewer than one a tile, a resident grid skips
// the empty tiles)
void launch_big_gather(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                       int64_t nbig, const int64_t *tile_off, BigPrep *prep, int64_t *rows, int32_t *row0,
                       hipStream_t st);
void launch_big(int64_t nbig, const BigPrep *prep, const int64_t *rows, const MapGeom &g, double *map, double *diff,
                hipStream_t st);
void launch_diff_rows(const MapGeom &g, const double *diff, double *map, hipStream_t st);
// statistics: (triangle, pixel) pieces of cell rows [cb0, cb1) inside the map, added to *out
void launch_count_pieces(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                         unsigned long long *out, hipStream_t st);
int band_height(int32_t n1, int32_t n2);
void launch_band_count(int64_t nbig, const int32_t *row0, const int64_t *rows, int bh, int32_t nbands, int32_t *count,
                       hipStream_t st);
void launch_band_scatter(int64_t nbig, const int32_t *row0, const int64_t *rows, int bh, int32_t nbands,
                         unsigned long long *cursor, int32_t *list, hipStream_t st);
void launch_big_count(const double2 *verts, int64_t nr1, int64_t cb0, int64_t cb1, int64_t vb0, const MapGeom &g,
                      int32_t *tile_big, hipStream_t st);
void launch_ipm_batch(const BatchMap *maps, int32_t nmaps, int64_t nctiles, int32_t *tile_big, hipStream_t st);
void launch_big_gather_batch(const BatchMap *maps, int32_t nmaps, int64_t nctiles, const int64_t *tile_off,
                             BigPrep *prep, int64_t *rows, int32_t *row0, hipStream_t st);
void launch_band_count_batch(const BatchMap *maps, int64_t nslices, const int32_t *slice_map, const int64_t *slice_lo,
                             int32_t max_bands, const int32_t *row0, const int64_t *rows, int32_t *count,
                             hipStream_t st);
void launch_band_scatter_batch(const BatchMap *maps, int64_t nslices, const int32_t *slice_map,
                               const int64_t *slice_lo, int32_t max_bands, const int32_t *row0, const int64_t *rows,
                               unsigned long long *cursor, int32_t *list, hipStream_t st);
void launch_band_queue(const BatchMap *maps, int32_t nmaps, const BandItem *items, int64_t nitems,
                       const ItemParts &parts, unsigned long long *queue, const int32_t *list, const BigPrep *prep,
                       const int64_t *rows, int64_t lds_doubles, hipStream_t st);
void launch_band_queue1(const BandItem *items, int64_t nitems, const ItemParts &parts, unsigned long long *queue,
                        const int32_t *list,
                        const BigPrep *prep, const int64_t *rows, int bh, const MapGeom &g, double *map,
                        unsigned long long *work, bool atomic_all, hipStream_t st);
int64_t scan_i32_to_u64(mlm_lens *lens, const int32_t *in, unsigned long long *out, int64_t n, hipStream_t st);

// scan.hip: device-wide prefix sums (tmp: scan_tmp_bytes(n)); the total is
// stored to total_dev and/or total_host when they are given: total_host[0]
// the total, then (after a system-scope fence) total_host[1] = seq, so a host
// thread can wait for it without synchronising the stream
size_t scan_tmp_bytes(int64_t n);
void dev_scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, void *tmp, int64_t *total_dev,
                  int64_t *total_host, int64_t seq, hipStream_t st);
void dev_scan_i32_i64(const int32_t *in, int64_t *out, int64_t n, bool inclusive, void *tmp, int64_t *total_dev,
                      int64_t *total_host, int64_t seq, hipStream_t st);
void dev_scan_i64(const int64_t *in, int64_t *out, int64_t n, bool inclusive, void *tmp, int64_t *total_dev,
                  int64_t *total_host, int64_t seq, hipStream_t st);
// stable radix sort of (key, value) pairs by key bits [0, bits); the result
// ends in kout/vout, kin/vin are overwritten (tmp: radix_sort_tmp_bytes(n))
size_t radix_sort_tmp_bytes(int64_t n);
void radix_sort_pairs(uint64_t *kin, int32_t *vin, uint64_t *kout, int32_t *vout, int64_t n, int bits, void *tmp,
                      hipStream_t st);
int64_t scan_total_i64(mlm_lens *lens, const int64_t *in, int64_t *out, int64_t n, hipStream_t st);
int64_t scan_i32_to_i64(mlm_lens *lens, const int32_t *in, int64_t *out, int64_t n, hipStream_t st);

// products.hip
void launch_light_curve(const double *mu, const MapGeom &g, double y1a, double y2a, double y1b, double y2b,
                        int64_t npts, double *out, hipStream_t st);
void launch_histogram(const double *mu, int64_t npix, double lo, double hi, int nbins, unsigned long long *counts,
                      hipStream_t st);

// refine.hip
size_t refine_subcell_bytes();
void launch_refine_test(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau, int depth,
                        int window, int64_t n, const int64_t *cand, const void *list, int64_t nr1, int64_t vb0,
                        const double2 *verts, int32_t *flag, uint8_t *label, unsigned long long *stats, hipStream_t st);
void launch_refine_expand(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau, int depth,
                          int window, int64_t n, const int64_t *cand, const void *list, int64_t nr1, int64_t vb0,
                          const double2 *verts, const int32_t *flag, const int64_t *pos, double *map, void *out,
                          hipStream_t st);
void launch_sample_features(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, int64_t n,
                            const int64_t *ab, float *feats, hipStream_t st);
void launch_sample_labels(const Tree &T, const Region &R, const LensConst &lc, const MapGeom &g, double tau,
                          int window, int64_t n, const int64_t *ab, uint8_t *label, hipStream_t st);
void launch_compact(int64_t n, const int32_t *flag, const int64_t *pos, int64_t base, int64_t *cand, hipStream_t st);

// mlp.hip
void mlp_pack(const float *P, uint16_t *W1b, uint16_t *W2b, hipStream_t st);
// flag[t] for the cells t of a strip (cells cb0 + t / (nr1 - 1) rows, vertex
// rows from vb0): the network's logit of the cell's features above thr, or
// the cell folded; the features are formed on the fly
void mlp_flag_cells(int64_t nr1, int64_t cb0, int64_t ncells, int64_t vb0, const double2 *verts, const uint16_t *W1b,
                    const uint16_t *W2b, const float *P, float thr, int32_t *flag, hipStream_t st);
void mlp_predict(const float *feats, int64_t n, const uint16_t *W1b, const uint16_t *W2b, const float *P,
                 float *logits, hipStream_t st);
// rows of per-wavefront partial gradients (MLM_REFINER_PARAMS + 1 floats
// each) that a batch of n samples needs
int64_t mlp_part_rows(int64_t n);
// the gradient (and loss, at [MLM_REFINER_PARAMS]) of n samples, each
// sample's term divided by norm, added to grad in a fixed order: the same
// bits on every run
void mlp_train_batch(const float *feats, const uint8_t *y, const int64_t *idx, int64_t n, const uint16_t *W1b,
                     const uint16_t *W2b, const float *P, float pos_weight, float norm, float *grad, float *part,
                     float *xbuf, hipStream_t st);
void mlp_adam(float *P, float *M, float *V, float *grad, float lr, const int64_t *tstep, hipStream_t st);
void mlp_step_end(float *G, int64_t *tstep, double *lacc, float nb, hipStream_t st);
void mlp_zero(float *p, int64_t n, hipStream_t st);
void mlp_step_reset(int64_t *tstep, double *lacc, bool steps, hipStream_t st);

// helpers
void *pinned(mlm_lens *lens, size_t bytes);
// host memory the device writes coherently while it runs (zeroed)
void *coherent_pinned(size_t bytes);

}  // namespace mlm
