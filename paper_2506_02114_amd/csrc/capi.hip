// C ABI of the library and the orchestration of a map.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <set>
#include <chrono>
#include <condition_variable>
#include <thread>
#include <tuple>
#include <vector>

#include "dev.hpp"

namespace mlm {

namespace {
thread_local std::string g_last_error;
// Device and pinned-host allocations and frees of the library's growing
// buffers are made one at a time, process-wide: a batch prepares its maps on
// several host threads at once.
std::mutex g_alloc_mu;
}

void fail(mlm_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    throw Error{st, buf};
}

Arena *&thread_arena()
{
    static thread_local Arena *a = nullptr;
    return a;
}

void *Arena::take(size_t bytes)
{
    const size_t b = (bytes + 255) & ~(size_t)255;
    if (b > cap - used)
        fail(MLM_ERANGE, "the scratch array of %zu MiB is exhausted (%zu bytes more needed); mlm_map takes this map",
             cap >> 20, b - (cap - used));
    void *q = base + used;
    used += b;
    return q;
}

void *Arena::reserve(DevBuf &b, size_t bytes)
{
    if (owns(b.p) && bytes <= b.cap) return b.p;
    if (!owns(b.p)) {
        if (nsaved == MAX_BUFS) fail(MLM_ERANGE, "too many scratch buffers");
        saved[nsaved++] = Saved{&b, b.p, b.cap};
    }
    b.p = take(bytes);
    b.cap = (bytes + 255) & ~(size_t)255;
    return b.p;
}

void Arena::restore()
{
    while (nsaved > 0) {
        const Saved &s = saved[--nsaved];
        s.buf->p = s.p;
        s.buf->cap = s.cap;
    }
    used = 0;
}

void *DevBuf::reserve(size_t bytes)
{
    if (Arena *a = thread_arena()) return a->reserve(*this, bytes);
    if (p && bytes <= cap) return p;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    if (p) {
        MLM_HIP(hipDeviceSynchronize());   // the old buffer may still be in use by queued work
        MLM_HIP(hipFree(p));
        p = nullptr;
        cap = 0;
    }
    size_t c = bytes + bytes / 4;
    if (c < 256) c = 256;
    MLM_HIP(hipMalloc(&p, c));
    cap = c;
    return p;
}

void *DevBuf::grow_keep(size_t keep, size_t bytes, hipStream_t st)
{
    if (bytes <= cap && (!thread_arena() || thread_arena()->owns(p))) return p;
    size_t c = cap ? cap : 4096;
    while (c < bytes) c *= 2;
    void *q = nullptr;
    if (Arena *a = thread_arena()) {
        q = a->take(c);
        if (p && keep) MLM_HIP(hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, st));
        if (!a->owns(p)) {
            if (a->nsaved == Arena::MAX_BUFS) fail(MLM_ERANGE, "too many scratch buffers");
            a->saved[a->nsaved++] = Arena::Saved{this, p, cap};
        }
        p = q;
        cap = c;
        return p;
    }
    {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        MLM_HIP(hipMalloc(&q, c));
    }
    if (p && keep) MLM_HIP(hipMemcpyAsync(q, p, keep, hipMemcpyDeviceToDevice, st));
    MLM_HIP(hipStreamSynchronize(st));
    if (p) {
        std::lock_guard<std::mutex> g(g_alloc_mu);
        MLM_HIP(hipFree(p));
    }
    p = q;
    cap = c;
    return p;
}

void DevBuf::release()
{
    if (!p) return;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    (void)hipFree(p);
    p = nullptr;
    cap = 0;
}

Workspace::~Workspace()
{
    if (side) (void)hipStreamDestroy(side);
    if (fork) (void)hipEventDestroy(fork);
    if (join) (void)hipEventDestroy(join);
    std::lock_guard<std::mutex> g(g_alloc_mu);
    if (pinned) (void)hipHostFree(pinned);
    if (spin) (void)hipHostFree(spin);
}

void *coherent_pinned(size_t bytes)
{
    std::lock_guard<std::mutex> g(g_alloc_mu);
    void *p = nullptr;
    MLM_HIP(hipHostMalloc(&p, bytes, hipHostMallocCoherent));
    std::memset(p, 0, bytes);
    return p;
}

void *pinned(mlm_lens *lens, size_t bytes)
{
    Workspace &ws = lens->ws;
    if (ws.pinned && bytes <= ws.pinned_cap) return ws.pinned;
    std::lock_guard<std::mutex> g(g_alloc_mu);
    if (ws.pinned) {
        MLM_HIP(hipDeviceSynchronize());
        MLM_HIP(hipHostFree(ws.pinned));
        ws.pinned = nullptr;
    }
    size_t c = bytes < 4096 ? 4096 : bytes;
    MLM_HIP(hipHostMalloc(&ws.pinned, c, hipHostMallocDefault));
    ws.pinned_cap = c;
    return ws.pinned;
}

namespace {

constexpr int64_t STRIP_VERTS = 1ll << 26;   // vertices per strip buffer (1 GiB of double2)
constexpr int64_t IRS_STRIP_RAYS = 1ll << 30;   // rays per inverse-ray-shooting launch (nothing stored per ray)
constexpr double FINE_CELLS_PER_PIXEL = 256.0;  // cells per map pixel from which the cell pass takes its 16 x 16 window

__global__ void k_fill(double *p, int64_t n, double v)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = v;
}

__global__ void k_zero_u64(unsigned long long *p, int n)
{
    if (threadIdx.x < n) p[threadIdx.x] = 0;
}

__global__ void k_zero_i32(int32_t *p, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

// ray-star pairs and rays of a strip (for the statistics)
__global__ void k_strip_work(int64_t nleaves, const LeafInfo *__restrict__ lv, unsigned long long *cnt)
{
    int64_t lf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    unsigned long long rays = 0, pairs = 0;
    if (lf < nleaves) {
        LeafInfo li = lv[lf];
        if (li.na > 0 && li.nb > 0) {
            rays = (unsigned long long)li.na * (unsigned long long)li.nb;
            pairs = rays * (unsigned long long)li.near_cnt;
        }
    }
    if (rays) {
        atomicAdd(cnt + 1, pairs);
        atomicAdd(cnt + 2, rays);
    }
}

void fill(double *p, int64_t n, double v, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n, v);
}

struct Timer {
    bool on;
    hipStream_t st;
    std::vector<hipEvent_t> ev;
    Timer(bool on_, hipStream_t st_) : on(on_), st(st_) {}
    int mark() { return mark_on(st); }
    int mark_on(hipStream_t s)
    {
        if (!on) return -1;
        hipEvent_t e;
        MLM_HIP(hipEventCreate(&e));
        MLM_HIP(hipEventRecord(e, s));
        ev.push_back(e);
        return (int)ev.size() - 1;
    }
    double ms(int a, int b) const
    {
        if (!on || a < 0 || b < 0) return 0.0;
        float t = 0;
        MLM_HIP(hipEventElapsedTime(&t, ev[a], ev[b]));
        return t;
    }
    ~Timer()
    {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

void check_request(const mlm_map_request *q)
{
    if (!q) fail(MLM_EINVAL, "request is NULL");
    if (q->precision != MLM_PREC_FP64 && q->precision != MLM_PREC_MIXED)
        fail(MLM_EINVAL, "unknown precision %d", q->precision);
    if (q->precision == MLM_PREC_MIXED && q->method == MLM_METHOD_DIRECT)
        fail(MLM_ENOTSUP, "the direct-sum method runs in FP64 only");
    if (q->method != MLM_METHOD_FMM && q->method != MLM_METHOD_DIRECT) fail(MLM_EINVAL, "unknown method %d", q->method);
    if (q->order < 0 || q->order > MAX_ORDER) fail(MLM_EINVAL, "order %d outside [0, %d]", q->order, MAX_ORDER);
    if (q->leaf_max < 0 || q->max_level < 0 || q->max_level > KEY_BITS)
        fail(MLM_EINVAL, "leaf_max must be >= 0 and max_level in [0, %d]", KEY_BITS);
    if (!(q->eps >= 0) || !std::isfinite(q->eps)) fail(MLM_EINVAL, "eps must be finite and >= 0");
    if (q->refine < MLM_REFINE_NONE || q->refine > MLM_REFINE_LEARNED) fail(MLM_EINVAL, "unknown refine %d", q->refine);
    if (q->mapping != MLM_MAP_IPM && q->mapping != MLM_MAP_IRS) fail(MLM_EINVAL, "unknown mapping %d", q->mapping);
    if (q->big_pixels < 0) fail(MLM_EINVAL, "big_pixels must be >= 0");
    if (q->mapping == MLM_MAP_IRS && (q->refine != MLM_REFINE_NONE || q->w_out))
        fail(MLM_ENOTSUP, "ray shooting (IRS) maps take no cell refinement and no w_out");
    if (q->refine != MLM_REFINE_NONE) {
        if (q->precision != MLM_PREC_FP64 || q->method != MLM_METHOD_FMM)
            fail(MLM_ENOTSUP, "cell refinement needs FP64 and the FMM");
        if (q->refine_depth < 1 || q->refine_depth > 4 || q->refine_window < 1 || !(q->refine_tau >= 0) ||
            !std::isfinite(q->refine_tau) || !std::isfinite(q->refine_threshold))
            fail(MLM_EINVAL, "refine_depth in [1, 4], refine_window >= 1, refine_tau >= 0 and finite");
        if (q->refine == MLM_REFINE_LEARNED && !q->refiner) fail(MLM_EINVAL, "learned refinement needs a refiner");
    }
}

// tree + FMM + leaf tables for a request
void prepare_fmm(mlm_lens *lens, const Region &R, const mlm_map_request &q, Tree &T, hipStream_t st)
{
    build_tree(lens, R, q, T, st);
    T.mixed = q.precision == MLM_PREC_MIXED;
    int p = q.order;
    if (p <= 0) {
        double Lmin = std::ldexp(R.L0, -(T.nlevels - 1));
        p = auto_order(R.mean_m, R.mean_m2, Lmin, q.eps > 0 ? q.eps : 1e-7);
    }
    run_fmm(lens, T, p, st);
    build_leaf_tables(lens, T, st);
}

hipStream_t stream_of(const mlm_map_request *q) { return q ? static_cast<hipStream_t>(q->stream) : nullptr; }

__global__ void k_zero_u64n(unsigned long long *p, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0;
}

// out[m] = toff[maps[m].ctile_lo], out[nmaps] = toff[ntiles]: where each
// map's large triangles start in the gathered list
__global__ void k_map_big_bounds(const BatchMap *maps, int32_t nmaps, int64_t ntiles, const int64_t *toff,
                                 int64_t *out)
{
    const int32_t m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nmaps) out[m] = toff[maps[m].ctile_lo];
    if (m == nmaps) out[m] = toff[ntiles];
}

// --------------------------------------------------------------------------
// batched maps
// --------------------------------------------------------------------------

// device buffers of the fused batch passes (one set per process, on the
// device of the calls; calls are serialised by `mu`)
// host threads (each with a stream of its own) that prepare a batch's maps
constexpr int PREP_THREADS = 8;
// slices of the persistent band pass: at least this many list entries, and
// about this many items per chunk
constexpr int64_t BAND_SLICE_MIN = 256;
constexpr int64_t BAND_ITEMS_TARGET = 4096;

struct BatchWs {
    std::mutex mu;
    DevBuf maps, verts, tbig, toff, prep, rows, row0, bcnt, boffs, bcur, blist, counters, bounds, slice_map, slice_lo,
        items, queue;
    hipStream_t prep_st[PREP_THREADS] = {};   // created on first use, default priority
    std::vector<hipEvent_t> ready;            // per map: prepared (recorded on its preparing stream)
};

BatchWs &batch_ws()
{
    static BatchWs *w = new BatchWs;   // never destroyed: outlives every call, even at exit
    return *w;
}

struct MapPlan {
    mlm_lens *lens = nullptr;
    mlm_map_request q{};
    Region R{};
    Tree T;
    MapGeom g{};
    LensConst lc{};
    double *map = nullptr;
    int64_t nverts = 0, ncells = 0, ntiles = 0, nctiles = 0, nbands = 0;
    int32_t bh = 0;
    Timer *tm = nullptr;   // the preparing thread's timer, and its marks
    int e_tree0 = -1, e_tree1 = -1, e_fmm1 = -1;
};

MapGeom map_geom(const mlm_map_request &q, const Region &R)
{
    MapGeom g;
    g.ylo1 = q.y1c - q.hw1;
    g.ylo2 = q.y2c - q.hw2;
    g.pix1 = R.pix1;
    g.pix2 = R.pix2;
    g.n1 = q.n1;
    g.n2 = q.n2;
    g.tri_weight = 0.5 * R.d1 * R.d2 / (R.pix1 * R.pix2);
    g.big_px = big_pixels_of(q);
    return g;
}

int order_for(const mlm_map_request &q, const Region &R, const Tree &T)
{
    if (q.order > 0) return q.order;
    return auto_order(R.mean_m, R.mean_m2, std::ldexp(R.L0, -(T.nlevels - 1)), q.eps > 0 ? q.eps : 1e-7);
}

void map_impl(mlm_lens *lens, const mlm_map_request *req, double *mu, mlm_map_stats *stats);

// Autotuner of a class of maps (precision, order, log2 of rays per star):
// 1. the leaf size (the split threshold of app. C.1) that minimises the time
//    of tree + FMM + shooting, from timed trials on the map's own stars and a
//    sample of its grid rows; the expansion order follows from the accuracy
//    rule for each candidate tree (a bigger leaf needs a lower order);
// 2. then the IPM's band threshold (bounding-box pixels above which a triangle
//    goes by row bands) that minimises the time of the same sample strip mapped
//    whole.
// The result is cached per class for the process; the batch call tunes every
// class before its preparing threads start, on an otherwise idle device.
struct Tuned {
    int leaf_max, big_px;
};
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuned> g_tune_cache;

Tuned tune_map(mlm_lens *lens, const mlm_map_request &q, const Region &R, hipStream_t st)
{
    const double rays = (double)R.nr1 * (double)R.nr2;
    const int cls = (int)std::floor(std::log2(std::max(1.0, rays / std::max<int64_t>(lens->n, 1))));
    const auto key = std::make_tuple(q.precision, q.order, cls);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) return it->second;
    }
    const int64_t srows = std::min<int64_t>(R.nr2, std::max<int64_t>(64, R.nr2 / 16));
    const int64_t vb0 = (R.nr2 - srows) / 2;
    Tuned best{32, big_pixels_of(q)};
    {
        double2 *verts = static_cast<double2 *>(lens->ws.verts.reserve((size_t)(srows * R.nr1) * sizeof(double2)));
        const MapGeom g = map_geom(q, R);
        const LensConst lc = lens_const(lens, R);
        double best_t = 1e300;
        for (int cand : {8, 16, 32, 64}) {
            mlm_map_request qc = q;
            qc.leaf_max = cand;
            Timer tm(true, st);
            const int a = tm.mark();
            Tree T;
            build_tree(lens, R, qc, T, st);
            T.mixed = qc.precision == MLM_PREC_MIXED;
            run_fmm(lens, T, order_for(qc, R, T), st);
            build_leaf_tables(lens, T, st);
            const int b = tm.mark();
            const int64_t nt = plan_tiles(lens, T, R, vb0, vb0 + srows, st);
            const int c = tm.mark();
            launch_shoot(lens, T, R, lc, g, nt, vb0, verts, nullptr, st);
            const int d = tm.mark();
            MLM_HIP(hipStreamSynchronize(st));
            const double est = tm.ms(a, b) + tm.ms(c, d) * (double)R.nr2 / (double)srows;
            if (est < best_t) {
                best_t = est;
                best.leaf_max = cand;
            }
        }
    }
    if (q.mapping == MLM_MAP_IPM) {
        // the sample strip mapped whole (device timing of the call) at each band threshold
        const int64_t npix = (int64_t)q.n1 * q.n2;
        double *mu = static_cast<double *>(lens->ws.tune_map.reserve((size_t)npix * sizeof(double)));
        double best_t = 1e300;
        for (int cand : {32, 64, 128, 192}) {
            mlm_map_request qc = q;
            qc.leaf_max = best.leaf_max;
            qc.big_pixels = cand;
            qc.row_begin = vb0;
            qc.row_end = vb0 + srows - 1;
            qc.device_out = 1;
            qc.stream = st;
            qc.timing = 1;
            qc.refine = MLM_REFINE_NONE;
            qc.w_out = nullptr;
            mlm_map_stats S{};
            map_impl(lens, &qc, mu, &S);
            const double t = S.t_total_ms - S.t_tree_ms - S.t_fmm_ms;
            if (t < best_t) {
                best_t = t;
                best.big_px = cand;
            }
        }
    }
    std::lock_guard<std::mutex> g2(g_tune_mu);
    g_tune_cache[key] = best;
    return best;
}

// p[t] = t
__global__ void k_iota64(int64_t *p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = t;
}

}  // namespace
}  // namespace mlm

using namespace mlm;

#define API_BEGIN try {
#define API_END                                                        \
    }                                                                  \
    catch (const Error &e)                                             \
    {                                                                  \
        g_last_error = e.msg;                                          \
        return e.status;                                               \
    }                                                                  \
    catch (const std::bad_alloc &)                                     \
    {                                                                  \
        g_last_error = "host allocation failed";                       \
        return MLM_ENOMEM;                                             \
    }                                                                  \
    catch (...)                                                        \
    {                                                                  \
        g_last_error = "unexpected internal error";                    \
        return MLM_EDEVICE;                                            \
    }                                                                  \
    return MLM_OK;

extern "C" {

int32_t mlm_abi_version(void) { return MLM_ABI_VERSION; }

const char *mlm_status_str(mlm_status s)
{
    switch (s) {
    case MLM_OK: return "MLM_OK";
    case MLM_EINVAL: return "MLM_EINVAL";
    case MLM_EDEGENERATE: return "MLM_EDEGENERATE";
    case MLM_ERANGE: return "MLM_ERANGE";
    case MLM_ENOMEM: return "MLM_ENOMEM";
    case MLM_EDEVICE: return "MLM_EDEVICE";
    case MLM_ENOTSUP: return "MLM_ENOTSUP";
    }
    return "MLM_UNKNOWN";
}

const char *mlm_last_error(void) { return g_last_error.c_str(); }

void mlm_map_request_init(mlm_map_request *r)
{
    if (!r) return;
    std::memset(r, 0, sizeof *r);
    r->hw1 = r->hw2 = 1.0;
    r->n1 = r->n2 = 1;
    r->rays_per_pixel = 1.0;
    r->flux_fraction = 0.01;
    r->leaf_max = 32;
    r->max_level = KEY_BITS;
    r->precision = MLM_PREC_FP64;
    r->method = MLM_METHOD_FMM;
    r->eps = 1e-7;
    r->row_begin = 0;
    r->row_end = -1;
    r->refine = MLM_REFINE_NONE;
    r->refine_depth = 3;
    r->refine_window = 8;
    r->refine_tau = 1e-3;
    r->refine_threshold = 0.0;
}

void mlm_train_opts_init(mlm_train_opts *o)
{
    if (!o) return;
    std::memset(o, 0, sizeof *o);
    o->epochs = 4;
    o->batch = 4096;
    o->lr = 1e-3f;
    o->pos_weight = 1.0f;
    o->graph = 1;
}

}  // extern "C"

namespace mlm {
namespace {

void check_lens_params(const mlm_lens_params &P, int64_t n)
{
    if (!std::isfinite(P.kappa_star) || !std::isfinite(P.kappa_smooth) || !std::isfinite(P.gamma))
        fail(MLM_EINVAL, "kappa_star, kappa_smooth, gamma must be finite");
    if (P.kappa_star < 0) fail(MLM_EINVAL, "kappa_star must be >= 0");
    if (P.sheet != MLM_SHEET_CIRCLE && P.sheet != MLM_SHEET_NONE && P.sheet != MLM_SHEET_RECT)
        fail(MLM_EINVAL, "unknown sheet %d", P.sheet);
    if (n > 0 && P.sheet != MLM_SHEET_NONE && P.kappa_star == 0)
        fail(MLM_EINVAL, "a compensating sheet needs kappa_star > 0");
    if (P.sheet == MLM_SHEET_RECT && (!(P.rect_aspect > 0) || !std::isfinite(P.rect_aspect)))
        fail(MLM_EINVAL, "a rectangular sheet needs a finite rect_aspect > 0");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(P.psi3[k])) fail(MLM_EINVAL, "psi3 must be finite");
}

// a lens from host copies of the stars (checked here); the library owns it
mlm_lens *lens_from_host(const mlm_lens_params &P, const std::vector<double> &hx, const std::vector<double> &hy,
                         const std::vector<double> &hm)
{
    const int64_t n = (int64_t)hx.size();
    double s1 = 0.0, s2 = 0.0, amax = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (!std::isfinite(hx[i]) || !std::isfinite(hy[i]) || !std::isfinite(hm[i]) || !(hm[i] > 0))
            fail(MLM_EINVAL, "star %lld has a non-finite position or a mass <= 0", (long long)i);
        s1 += hm[i];
        s2 += hm[i] * hm[i];
        if (std::fabs(hx[i]) > amax) amax = std::fabs(hx[i]);
        if (std::fabs(hy[i]) > amax) amax = std::fabs(hy[i]);
    }
    std::unique_ptr<mlm_lens> L(new mlm_lens());
    L->params = P;
    L->n = n;
    MLM_HIP(hipGetDevice(&L->device));
    L->mass_sum = s1;
    L->mass2_sum = s2;
    L->max_abs = amax;
    L->r_star = (n > 0 && P.kappa_star > 0) ? std::sqrt(s1 / P.kappa_star) : 0.0;
    if (n > 0 && P.kappa_star > 0 && P.sheet != MLM_SHEET_NONE)
        field_extent(P.sheet, P.kappa_star, s1, P.rect_aspect, L->ext1, L->ext2);
    size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(double);
    MLM_HIP(hipMalloc(&L->d_x, bytes));
    MLM_HIP(hipMalloc(&L->d_y, bytes));
    MLM_HIP(hipMalloc(&L->d_m, bytes));
    if (n > 0) {
        MLM_HIP(hipMemcpy(L->d_x, hx.data(), n * sizeof(double), hipMemcpyHostToDevice));
        MLM_HIP(hipMemcpy(L->d_y, hy.data(), n * sizeof(double), hipMemcpyHostToDevice));
        MLM_HIP(hipMemcpy(L->d_m, hm.data(), n * sizeof(double), hipMemcpyHostToDevice));
    }
    return L.release();
}

}  // namespace
}  // namespace mlm

extern "C" {

mlm_status mlm_lens_create(const mlm_lens_params *params, const double *x, const double *y, const double *m,
                           int64_t n, int32_t device_ptrs, mlm_lens **out)
{
    API_BEGIN
    if (!params || !out) fail(MLM_EINVAL, "params and out must not be NULL");
    if (n < 0) fail(MLM_EINVAL, "n must be >= 0");
    if (n > 0 && (!x || !y || !m)) fail(MLM_EINVAL, "star arrays must not be NULL");
    if (n >= (int64_t)INT32_MAX / 2) fail(MLM_ERANGE, "too many stars");
    check_lens_params(*params, n);
    std::vector<double> hx(n), hy(n), hm(n);
    if (n > 0 && device_ptrs) {
        MLM_HIP(hipMemcpy(hx.data(), x, n * sizeof(double), hipMemcpyDeviceToHost));
        MLM_HIP(hipMemcpy(hy.data(), y, n * sizeof(double), hipMemcpyDeviceToHost));
        MLM_HIP(hipMemcpy(hm.data(), m, n * sizeof(double), hipMemcpyDeviceToHost));
    } else if (n > 0) {
        std::memcpy(hx.data(), x, n * sizeof(double));
        std::memcpy(hy.data(), y, n * sizeof(double));
        std::memcpy(hm.data(), m, n * sizeof(double));
    }
    *out = lens_from_host(*params, hx, hy, hm);
    API_END
}

mlm_status mlm_lens_create_sampled(const mlm_lens_params *params, const mlm_field_params *f, mlm_lens **out)
{
    API_BEGIN
    if (!params || !f || !out) fail(MLM_EINVAL, "params, field and out must not be NULL");
    if (params->kappa_star != f->kappa_star) fail(MLM_EINVAL, "the lens's and the field's kappa_star differ");
    if (params->sheet != MLM_SHEET_NONE && params->sheet != f->shape)
        fail(MLM_EINVAL, "the lens's sheet must be the field's shape or none");
    std::vector<double> hx, hy, hm;
    double e1 = 0, e2 = 0;
    const int64_t n = field_sample(*f, hx, hy, hm, e1, e2);
    if (n >= (int64_t)INT32_MAX / 2) fail(MLM_ERANGE, "too many stars");
    mlm_lens_params P = *params;
    if (P.sheet == MLM_SHEET_RECT) P.rect_aspect = e2 / e1;
    check_lens_params(P, n);
    *out = lens_from_host(P, hx, hy, hm);
    API_END
}

mlm_status mlm_lens_stars(const mlm_lens *lens, double *x, double *y, double *m, int64_t cap, int64_t *n)
{
    API_BEGIN
    if (!lens || !n) fail(MLM_EINVAL, "lens and n must not be NULL");
    *n = lens->n;
    if (cap < lens->n) fail(MLM_ERANGE, "the lens has %lld stars, capacity %lld", (long long)lens->n, (long long)cap);
    const size_t b = (size_t)lens->n * sizeof(double);
    if (lens->n > 0) {
        if (x) MLM_HIP(hipMemcpy(x, lens->d_x, b, hipMemcpyDeviceToHost));
        if (y) MLM_HIP(hipMemcpy(y, lens->d_y, b, hipMemcpyDeviceToHost));
        if (m) MLM_HIP(hipMemcpy(m, lens->d_m, b, hipMemcpyDeviceToHost));
    }
    API_END
}

mlm_status mlm_field_moments(const mlm_field_params *f, double *mean_m, double *mean_m2)
{
    API_BEGIN
    if (!f || !mean_m || !mean_m2) fail(MLM_EINVAL, "field and outputs must not be NULL");
    mlm_field_params g = *f;   // only the mass function is checked here
    g.n_stars = 1;
    g.rect_aspect = 1;
    (void)field_count(g);
    field_moments(g, *mean_m, *mean_m2);
    API_END
}

mlm_status mlm_field_count(const mlm_field_params *f, int64_t *n)
{
    API_BEGIN
    if (!f || !n) fail(MLM_EINVAL, "field and n must not be NULL");
    *n = field_count(*f);
    API_END
}

mlm_status mlm_field_sample(const mlm_field_params *f, double *x, double *y, double *m, int64_t cap, int64_t *n,
                            double *extent1, double *extent2)
{
    API_BEGIN
    if (!f || !n) fail(MLM_EINVAL, "field and n must not be NULL");
    const int64_t cnt = field_count(*f);
    if (cnt > 0 && (!x || !y || !m)) fail(MLM_EINVAL, "star arrays must not be NULL");
    if (cap < cnt) {
        *n = cnt;
        fail(MLM_ERANGE, "the field has %lld stars, capacity %lld", (long long)cnt, (long long)cap);
    }
    std::vector<double> hx, hy, hm;
    double e1 = 0, e2 = 0;
    field_sample(*f, hx, hy, hm, e1, e2);
    std::memcpy(x, hx.data(), (size_t)cnt * sizeof(double));
    std::memcpy(y, hy.data(), (size_t)cnt * sizeof(double));
    std::memcpy(m, hm.data(), (size_t)cnt * sizeof(double));
    *n = cnt;
    if (extent1) *extent1 = e1;
    if (extent2) *extent2 = e2;
    API_END
}

mlm_status mlm_field_cover(const mlm_lens_params *params, const mlm_field_params *f, const mlm_map_request *req,
                           double margin, double *extent1, double *extent2)
{
    API_BEGIN
    if (!params || !f || !req || !extent1 || !extent2) fail(MLM_EINVAL, "arguments must not be NULL");
    if (!(margin >= 1) || !std::isfinite(margin)) fail(MLM_EINVAL, "margin must be finite and >= 1");
    check_request(req);
    mlm_field_params g = *f;
    if (g.n_stars == 0 && !(g.extent1 > 0)) {   // only the mass function matters here
        g.n_stars = 1;
        if (g.shape == MLM_SHEET_RECT && !(g.rect_aspect > 0)) g.rect_aspect = 1;
    }
    (void)field_count(g);
    double mm, mm2, X1, X2, dX1, dX2;
    field_moments(g, mm, mm2);
    // (a lens with third-order terms needs its region stated here: with no
    // star region yet there is nothing to search)
    shooting_region(*params, mm, mm2, 0.0, 0.0, *req, X1, X2, dX1, dX2);
    const double a1 = std::fabs(X1) + dX1, a2 = std::fabs(X2) + dX2;
    if (f->shape == MLM_SHEET_RECT) {
        *extent1 = margin * a1;
        *extent2 = margin * a2;
    } else {
        *extent1 = *extent2 = margin * std::sqrt(a1 * a1 + a2 * a2);
    }
    API_END
}

void mlm_lens_destroy(mlm_lens *lens)
{
    if (!lens) return;
    (void)hipDeviceSynchronize();
    if (lens->d_x) (void)hipFree(lens->d_x);
    if (lens->d_y) (void)hipFree(lens->d_y);
    if (lens->d_m) (void)hipFree(lens->d_m);
    delete lens;
}

mlm_status mlm_lens_get_info(const mlm_lens *lens, mlm_lens_info *out)
{
    API_BEGIN
    if (!lens || !out) fail(MLM_EINVAL, "lens and out must not be NULL");
    mlm_lens_info I{};
    I.n_stars = lens->n;
    I.mass_sum = lens->mass_sum;
    I.mean_m = lens->n ? lens->mass_sum / (double)lens->n : 0.0;
    I.mean_m2 = lens->n ? lens->mass2_sum / (double)lens->n : 0.0;
    I.r_star = lens->r_star;
    I.kappa = lens->params.kappa_star + lens->params.kappa_smooth;
    double l1 = 1.0 - I.kappa + lens->params.gamma, l2 = 1.0 - I.kappa - lens->params.gamma;
    I.mu_macro = 1.0 / (l1 * l2);
    I.max_abs = lens->max_abs;
    I.extent1 = lens->ext1;
    I.extent2 = lens->ext2;
    *out = I;
    API_END
}

mlm_status mlm_map_region(const mlm_lens *lens, const mlm_map_request *req, mlm_region *out)
{
    API_BEGIN
    if (!lens || !out) fail(MLM_EINVAL, "lens and out must not be NULL");
    check_request(req);
    Region R{};
    setup_region(lens, req, &R);
    mlm_region o{};
    o.lam1 = R.lam1;
    o.lam2 = R.lam2;
    o.mu_macro = R.mu_macro;
    o.border = R.border;
    o.X1 = R.X1;
    o.X2 = R.X2;
    o.dX1 = R.dX1;
    o.dX2 = R.dX2;
    o.pix1 = R.pix1;
    o.pix2 = R.pix2;
    o.d1 = R.d1;
    o.d2 = R.d2;
    o.x0 = R.x0;
    o.y0 = R.y0;
    o.L0 = R.L0;
    o.nr1 = R.nr1;
    o.nr2 = R.nr2;
    o.order = req->order;
    *out = o;
    API_END
}

}  // extern "C"

namespace mlm {
namespace {

// one map (the body of mlm_map and of mlm_map_noalloc); the lens is locked
void map_impl(mlm_lens *lens, const mlm_map_request *req, double *mu, mlm_map_stats *stats)
{
    const mlm_map_request &q = *req;
    Region R{};
    setup_region(lens, req, &R);
    int64_t cb0 = q.row_begin > 0 ? q.row_begin : 0;
    int64_t cb1 = q.row_end < 0 ? R.nr2 - 1 : q.row_end;
    if (cb0 > cb1 || cb1 > R.nr2 - 1) fail(MLM_EINVAL, "cell rows [%lld, %lld) outside [0, %lld)", (long long)cb0,
                                           (long long)cb1, (long long)(R.nr2 - 1));
    Workspace &ws = lens->ws;
    hipStream_t st = stream_of(req);
    Timer tm(q.timing != 0, st);
    int e_start = tm.mark();

    int64_t npix = (int64_t)q.n1 * q.n2;
    double *map = q.device_out ? mu : static_cast<double *>(ws.map.reserve(npix * sizeof(double)));
    fill(map, npix, 0.0, st);
    // counters: [0] skipped triangles, [1] ray-star pairs, [2] rays, [3] unused,
    // [4] band row items, [5] band boundary pieces (if timing), [6] (triangle,
    // pixel) pieces (timing 2), [7] unused, then (if
    // timing) WORK_SLOTS partial sums each of small triangles, column items
    // and column pieces
    constexpr int NCNT = 8 + 3 * WORK_SLOTS;
    unsigned long long *cnt = static_cast<unsigned long long *>(ws.counters.reserve(NCNT * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_zero_u64n, dim3((NCNT + 255) / 256), dim3(256), 0, st, cnt, (int64_t)NCNT);
    // column differences of the per-triangle row kernel, for maps too wide
    // for row bands
    double *diff = nullptr;
    if (band_height(q.n1, q.n2) <= 0) {
        const int64_t ndiff = (int64_t)q.n2 * (q.n1 + 1);
        diff = static_cast<double *>(ws.diff.reserve(ndiff * sizeof(double)));
        fill(diff, ndiff, 0.0, st);
    }

    Tree T;
    const bool fmm = q.method == MLM_METHOD_FMM;
    int e_tree = -1, e_fmm = -1;
    if (fmm) {
        build_tree(lens, R, q, T, st);
        T.mixed = q.precision == MLM_PREC_MIXED;
        e_tree = tm.mark();
        int p = q.order;
        if (p <= 0) p = auto_order(R.mean_m, R.mean_m2, std::ldexp(R.L0, -(T.nlevels - 1)), q.eps > 0 ? q.eps : 1e-7);
        run_fmm(lens, T, p, st);
        build_leaf_tables(lens, T, st);
        e_fmm = tm.mark();
    }

    MapGeom g;
    g.ylo1 = q.y1c - q.hw1;
    g.ylo2 = q.y2c - q.hw2;
    g.pix1 = R.pix1;
    g.pix2 = R.pix2;
    g.n1 = q.n1;
    g.n2 = q.n2;
    g.tri_weight = 0.5 * R.d1 * R.d2 / (R.pix1 * R.pix2);
    g.big_px = big_pixels_of(q);
    LensConst lc = lens_const(lens, R);

    int64_t n_big = 0, n_big_rows = 0, n_cand = 0, n_refined = 0;
    double t_refine = 0.0;
    bool refine_stats_zeroed = false;

    double t_shoot = 0.0, t_ipm = 0.0, t_cells = 0.0, t_band = 0.0;
    int64_t tiles = 0;
    int nstrips = 0;
    const bool irs = q.mapping == MLM_MAP_IRS;
    if (irs) {
        // inverse ray shooting: one ray per cell centre, counted per pixel;
        // nothing is stored per ray, so strips are only bounded by the tile plan
        unsigned long long *irs_cnt =
            static_cast<unsigned long long *>(ws.irs_counts.reserve((size_t)npix * sizeof(unsigned long long)));
        hipLaunchKernelGGL(k_zero_u64n, dim3((unsigned)((npix + 255) / 256)), dim3(256), 0, st, irs_cnt, npix);
        const int64_t rows = std::max<int64_t>(1, IRS_STRIP_RAYS / std::max<int64_t>(R.nr1 - 1, 1));
        for (int64_t r0 = cb0; r0 < cb1; ++nstrips) {
            const int64_t r1 = std::min(cb1, r0 + rows);
            int64_t nt = 0;
            if (fmm) {
                nt = plan_tiles(lens, T, R, r0, r1, st, true);
                hipLaunchKernelGGL(k_strip_work, dim3((unsigned)((T.nleaves + 255) / 256)), dim3(256), 0, st,
                                   T.nleaves, T.leaves, cnt);
            }
            const int ea = tm.mark();
            if (fmm) launch_shoot_irs(lens, T, R, lc, g, nt, r0, irs_cnt, st);
            else launch_shoot_irs_direct(lens, R, lc, g, r0, r1, irs_cnt, st);
            const int eb = tm.mark();
            MLM_HIP(hipStreamSynchronize(st));
            t_shoot += tm.ms(ea, eb);
            tiles += nt;
            r0 = r1;
        }
        const int ea = tm.mark();
        launch_irs_mu(irs_cnt, npix, R.d1 * R.d2 / (R.pix1 * R.pix2), map, st);
        const int eb = tm.mark();
        MLM_HIP(hipStreamSynchronize(st));
        t_ipm += tm.ms(ea, eb);
    } else {
        int64_t rows_per_strip = STRIP_VERTS / R.nr1;
        if (Arena *a = thread_arena()) {
            // inside a scratch arena the vertex strip takes at most a quarter of
            // what is left; the rest serves the IPM's per-strip buffers
            const int64_t fit = (int64_t)((a->cap - a->used) / 4 / (sizeof(double2) * (size_t)R.nr1));
            rows_per_strip = std::min(rows_per_strip, fit);
        }
        if (rows_per_strip < 2) rows_per_strip = 2;
        int64_t nbuf = rows_per_strip * R.nr1;
        int64_t vrows = cb1 - cb0 + 1;
        if (vrows < rows_per_strip) nbuf = vrows * R.nr1;
        double2 *verts = static_cast<double2 *>(ws.verts.reserve((size_t)nbuf * sizeof(double2)));
        double *wdev = nullptr;
        if (q.w_out) wdev = q.device_out ? q.w_out : static_cast<double *>(ws.wbuf.reserve((size_t)nbuf * sizeof(double2)));

        // The cell pass sums its deposits in a 48 x 48 pixel LDS window per tile
        // of 16 x 16 cells, or in a 16 x 16 one where the map holds so many
        // cells per pixel that a tile lands in a pixel or two: there clearing
        // and flushing 2304 window entries would cost more than the tile's
        // cells (the shooting region covers the map, so cells per map pixel
        // is how finely the cells divide a pixel on average).
        const bool fine = (double)(R.nr1 - 1) * (double)(R.nr2 - 1) >= FINE_CELLS_PER_PIXEL * (double)g.n1 * (double)g.n2;
        for (int64_t r0 = cb0; r0 < cb1; ++nstrips) {
            int64_t r1 = std::min(cb1, r0 + rows_per_strip - 1);   // cells [r0, r1), vertex rows [r0, r1]
            int64_t vb0 = r0, vb1 = r1 + 1;
            double *w_here = nullptr;
            if (wdev) w_here = q.device_out ? wdev + 2 * (vb0 - cb0) * R.nr1 : wdev;
            int64_t nt = 0;
            if (fmm) {
                nt = plan_tiles(lens, T, R, vb0, vb1, st);
                hipLaunchKernelGGL(k_strip_work, dim3((unsigned)((T.nleaves + 255) / 256)), dim3(256), 0, st, T.nleaves,
                                   T.leaves, cnt);
            }
            int ea = tm.mark();
            if (fmm) launch_shoot(lens, T, R, lc, g, nt, vb0, verts, w_here, st);
            else launch_shoot_direct(lens, R, lc, g, vb0, vb1, verts, w_here, st);
            int eb = tm.mark();
            // IPM: the cell pass apportions the ordinary triangles; the large ones
            // are counted per cell tile, gathered, binned by pixel bands and
            // apportioned band by band.  With row bands and a second stream (the
            // default) that chain runs beside the cell pass: it counts the large
            // triangles itself and adds its band rows to the map atomically.
            const int64_t ncells = (R.nr1 - 1) * (r1 - r0);
            const int64_t ntl = ipm_tile_count(R.nr1, r1 - r0);
            const int bh = band_height(g.n1, g.n2);
            const bool overlap = bh > 0 && !q.one_stream && !thread_arena();
            hipStream_t bst = st;   // stream of the large-triangle chain
            if (overlap) {
                if (!ws.side) MLM_HIP(hipStreamCreateWithFlags(&ws.side, hipStreamNonBlocking));
                if (!ws.fork) MLM_HIP(hipEventCreateWithFlags(&ws.fork, hipEventDisableTiming));
                if (!ws.join) MLM_HIP(hipEventCreateWithFlags(&ws.join, hipEventDisableTiming));
                bst = ws.side;
                MLM_HIP(hipEventRecord(ws.fork, st));
                MLM_HIP(hipStreamWaitEvent(bst, ws.fork, 0));
            }
            int32_t *tbig = static_cast<int32_t *>(ws.tbig.reserve((size_t)std::max<int64_t>(ntl, 1) * sizeof(int32_t)));
            int64_t *toff = static_cast<int64_t *>(ws.tbigoff.reserve((size_t)(ntl + 1) * sizeof(int64_t)));
            if (overlap) {
                launch_big_count(verts, R.nr1, r0, r1, vb0, g, tbig, bst);
            } else if (ntl > 0) {
                hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((ntl + 255) / 256)), dim3(256), 0, st, tbig, ntl);
            }
            const int e_cells0 = tm.mark();
            launch_ipm(verts, R.nr1, r0, r1, vb0, g, map, cnt, overlap ? nullptr : tbig, q.precision == MLM_PREC_MIXED,
                       fine, q.timing >= 2 ? cnt + 8 : nullptr, st);
            const int e_cells = tm.mark();
            int e_band0 = -1, e_band1 = -1;
            const int64_t nb = scan_i32_to_i64(lens, tbig, toff, ntl, bst);
            if (nb > 0) {
                BigPrep *prep = static_cast<BigPrep *>(ws.bigprep.reserve((size_t)nb * sizeof(BigPrep)));
                int64_t *rows = static_cast<int64_t *>(ws.bigrows.reserve((size_t)nb * sizeof(int64_t)));
                int32_t *row0 = static_cast<int32_t *>(ws.bigrow0.reserve((size_t)nb * sizeof(int32_t)));
                launch_big_gather(verts, R.nr1, r0, r1, vb0, g, nb, toff, prep, rows, row0, bst);
                if (bh > 0) {
                    // large triangles by pixel bands: owned rows, LDS accumulation
                    const int32_t nbands = (int32_t)((g.n2 + bh - 1) / bh);
                    int32_t *bcnt = static_cast<int32_t *>(ws.bandcnt.reserve((size_t)nbands * sizeof(int32_t)));
                    unsigned long long *boffs =
                        static_cast<unsigned long long *>(ws.bandoff.reserve((size_t)(nbands + 1) * sizeof(unsigned long long)));
                    unsigned long long *bcur =
                        static_cast<unsigned long long *>(ws.bandcur.reserve((size_t)(nbands + 1) * sizeof(unsigned long long)));
                    hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((nbands + 255) / 256)), dim3(256), 0, bst, bcnt, nbands);
                    launch_band_count(nb, row0, rows, bh, nbands, bcnt, bst);
                    const int64_t nlist = scan_i32_to_u64(lens, bcnt, boffs, nbands, bst);
                    int32_t *blist = static_cast<int32_t *>(ws.bandlist.reserve((size_t)(nlist > 0 ? nlist : 1) * sizeof(int32_t)));
                    MLM_HIP(hipMemcpyAsync(bcur, boffs, (size_t)nbands * sizeof(unsigned long long), hipMemcpyDeviceToDevice, bst));
                    launch_band_scatter(nb, row0, rows, bh, nbands, bcur, blist, bst);
                    // the persistent band pass: every band with a list, cut into
                    // slices of at most `cut` entries
                    std::vector<unsigned long long> hoff((size_t)nbands + 1);
                    MLM_HIP(hipMemcpyAsync(hoff.data(), boffs, hoff.size() * sizeof(unsigned long long),
                                           hipMemcpyDeviceToHost, bst));
                    MLM_HIP(hipStreamSynchronize(bst));
                    const int64_t cut = std::max<int64_t>(BAND_SLICE_MIN, nlist / BAND_ITEMS_TARGET);
                    std::vector<BandItem> items;
                    for (int64_t b = 0; b < nbands; ++b) {
                        const int64_t lo = (int64_t)hoff[b], hi = (int64_t)hoff[b + 1];
                        if (hi <= lo) continue;
                        const int64_t k = (hi - lo + cut - 1) / cut;
                        for (int64_t a = lo; a < hi; a += cut)
                            items.push_back(BandItem{b, a, std::min(hi, a + cut), k > 1 ? 1 : 0, 0});
                    }
                    const int64_t nitems = (int64_t)items.size();
                    BandItem *ditems =
                        static_cast<BandItem *>(ws.bitems.reserve((size_t)std::max<int64_t>(nitems, 1) * sizeof(BandItem)));
                    unsigned long long *queue = static_cast<unsigned long long *>(ws.bqueue.reserve(QUEUE_BYTES));
                    if (nitems > 0) {
                        MLM_HIP(hipMemcpyAsync(ditems, items.data(), (size_t)nitems * sizeof(BandItem),
                                               hipMemcpyHostToDevice, bst));
                        MLM_HIP(hipStreamSynchronize(bst));   // the host item table is released at the end of this block
                    }
                    e_band0 = tm.mark_on(bst);
                    launch_band_queue1(ditems, nitems, split_items(items.data(), nitems), queue, blist, prep, rows,
                                       bh, g, map, q.timing >= 2 ? cnt + 4 : nullptr, overlap, bst);
                    e_band1 = tm.mark_on(bst);
                } else {
                    launch_big(nb, prep, rows, g, map, diff, st);
                }
                if (q.timing >= 2) {   // statistics only
                    int64_t *rowoff = static_cast<int64_t *>(ws.rowoff.reserve((size_t)nb * sizeof(int64_t)));
                    n_big_rows += scan_total_i64(lens, rows, rowoff, nb, bst);
                }
                n_big += nb;
            }
            if (overlap) {   // the map waits for both streams
                MLM_HIP(hipEventRecord(ws.join, bst));
                MLM_HIP(hipStreamWaitEvent(st, ws.join, 0));
            }
            if (q.timing >= 2) launch_count_pieces(verts, R.nr1, r0, r1, vb0, g, cnt + 6, st);   // statistics only
            int ec = tm.mark();
            if (q.refine != MLM_REFINE_NONE) {
                // cell refinement of this strip's cells (a + (nr1 - 1) b, b in [r0, r1))
                const int64_t base = (R.nr1 - 1) * r0;
                int64_t *cand = static_cast<int64_t *>(ws.rcand.reserve((size_t)ncells * sizeof(int64_t)));
                int64_t ncand = ncells;
                if (q.refine == MLM_REFINE_LEARNED) {
                    mlm_refiner *nn = q.refiner;
                    int32_t *flag = static_cast<int32_t *>(ws.rflag.reserve((size_t)ncells * sizeof(int32_t)));
                    int64_t *pos = static_cast<int64_t *>(ws.rpos.reserve((size_t)(ncells + 1) * sizeof(int64_t)));
                    mlp_flag_cells(R.nr1, r0, ncells, vb0, verts, nn->W1b.as<uint16_t>(), nn->W2b.as<uint16_t>(),
                                   nn->P.as<float>(), (float)q.refine_threshold, flag, st);
                    ncand = scan_i32_to_i64(lens, flag, pos, ncells, st);
                    launch_compact(ncells, flag, pos, base, cand, st);
                } else {
                    launch_compact(ncells, nullptr, nullptr, base, cand, st);
                }
                uint8_t *lab = static_cast<uint8_t *>(ws.rlabel.reserve((size_t)std::max<int64_t>(ncand, 1)));
                unsigned long long *rst3 = static_cast<unsigned long long *>(ws.rstats.reserve(4 * sizeof(unsigned long long)));
                if (!refine_stats_zeroed) {
                    hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(64), 0, st, rst3, 4);
                    refine_stats_zeroed = true;
                }
                // level by level: test every item of a level, number the refined
                // ones by a scan, expand them into the next level's subcells
                const size_t sub = refine_subcell_bytes();
                int64_t nlev = ncand;
                const void *list = nullptr;   // level 0: the candidate cells themselves
                DevBuf *next = &ws.rsub0;
                for (int d = 0; d < q.refine_depth && nlev > 0; ++d) {
                    int32_t *flag = static_cast<int32_t *>(ws.rtflag.reserve((size_t)nlev * sizeof(int32_t)));
                    int64_t *pos = static_cast<int64_t *>(ws.rtpos.reserve((size_t)(nlev + 1) * sizeof(int64_t)));
                    launch_refine_test(T, R, lc, g, q.refine_tau, q.refine_depth, q.refine_window, nlev, cand, list,
                                       R.nr1, vb0, verts, flag, d == 0 ? lab : nullptr, rst3, st);
                    const int64_t nref = scan_i32_to_i64(lens, flag, pos, nlev, st);
                    if (d == 0) n_refined += nref;
                    if (nref == 0) break;
                    void *out = next->reserve((size_t)(4 * nref) * sub);
                    launch_refine_expand(T, R, lc, g, q.refine_tau, q.refine_depth, q.refine_window, nlev, cand, list,
                                         R.nr1, vb0, verts, flag, pos, map, out, st);
                    list = out;
                    nlev = 4 * nref;
                    next = next == &ws.rsub0 ? &ws.rsub1 : &ws.rsub0;
                }
                n_cand += ncand;
            }
            int ed = tm.mark();
            if (q.w_out && !q.device_out)
                MLM_HIP(hipMemcpyAsync(q.w_out + 2 * (vb0 - cb0) * R.nr1, wdev, (size_t)(vb1 - vb0) * R.nr1 * 2 * sizeof(double),
                                       hipMemcpyDeviceToHost, st));
            MLM_HIP(hipStreamSynchronize(st));
            t_shoot += tm.ms(ea, eb);
            t_ipm += tm.ms(eb, ec);
            t_refine += tm.ms(ec, ed);
            t_cells += tm.ms(e_cells0, e_cells);
            t_band += tm.ms(e_band0, e_band1);
            tiles += nt;
            r0 = r1;
        }
    }
    if (diff) launch_diff_rows(g, diff, map, st);
    if (!q.device_out) MLM_HIP(hipMemcpyAsync(mu, map, npix * sizeof(double), hipMemcpyDeviceToHost, st));
    unsigned long long hc_local[NCNT];
    unsigned long long *hc =
        thread_arena() ? hc_local : static_cast<unsigned long long *>(pinned(lens, NCNT * sizeof(unsigned long long)));
    MLM_HIP(hipMemcpyAsync(hc, cnt, NCNT * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    int e_end = tm.mark();
    MLM_HIP(hipStreamSynchronize(st));
    if (stats) {
        mlm_map_stats S{};
        S.n_rays = irs ? (cb1 - cb0) * (R.nr1 - 1) : (cb1 - cb0 + 1) * R.nr1;
        S.n_cells = (cb1 - cb0) * (R.nr1 - 1);
        S.n_skipped = (int64_t)hc[0];
        S.n_nodes = T.nnodes;
        S.n_leaves = T.nleaves;
        S.n_levels = T.nlevels;
        S.order = T.p;
        S.near_pairs = (int64_t)hc[1];
        S.n_tiles = tiles;
        S.tri_area = 0.5 * R.d1 * R.d2;
        S.t_tree_ms = fmm ? tm.ms(e_start, e_tree) : 0.0;
        S.t_fmm_ms = fmm ? tm.ms(e_tree, e_fmm) : 0.0;
        S.t_shoot_ms = t_shoot;
        S.t_ipm_ms = t_ipm;
        S.t_total_ms = tm.ms(e_start, e_end);
        S.n_shoot_launches = nstrips;
        S.n_ipm_launches = nstrips;
        S.n_big = n_big;
        S.n_big_rows = n_big_rows;
        S.t_cells_ms = t_cells;
        S.t_band_ms = t_band;
        S.n_band_rows = q.timing >= 2 ? (int64_t)hc[4] : 0;
        S.n_band_pieces = q.timing >= 2 ? (int64_t)hc[5] : 0;
        int64_t wsum[3] = {0, 0, 0};
        for (int k = 0; k < 3 * WORK_SLOTS; ++k) wsum[k / WORK_SLOTS] += (int64_t)hc[8 + k];
        S.n_small = wsum[0];
        S.n_col_items = wsum[1];
        S.n_col_pieces = wsum[2];
        S.n_pieces = q.timing >= 2 && !irs ? (int64_t)hc[6] : 0;
        S.leaf_max = fmm ? T.nmax : 0;
        S.big_pixels = g.big_px;
        S.n_refine_candidates = n_cand;
        S.n_refined = n_refined;
        if (refine_stats_zeroed) {
            unsigned long long h3[4];
            MLM_HIP(hipMemcpy(h3, ws.rstats.p, sizeof h3, hipMemcpyDeviceToHost));
            S.n_refine_tests = (int64_t)h3[0];
            S.n_refine_large = (int64_t)h3[2];
        }
        S.t_refine_ms = t_refine;
        *stats = S;
    }
}

}  // namespace
}  // namespace mlm

extern "C" {

mlm_status mlm_map(mlm_lens *lens, const mlm_map_request *req, double *mu, mlm_map_stats *stats)
{
    API_BEGIN
    if (!lens || !mu) fail(MLM_EINVAL, "lens and mu must not be NULL");
    check_request(req);
    std::lock_guard<std::mutex> guard(lens->mu);
    map_impl(lens, req, mu, stats);
    API_END
}

}  // extern "C"

namespace mlm {
namespace {

// The scratch array of mlm_map_noalloc: one per device the library runs on,
// held until the process ends.  In host code its name is only a stand-in;
// the device address comes from hipGetSymbolAddress, once per device.
constexpr size_t SCRATCH_BYTES = (size_t)MLM_NOALLOC_SCRATCH_MIB << 20;
__device__ __align__(256) char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu[MAX_DEVICES];   // one call at a time per device
char *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of this device's scratch array (the device is current).
char *scratch_on(int dev)
{
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        MLM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = static_cast<char *>(ptr);
    }
    return g_scratch_ptr[dev];
}

// installs an arena over the scratch for the duration of a call; on the way
// out (also after an error) the stream is drained, so no kernel of this call
// still reads the scratch, and the lens's own buffers are put back
struct ArenaScope {
    Arena &a;
    Workspace &ws;
    hipStream_t st;
    int ops_p;
    ArenaScope(Arena &a_, Workspace &ws_, hipStream_t st_) : a(a_), ws(ws_), st(st_), ops_p(ws_.ops_p)
    {
        thread_arena() = &a;
    }
    ~ArenaScope()
    {
        (void)hipStreamSynchronize(st);
        thread_arena() = nullptr;
        a.restore();
        ws.ops_p = ops_p;   // operator tables uploaded into the scratch are gone
    }
};

}  // namespace
}  // namespace mlm

extern "C" {

mlm_status mlm_map_noalloc(mlm_lens *lens, const mlm_map_request *req, double *mu, mlm_map_stats *stats)
{
    API_BEGIN
    if (!lens || !mu) fail(MLM_EINVAL, "lens and mu must not be NULL");
    check_request(req);
    if (req->refine != MLM_REFINE_NONE) fail(MLM_ENOTSUP, "mlm_map_noalloc does not refine cells");
    int dev = 0;
    MLM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) fail(MLM_ERANGE, "device %d beyond the library's %d", dev, MAX_DEVICES);
    // sizes known before any device work: the sorted stars and their keys
    // (48 bytes a star), two vertex rows, the map if it goes to the host,
    // and the column differences of maps too wide for row bands
    Region R{};
    setup_region(lens, req, &R);
    const double need = 48.0 * (double)lens->n + 2.0 * 16.0 * (double)R.nr1 +
                        (req->device_out ? 0.0 : 8.0 * (double)req->n1 * (double)req->n2) +
                        (band_height(req->n1, req->n2) <= 0 ? 8.0 * (double)req->n2 * (double)(req->n1 + 1) : 0.0) +
                        (req->mapping == MLM_MAP_IRS ? 8.0 * (double)req->n1 * (double)req->n2 : 0.0);
    if (need > (double)SCRATCH_BYTES)
        fail(MLM_ERANGE, "the map needs at least %.0f MiB of scratch, more than the %zu MiB of mlm_map_noalloc",
             need / 1048576.0, SCRATCH_BYTES >> 20);
    std::lock_guard<std::mutex> sguard(g_scratch_mu[dev]);
    std::lock_guard<std::mutex> guard(lens->mu);
    Arena a;
    a.base = scratch_on(dev);
    a.cap = SCRATCH_BYTES;
    ArenaScope scope(a, lens->ws, stream_of(req));
    map_impl(lens, req, mu, stats);
    API_END
}

}  // extern "C"

namespace mlm {
namespace {

// the pixel geometry of a request (no lens needed)
MapGeom request_geom(const mlm_map_request *q)
{
    if (!(q->hw1 > 0) || !(q->hw2 > 0) || !std::isfinite(q->hw1) || !std::isfinite(q->hw2) || q->n1 <= 0 ||
        q->n2 <= 0 || !std::isfinite(q->y1c) || !std::isfinite(q->y2c))
        fail(MLM_EINVAL, "map centre/half-widths must be finite, half-widths > 0, pixels >= 1");
    MapGeom g{};
    g.ylo1 = q->y1c - q->hw1;
    g.ylo2 = q->y2c - q->hw2;
    g.pix1 = 2.0 * q->hw1 / (double)q->n1;
    g.pix2 = 2.0 * q->hw2 / (double)q->n2;
    g.n1 = q->n1;
    g.n2 = q->n2;
    return g;
}

// device buffers of the product calls (one set per process, serialised)
struct ProductWs {
    std::mutex mu;
    DevBuf map, out;
};

ProductWs &product_ws()
{
    static ProductWs *w = new ProductWs;   // never destroyed: outlives every call
    return *w;
}

}  // namespace
}  // namespace mlm

extern "C" {

mlm_status mlm_light_curve(const mlm_map_request *req, const double *mu, double y1a, double y2a, double y1b,
                           double y2b, int64_t npts, double *out)
{
    API_BEGIN
    if (!req || !mu || (npts > 0 && !out) || npts < 0) fail(MLM_EINVAL, "request, map and output must be given");
    if (!std::isfinite(y1a) || !std::isfinite(y2a) || !std::isfinite(y1b) || !std::isfinite(y2b))
        fail(MLM_EINVAL, "the track's ends must be finite");
    const MapGeom g = request_geom(req);
    hipStream_t st = stream_of(req);
    if (npts == 0) return MLM_OK;
    if (req->device_out) {
        launch_light_curve(mu, g, y1a, y2a, y1b, y2b, npts, out, st);
        MLM_HIP(hipStreamSynchronize(st));
        return MLM_OK;
    }
    ProductWs &P = product_ws();
    std::lock_guard<std::mutex> guard(P.mu);
    const size_t npix = (size_t)g.n1 * (size_t)g.n2;
    double *dm = static_cast<double *>(P.map.reserve(npix * sizeof(double)));
    double *dout = static_cast<double *>(P.out.reserve((size_t)npts * sizeof(double)));
    MLM_HIP(hipMemcpyAsync(dm, mu, npix * sizeof(double), hipMemcpyHostToDevice, st));
    launch_light_curve(dm, g, y1a, y2a, y1b, y2b, npts, dout, st);
    MLM_HIP(hipMemcpyAsync(out, dout, (size_t)npts * sizeof(double), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    API_END
}

mlm_status mlm_histogram(const mlm_map_request *req, const double *mu, double lo, double hi, int32_t nbins,
                         int64_t *counts)
{
    API_BEGIN
    if (!req || !mu || !counts) fail(MLM_EINVAL, "request, map and counts must be given");
    if (nbins < 1 || !(hi > lo) || !std::isfinite(lo) || !std::isfinite(hi))
        fail(MLM_EINVAL, "need nbins >= 1 and finite lo < hi");
    const MapGeom g = request_geom(req);
    hipStream_t st = stream_of(req);
    const int64_t npix = (int64_t)g.n1 * g.n2;
    if (req->device_out) {
        launch_histogram(mu, npix, lo, hi, nbins, reinterpret_cast<unsigned long long *>(counts), st);
        MLM_HIP(hipStreamSynchronize(st));
        return MLM_OK;
    }
    ProductWs &P = product_ws();
    std::lock_guard<std::mutex> guard(P.mu);
    double *dm = static_cast<double *>(P.map.reserve((size_t)npix * sizeof(double)));
    unsigned long long *dc =
        static_cast<unsigned long long *>(P.out.reserve((size_t)(nbins + 2) * sizeof(unsigned long long)));
    MLM_HIP(hipMemcpyAsync(dm, mu, (size_t)npix * sizeof(double), hipMemcpyHostToDevice, st));
    launch_histogram(dm, npix, lo, hi, nbins, dc, st);
    MLM_HIP(hipMemcpyAsync(counts, dc, (size_t)(nbins + 2) * sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    API_END
}

mlm_status mlm_map_batch(mlm_lens *const *lenses, const mlm_map_request *reqs, int32_t nmaps, double *const *mus,
                         mlm_map_stats *stats, const mlm_batch_opts *opts, mlm_batch_stats *bstats)
{
    API_BEGIN
    if (!lenses || !reqs || !mus || nmaps <= 0) fail(MLM_EINVAL, "lenses, reqs and mus must hold nmaps >= 1 entries");
    std::set<mlm_lens *> seen;
    for (int32_t i = 0; i < nmaps; ++i) {
        const mlm_map_request &q = reqs[i];
        if (!lenses[i] || !mus[i]) fail(MLM_EINVAL, "map %d: lens and output must not be NULL", i);
        if (!seen.insert(lenses[i]).second) fail(MLM_EINVAL, "map %d: every map of a batch needs its own lens", i);
        check_request(&q);
        if (q.method != MLM_METHOD_FMM) fail(MLM_EINVAL, "map %d: batched maps use the FMM", i);
        if (q.mapping != MLM_MAP_IPM) fail(MLM_ENOTSUP, "map %d: batched maps use inverse polygon mapping", i);
        if (q.row_begin > 0 || q.row_end >= 0) fail(MLM_EINVAL, "map %d: batched maps cover all rows", i);
        if (q.w_out) fail(MLM_EINVAL, "map %d: batched maps have no w_out", i);
        if ((q.device_out != 0) != (reqs[0].device_out != 0)) fail(MLM_EINVAL, "map %d: device_out differs", i);
    }
    mlm_batch_opts o{};
    if (opts) o = *opts;
    hipStream_t st = stream_of(&reqs[0]);
    // every lens locked, in address order
    std::vector<std::unique_lock<std::mutex>> locks;
    for (mlm_lens *l : seen) locks.emplace_back(l->mu);
    BatchWs &B = batch_ws();
    std::lock_guard<std::mutex> bguard(B.mu);
    Timer tm(bstats != nullptr || (stats && reqs[0].timing), st);
    const int e_start = tm.mark();

    // per map: region, (tuned) tree, FMM, leaf tables and tile plan, all kept
    // in the map's lens workspace
    std::vector<MapPlan> P(nmaps);
    unsigned long long *cnt =
        static_cast<unsigned long long *>(B.counters.reserve((size_t)nmaps * 8 * sizeof(unsigned long long)));
    hipLaunchKernelGGL(k_zero_u64n, dim3((unsigned)((nmaps * 8 + 255) / 256)), dim3(256), 0, st, cnt,
                       (int64_t)nmaps * 8);
    // Leaf sizes are tuned first, one class of map at a time on the caller's
    // stream while nothing else runs, so the trials are timed on an idle
    // device and each class is tuned once; the preparing threads then find
    // every class in the cache.
    if (o.autotune)
        for (int32_t i = 0; i < nmaps; ++i) {
            mlm_map_request qi = reqs[i];
            Region Ri{};
            setup_region(lenses[i], &qi, &Ri);
            (void)tune_map(lenses[i], qi, Ri, st);
        }
    // Regions, sizes and the chunks first (host arithmetic only): chunks of
    // consecutive maps that fit the vertex budget, one fused launch per stage
    // for all maps of a chunk.
    int64_t max_verts = 0;
    for (int32_t i = 0; i < nmaps; ++i) {
        MapPlan &m = P[i];
        m.lens = lenses[i];
        m.q = reqs[i];
        setup_region(m.lens, &m.q, &m.R);
        if (m.R.nr1 > INT32_MAX || m.R.nr2 > INT32_MAX) fail(MLM_ERANGE, "map %d: ray grid too large", i);
        m.bh = band_height(m.q.n1, m.q.n2);
        if (m.bh <= 0) fail(MLM_ENOTSUP, "map %d: %d x %d pixels is too wide for batched row bands", i, m.q.n1, m.q.n2);
        m.nbands = (m.q.n2 + m.bh - 1) / m.bh;
        m.nverts = m.R.nr1 * m.R.nr2;
        m.ncells = (m.R.nr1 - 1) * (m.R.nr2 - 1);
        m.nctiles = ((m.R.nr1 - 1 + 15) / 16) * ((m.R.nr2 - 1 + 15) / 16);
        max_verts = std::max(max_verts, m.nverts);
    }
    const int64_t budget = std::max<int64_t>(o.vertex_budget > 0 ? o.vertex_budget : (1ll << 28), max_verts);
    std::vector<int32_t> chunk_lo;
    for (int32_t c0 = 0; c0 < nmaps;) {
        chunk_lo.push_back(c0);
        int32_t c1 = c0;
        int64_t sv = 0;
        while (c1 < nmaps && (c1 == c0 || sv + P[c1].nverts <= budget)) sv += P[c1++].nverts;
        c0 = c1;
    }
    chunk_lo.push_back(nmaps);

    // A tree is built level by level with a host read of each level's size,
    // so one stream would idle between levels: PREP_THREADS host threads take
    // the maps in order, each on a stream of its own that first waits for the
    // caller's stream; a prepared map records an event there.  The chunks'
    // map passes start on the caller's stream as soon as their maps are
    // prepared, while the threads go on with later maps.
    for (hipStream_t &ps : B.prep_st)
        if (!ps) MLM_HIP(hipStreamCreateWithFlags(&ps, hipStreamNonBlocking));
    while ((int32_t)B.ready.size() < nmaps) {
        hipEvent_t e;
        MLM_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        B.ready.push_back(e);
    }
    hipEvent_t go;
    MLM_HIP(hipEventCreateWithFlags(&go, hipEventDisableTiming));
    MLM_HIP(hipEventRecord(go, st));
    std::vector<std::unique_ptr<Timer>> ptm;
    for (int t = 0; t < PREP_THREADS; ++t) ptm.emplace_back(new Timer(tm.on, B.prep_st[t]));
    std::atomic<int32_t> next{0};
    std::atomic<bool> failed{false};
    std::exception_ptr err;
    std::mutex done_mu;                     // guards done[], err
    std::condition_variable done_cv;
    std::vector<char> done((size_t)nmaps, 0);
    std::atomic<double> prep_ms{0.0};
    const auto t_prep0 = std::chrono::steady_clock::now();
    auto prep_worker = [&](int t) {
        const hipStream_t ps = B.prep_st[t];
        Timer &pt = *ptm[t];
        try {
            MLM_HIP(hipStreamWaitEvent(ps, go, 0));
            for (int32_t i = next++; i < nmaps && !failed; i = next++) {
                MapPlan &m = P[i];
                if (o.autotune) {
                    const Tuned tu = tune_map(m.lens, m.q, m.R, ps);
                    m.q.leaf_max = tu.leaf_max;
                    m.q.big_pixels = tu.big_px;
                }
                m.tm = &pt;
                m.e_tree0 = pt.mark();
                build_tree(m.lens, m.R, m.q, m.T, ps);
                m.T.mixed = m.q.precision == MLM_PREC_MIXED;
                m.e_tree1 = pt.mark();
                run_fmm(m.lens, m.T, order_for(m.q, m.R, m.T), ps);
                build_leaf_tables(m.lens, m.T, ps);
                m.e_fmm1 = pt.mark();
                m.ntiles = plan_tiles(m.lens, m.T, m.R, 0, m.R.nr2, ps);
                m.g = map_geom(m.q, m.R);
                m.lc = lens_const(m.lens, m.R);
                const int64_t npix = (int64_t)m.q.n1 * m.q.n2;
                m.map = m.q.device_out ? mus[i] : static_cast<double *>(m.lens->ws.map.reserve(npix * sizeof(double)));
                fill(m.map, npix, 0.0, ps);
                MLM_HIP(hipEventRecord(B.ready[i], ps));
                {
                    std::lock_guard<std::mutex> g(done_mu);
                    done[i] = 1;
                }
                done_cv.notify_all();
            }
            MLM_HIP(hipStreamSynchronize(ps));
        } catch (...) {
            failed = true;
            (void)hipStreamSynchronize(ps);
            {
                std::lock_guard<std::mutex> g(done_mu);
                if (!err) err = std::current_exception();
            }
            done_cv.notify_all();
        }
        const double ms =
            std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_prep0).count();
        double cur = prep_ms.load();
        while (ms > cur && !prep_ms.compare_exchange_weak(cur, ms)) {
        }
    };
    std::vector<std::thread> pool;
    for (int t = 0; t < PREP_THREADS; ++t) pool.emplace_back(prep_worker, t);
    // the preparing threads are joined on every way out of this call
    struct Joiner {
        std::vector<std::thread> &pool;
        std::atomic<bool> &failed;
        ~Joiner()
        {
            bool any = false;
            for (std::thread &th : pool) any = any || th.joinable();
            if (!any) return;
            failed = true;   // leaving early: the threads stop at their next map
            for (std::thread &th : pool)
                if (th.joinable()) th.join();
        }
    } joiner{pool, failed};

    // chunks of consecutive maps that fit the vertex budget: one fused launch
    // per stage for all maps of a chunk
    double t_shoot = 0.0, t_ipm = 0.0;
    int64_t n_chunks = 0, n_big = 0, n_rays = 0, n_cells = 0;
    std::vector<BatchMap> hm;
    for (size_t ci = 0; ci + 1 < chunk_lo.size(); ++ci, ++n_chunks) {
        const int32_t c0 = chunk_lo[ci], c1 = chunk_lo[ci + 1];
        {   // the chunk's maps prepared (or a preparing thread failed)
            std::unique_lock<std::mutex> g(done_mu);
            done_cv.wait(g, [&] {
                if (err) return true;
                for (int32_t i = c0; i < c1; ++i)
                    if (!done[i]) return false;
                return true;
            });
            if (err) break;
        }
        for (int32_t i = c0; i < c1; ++i) MLM_HIP(hipStreamWaitEvent(st, B.ready[i], 0));
        const int32_t nm = c1 - c0;
        int64_t sv = 0, max_band_lds = 0;
        for (int32_t i = c0; i < c1; ++i) {
            sv += P[i].nverts;
            max_band_lds = std::max<int64_t>(max_band_lds, (int64_t)P[i].bh * P[i].q.n1);
        }
        double2 *verts = static_cast<double2 *>(B.verts.reserve((size_t)sv * sizeof(double2)));
        hm.assign(nm, BatchMap{});
        int64_t vo = 0, tl = 0, ctl = 0, cl = 0, bl = 0;
        for (int32_t k = 0; k < nm; ++k) {
            const MapPlan &m = P[c0 + k];
            BatchMap &d = hm[k];
            d.x0 = m.R.x0;
            d.y0 = m.R.y0;
            d.d1 = m.R.d1;
            d.d2 = m.R.d2;
            d.nr1 = m.R.nr1;
            d.nrows = m.R.nr2 - 1;
            d.lc = m.lc;
            d.g = m.g;
            d.tile_leaf = m.lens->ws.tile_leaf.as<int32_t>();
            d.tile_off = m.lens->ws.tile_off.as<int32_t>();
            d.leaves = m.T.leaves;
            d.near = m.T.near;
            d.deriv = m.T.mixed ? static_cast<const void *>(m.T.deriv_f) : static_cast<const void *>(m.T.deriv);
            d.verts = verts + vo;
            d.map = m.map;
            d.counters = cnt + 8 * (c0 + k);
            d.tile_lo = tl;
            d.ctile_lo = ctl;
            d.cell_lo = cl;
            d.band_lo = bl;
            d.bh = m.bh;
            d.nbands = (int32_t)m.nbands;
            d.p = m.T.p;
            d.mixed = m.T.mixed ? 1 : 0;
            d.staged = shoot_staged(m.R, m.T) ? 1 : 0;
            d.pad = 0;
            vo += m.nverts;
            tl += m.ntiles;
            ctl += m.nctiles;
            cl += m.ncells;
            bl += m.nbands;
        }
        BatchMap *dmaps = static_cast<BatchMap *>(B.maps.reserve((size_t)nm * sizeof(BatchMap)));
        MLM_HIP(hipMemcpyAsync(dmaps, hm.data(), (size_t)nm * sizeof(BatchMap), hipMemcpyHostToDevice, st));
        mlm_lens *scan_lens = P[c0].lens;
        const int ea = tm.mark();
        launch_shoot_batch(dmaps, nm, tl, st);
        const int eb = tm.mark();
        int32_t *tbig = static_cast<int32_t *>(B.tbig.reserve((size_t)std::max<int64_t>(ctl, 1) * sizeof(int32_t)));
        int64_t *toff = static_cast<int64_t *>(B.toff.reserve((size_t)(ctl + 1) * sizeof(int64_t)));
        if (ctl > 0) hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((ctl + 255) / 256)), dim3(256), 0, st, tbig, ctl);
        launch_ipm_batch(dmaps, nm, ctl, tbig, st);
        const int64_t nb = scan_i32_to_i64(scan_lens, tbig, toff, ctl, st);
        if (nb > 0) {
            BigPrep *prep = static_cast<BigPrep *>(B.prep.reserve((size_t)nb * sizeof(BigPrep)));
            int64_t *rows = static_cast<int64_t *>(B.rows.reserve((size_t)nb * sizeof(int64_t)));
            int32_t *row0 = static_cast<int32_t *>(B.row0.reserve((size_t)nb * sizeof(int32_t)));
            launch_big_gather_batch(dmaps, nm, ctl, toff, prep, rows, row0, st);
            // each map's slice of the gathered list, cut into workgroup-sized
            // slices for the binning passes
            int64_t *bnd = static_cast<int64_t *>(B.bounds.reserve((size_t)(nm + 1) * sizeof(int64_t)));
            hipLaunchKernelGGL(k_map_big_bounds, dim3((unsigned)((nm + 1 + 255) / 256)), dim3(256), 0, st, dmaps, nm, ctl,
                               toff, bnd);
            std::vector<int64_t> hb((size_t)nm + 1);
            MLM_HIP(hipMemcpyAsync(hb.data(), bnd, hb.size() * sizeof(int64_t), hipMemcpyDeviceToHost, st));
            MLM_HIP(hipStreamSynchronize(st));
            std::vector<int32_t> smap;
            std::vector<int64_t> slo;
            int32_t max_bands = 0;
            for (int32_t k = 0; k < nm; ++k) {
                hm[k].big_lo = hb[k];
                hm[k].big_hi = hb[k + 1];
                for (int64_t a = hb[k]; a < hb[k + 1]; a += BIN_TRIS) {
                    smap.push_back(k);
                    slo.push_back(a);
                }
                if (hb[k + 1] > hb[k]) max_bands = std::max(max_bands, hm[k].nbands);
            }
            const int64_t ns = (int64_t)smap.size();
            int32_t *dsm = static_cast<int32_t *>(B.slice_map.reserve((size_t)ns * sizeof(int32_t)));
            int64_t *dsl = static_cast<int64_t *>(B.slice_lo.reserve((size_t)ns * sizeof(int64_t)));
            MLM_HIP(hipMemcpyAsync(dsm, smap.data(), (size_t)ns * sizeof(int32_t), hipMemcpyHostToDevice, st));
            MLM_HIP(hipMemcpyAsync(dsl, slo.data(), (size_t)ns * sizeof(int64_t), hipMemcpyHostToDevice, st));
            MLM_HIP(hipMemcpyAsync(dmaps, hm.data(), (size_t)nm * sizeof(BatchMap), hipMemcpyHostToDevice, st));
            int32_t *bcnt = static_cast<int32_t *>(B.bcnt.reserve((size_t)bl * sizeof(int32_t)));
            hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((bl + 255) / 256)), dim3(256), 0, st, bcnt, bl);
            launch_band_count_batch(dmaps, ns, dsm, dsl, max_bands, row0, rows, bcnt, st);
            unsigned long long *boffs =
                static_cast<unsigned long long *>(B.boffs.reserve((size_t)(bl + 1) * sizeof(unsigned long long)));
            const int64_t nlist = scan_i32_to_u64(scan_lens, bcnt, boffs, bl, st);
            int32_t *blist = static_cast<int32_t *>(B.blist.reserve((size_t)std::max<int64_t>(nlist, 1) * sizeof(int32_t)));
            unsigned long long *bcur =
                static_cast<unsigned long long *>(B.bcur.reserve((size_t)bl * sizeof(unsigned long long)));
            MLM_HIP(hipMemcpyAsync(bcur, boffs, (size_t)bl * sizeof(unsigned long long), hipMemcpyDeviceToDevice, st));
            launch_band_scatter_batch(dmaps, ns, dsm, dsl, max_bands, row0, rows, bcur, blist, st);
            // work items of the persistent band pass: every band with a list,
            // cut into slices of at most `cut` entries so that the items number
            // a few per workgroup the device holds
            std::vector<unsigned long long> hoff((size_t)bl + 1);
            MLM_HIP(hipMemcpyAsync(hoff.data(), boffs, hoff.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                                   st));
            MLM_HIP(hipStreamSynchronize(st));   // the host slice tables are released at the end of this block
            const int64_t cut = std::max<int64_t>(BAND_SLICE_MIN, nlist / BAND_ITEMS_TARGET);
            std::vector<BandItem> items;
            for (int64_t b = 0; b < bl; ++b) {
                const int64_t lo = (int64_t)hoff[b], hi = (int64_t)hoff[b + 1];
                if (hi <= lo) continue;
                const int64_t k = (hi - lo + cut - 1) / cut;
                for (int64_t a = lo; a < hi; a += cut)
                    items.push_back(BandItem{b, a, std::min(hi, a + cut), k > 1 ? 1 : 0, 0});
            }
            const int64_t nitems = (int64_t)items.size();
            BandItem *ditems = static_cast<BandItem *>(B.items.reserve((size_t)std::max<int64_t>(nitems, 1) * sizeof(BandItem)));
            unsigned long long *queue = static_cast<unsigned long long *>(B.queue.reserve(QUEUE_BYTES));
            if (nitems > 0)
                MLM_HIP(hipMemcpyAsync(ditems, items.data(), (size_t)nitems * sizeof(BandItem), hipMemcpyHostToDevice, st));
            launch_band_queue(dmaps, nm, ditems, nitems, split_items(items.data(), nitems), queue, blist, prep, rows,
                              max_band_lds, st);
            MLM_HIP(hipStreamSynchronize(st));   // the host item table is released at the end of this block
        }
        const int ec = tm.mark();
        MLM_HIP(hipStreamSynchronize(st));   // the chunk's buffers are reused by the next one
        t_shoot += tm.ms(ea, eb);
        t_ipm += tm.ms(eb, ec);
        n_big += nb;
        n_rays += vo;
        n_cells += cl;
    }
    for (std::thread &th : pool) th.join();
    (void)hipEventDestroy(go);
    if (err) std::rethrow_exception(err);
    std::vector<unsigned long long> hc((size_t)nmaps * 8);
    MLM_HIP(hipMemcpyAsync(hc.data(), cnt, hc.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
    for (int32_t i = 0; i < nmaps; ++i)
        if (!P[i].q.device_out)
            MLM_HIP(hipMemcpyAsync(mus[i], P[i].map, (size_t)P[i].q.n1 * P[i].q.n2 * sizeof(double),
                                   hipMemcpyDeviceToHost, st));
    const int e_end = tm.mark();
    MLM_HIP(hipStreamSynchronize(st));
    if (stats)
        for (int32_t i = 0; i < nmaps; ++i) {
            const MapPlan &m = P[i];
            mlm_map_stats S{};
            S.n_rays = m.nverts;
            S.n_cells = m.ncells;
            S.n_skipped = (int64_t)hc[8 * i];
            S.n_nodes = m.T.nnodes;
            S.n_leaves = m.T.nleaves;
            S.n_levels = m.T.nlevels;
            S.order = m.T.p;
            S.n_tiles = m.ntiles;
            S.tri_area = 0.5 * m.R.d1 * m.R.d2;
            S.t_tree_ms = m.tm ? m.tm->ms(m.e_tree0, m.e_tree1) : 0.0;
            S.t_fmm_ms = m.tm ? m.tm->ms(m.e_tree1, m.e_fmm1) : 0.0;
            S.leaf_max = m.T.nmax;
            S.big_pixels = m.g.big_px;
            S.n_shoot_launches = S.n_ipm_launches = 0;
            stats[i] = S;
        }
    if (bstats) {
        mlm_batch_stats b{};
        b.n_maps = nmaps;
        b.n_chunks = n_chunks;
        b.n_rays = n_rays;
        b.n_cells = n_cells;
        b.n_big = n_big;
        b.t_prep_ms = prep_ms.load();
        b.t_shoot_ms = t_shoot;
        b.t_ipm_ms = t_ipm;
        b.t_total_ms = tm.ms(e_start, e_end);
        *bstats = b;
    }
    API_END
}

// ---------------------------------------------------------------------------
// refinement network
// ---------------------------------------------------------------------------

static void refiner_upload(mlm_refiner *r, const float *params, hipStream_t st)
{
    MLM_HIP(hipMemcpyAsync(r->P.p, params, MLM_REFINER_PARAMS * sizeof(float), hipMemcpyHostToDevice, st));
    mlp_pack(r->P.as<float>(), r->W1b.as<uint16_t>(), r->W2b.as<uint16_t>(), st);
    MLM_HIP(hipStreamSynchronize(st));
}

mlm_status mlm_refiner_create(const float *params, uint64_t seed, mlm_refiner **out)
{
    API_BEGIN
    if (!out) fail(MLM_EINVAL, "out must not be NULL");
    *out = nullptr;
    std::unique_ptr<mlm_refiner> r(new mlm_refiner);
    const size_t nb = (MLM_REFINER_PARAMS + 1) * sizeof(float);
    r->P.reserve(nb);
    r->M.reserve(nb);
    r->V.reserve(nb);
    r->G.reserve(nb);
    r->W1b.reserve(16 * 64 * sizeof(uint16_t));
    r->W2b.reserve(64 * 64 * sizeof(uint16_t));
    r->tstep.reserve(sizeof(int64_t));
    r->lacc.reserve(sizeof(double));
    mlp_step_reset(r->tstep.as<int64_t>(), r->lacc.as<double>(), true, nullptr);
    mlp_zero(r->M.as<float>(), MLM_REFINER_PARAMS + 1, nullptr);
    mlp_zero(r->V.as<float>(), MLM_REFINER_PARAMS + 1, nullptr);
    mlp_zero(r->G.as<float>(), MLM_REFINER_PARAMS + 1, nullptr);
    std::vector<float> h(MLM_REFINER_PARAMS, 0.0f);
    if (params) {
        std::memcpy(h.data(), params, h.size() * sizeof(float));
    } else {
        // He-normal weights from a counter-free Box-Muller over splitmix64
        uint64_t x = seed;
        auto next = [&x]() {
            uint64_t z = (x += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            return (double)((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
        };
        auto normal = [&]() {
            const double u1 = std::max(next(), 1e-300), u2 = next();
            return std::sqrt(-2.0 * std::log(u1)) * std::cos(6.283185307179586 * u2);
        };
        for (int k = 0; k < 768; ++k) h[k] = (float)(normal() * std::sqrt(2.0 / 12));
        for (int k = 832; k < 4928; ++k) h[k] = (float)(normal() * std::sqrt(2.0 / 64));
        for (int k = 4992; k < 5056; ++k) h[k] = (float)(normal() * std::sqrt(2.0 / 64));
    }
    refiner_upload(r.get(), h.data(), nullptr);
    *out = r.release();
    API_END
}

void mlm_refiner_destroy(mlm_refiner *r) { delete r; }

mlm_status mlm_refiner_get_params(mlm_refiner *r, float *params)
{
    API_BEGIN
    if (!r || !params) fail(MLM_EINVAL, "refiner and params must not be NULL");
    std::lock_guard<std::mutex> g(r->mu);
    MLM_HIP(hipMemcpy(params, r->P.p, MLM_REFINER_PARAMS * sizeof(float), hipMemcpyDeviceToHost));
    API_END
}

mlm_status mlm_refiner_set_params(mlm_refiner *r, const float *params)
{
    API_BEGIN
    if (!r || !params) fail(MLM_EINVAL, "refiner and params must not be NULL");
    std::lock_guard<std::mutex> g(r->mu);
    for (int k = 0; k < MLM_REFINER_PARAMS; ++k)
        if (!std::isfinite(params[k])) fail(MLM_EINVAL, "parameter %d is not finite", k);
    refiner_upload(r, params, nullptr);
    API_END
}

// device copies of host rows (staging in the refiner's buffers)
static const float *stage_feats(mlm_refiner *r, const float *feats, int64_t n, int32_t dev, hipStream_t st)
{
    if (dev) return feats;
    float *d = static_cast<float *>(r->feats.reserve((size_t)n * 12 * sizeof(float)));
    MLM_HIP(hipMemcpyAsync(d, feats, (size_t)n * 12 * sizeof(float), hipMemcpyHostToDevice, st));
    return d;
}

mlm_status mlm_refiner_predict(mlm_refiner *r, const float *feats, int64_t n, float *logits, int32_t device_ptrs,
                               void *stream)
{
    API_BEGIN
    if (!r || n < 0 || (n > 0 && (!feats || !logits))) fail(MLM_EINVAL, "refiner, feats and logits must be given");
    std::lock_guard<std::mutex> g(r->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (n == 0) return MLM_OK;
    const float *df = stage_feats(r, feats, n, device_ptrs, st);
    float *dl = device_ptrs ? logits : static_cast<float *>(r->logits.reserve((size_t)n * sizeof(float)));
    mlp_predict(df, n, r->W1b.as<uint16_t>(), r->W2b.as<uint16_t>(), r->P.as<float>(), dl, st);
    if (!device_ptrs) MLM_HIP(hipMemcpyAsync(logits, dl, (size_t)n * sizeof(float), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    API_END
}

// rows per forward/backward launch: bounds the per-wavefront partial
// gradients (20 KB a wavefront of 32 rows) to 40 MB
constexpr int64_t GRAD_CHUNK = 65536;

// the staging and partial-gradient buffers of a batch of n rows (reserved
// before a graph is captured, so that capturing allocates nothing)
static void refiner_reserve(mlm_refiner *r, int64_t n)
{
    const int64_t c = std::min(n, GRAD_CHUNK);
    r->xbuf.reserve((size_t)((c + 127) / 128) * 128 * 12 * sizeof(float));
    r->gpart.reserve((size_t)mlp_part_rows(c) * (MLM_REFINER_PARAMS + 1) * sizeof(float));
}

// one forward/backward over rows idx[0, n) added to r->G (gradient + loss at
// [NP]), in chunks of GRAD_CHUNK rows taken in order; the loss of each chunk
// is divided by n
static void refiner_batch(mlm_refiner *r, const float *df, const uint8_t *dy, const int64_t *didx, int64_t n,
                          float pos_weight, hipStream_t st)
{
    refiner_reserve(r, n);
    for (int64_t c0 = 0; c0 < n; c0 += GRAD_CHUNK) {
        const int64_t c = std::min(GRAD_CHUNK, n - c0);
        mlp_train_batch(df, dy, didx + c0, c, r->W1b.as<uint16_t>(), r->W2b.as<uint16_t>(), r->P.as<float>(),
                        pos_weight, (float)n, r->G.as<float>(), r->gpart.as<float>(), r->xbuf.as<float>(), st);
    }
}

mlm_status mlm_refiner_grads(mlm_refiner *r, const float *feats, const uint8_t *labels, int64_t n, float pos_weight,
                             float *grads, double *loss, int32_t device_ptrs, void *stream)
{
    API_BEGIN
    if (!r || n <= 0 || !feats || !labels || !grads) fail(MLM_EINVAL, "refiner, rows, labels and grads must be given");
    if (!(pos_weight > 0) || !std::isfinite(pos_weight)) fail(MLM_EINVAL, "pos_weight must be finite and > 0");
    std::lock_guard<std::mutex> g(r->mu);
    hipStream_t st = static_cast<hipStream_t>(stream);
    const float *df = stage_feats(r, feats, n, device_ptrs, st);
    const uint8_t *dy = labels;
    if (!device_ptrs) {
        uint8_t *d = static_cast<uint8_t *>(r->labels.reserve((size_t)n));
        MLM_HIP(hipMemcpyAsync(d, labels, (size_t)n, hipMemcpyHostToDevice, st));
        dy = d;
    }
    int64_t *didx = static_cast<int64_t *>(r->idx.reserve((size_t)n * sizeof(int64_t)));
    hipLaunchKernelGGL(k_iota64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, didx, n);
    mlp_zero(r->G.as<float>(), MLM_REFINER_PARAMS + 1, st);
    refiner_batch(r, df, dy, didx, n, pos_weight, st);
    std::vector<float> h(MLM_REFINER_PARAMS + 1);
    MLM_HIP(hipMemcpyAsync(h.data(), r->G.p, h.size() * sizeof(float), hipMemcpyDeviceToHost, st));
    mlp_zero(r->G.as<float>(), MLM_REFINER_PARAMS + 1, st);
    MLM_HIP(hipStreamSynchronize(st));
    std::memcpy(grads, h.data(), MLM_REFINER_PARAMS * sizeof(float));
    if (loss) *loss = h[MLM_REFINER_PARAMS];
    API_END
}

mlm_status mlm_refiner_train(mlm_refiner *r, const mlm_train_opts *opts, const float *feats, const uint8_t *labels,
                             int64_t n, float *loss_per_epoch)
{
    API_BEGIN
    if (!r || !opts || n <= 0 || !feats || !labels) fail(MLM_EINVAL, "refiner, options and labelled rows must be given");
    const mlm_train_opts o = *opts;
    if (o.epochs < 0 || o.batch < 1 || !(o.lr > 0) || !(o.pos_weight > 0)) fail(MLM_EINVAL, "bad training options");
    std::lock_guard<std::mutex> g(r->mu);
    hipStream_t st = static_cast<hipStream_t>(o.stream);
    const float *df = stage_feats(r, feats, n, o.device_ptrs, st);
    const uint8_t *dy = labels;
    if (!o.device_ptrs) {
        uint8_t *d = static_cast<uint8_t *>(r->labels.reserve((size_t)n));
        MLM_HIP(hipMemcpyAsync(d, labels, (size_t)n, hipMemcpyHostToDevice, st));
        dy = d;
    }
    int64_t *didx = static_cast<int64_t *>(r->idx.reserve((size_t)n * sizeof(int64_t)));
    std::vector<int64_t> perm((size_t)n);
    uint64_t x = o.seed ^ 0x5DEECE66Dull;
    auto next = [&x]() {
        uint64_t z = (x += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    // the training runs on the refiner's own stream (a graph cannot be
    // captured on the null stream), after the caller's stream
    if (!r->gst) MLM_HIP(hipStreamCreateWithFlags(&r->gst, hipStreamNonBlocking));
    const hipStream_t ts = r->gst;
    hipEvent_t ready;
    MLM_HIP(hipEventCreateWithFlags(&ready, hipEventDisableTiming));
    MLM_HIP(hipEventRecord(ready, st));
    MLM_HIP(hipStreamWaitEvent(ts, ready, 0));
    (void)hipEventDestroy(ready);
    refiner_reserve(r, std::min<int64_t>(o.batch, n));
    float *G = r->G.as<float>();
    int64_t *tstep = r->tstep.as<int64_t>();
    double *lacc = r->lacc.as<double>();
    mlp_zero(G, MLM_REFINER_PARAMS + 1, ts);
    // one epoch's steps over the permutation in didx: the same kernels with the
    // same arguments every epoch (the permutation is rewritten in place, the
    // step count and the loss sum live on the device)
    auto epoch_steps = [&]() {
        for (int64_t b0 = 0; b0 < n; b0 += o.batch) {
            const int64_t nb = std::min<int64_t>(o.batch, n - b0);
            refiner_batch(r, df, dy, didx + b0, nb, o.pos_weight, ts);
            mlp_adam(r->P.as<float>(), r->M.as<float>(), r->V.as<float>(), G, o.lr, tstep, ts);
            mlp_step_end(G, tstep, lacc, (float)nb, ts);
            mlp_pack(r->P.as<float>(), r->W1b.as<uint16_t>(), r->W2b.as<uint16_t>(), ts);
        }
    };
    hipGraphExec_t ge = nullptr;
    if (o.graph && o.epochs > 0) {
        hipGraph_t gr = nullptr;
        MLM_HIP(hipStreamBeginCapture(ts, hipStreamCaptureModeThreadLocal));
        try {
            epoch_steps();
        } catch (...) {
            if (hipStreamEndCapture(ts, &gr) == hipSuccess && gr) (void)hipGraphDestroy(gr);
            throw;
        }
        MLM_HIP(hipStreamEndCapture(ts, &gr));
        const hipError_t ie = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
        (void)hipGraphDestroy(gr);
        MLM_HIP(ie);
    }
    try {
        for (int32_t e = 0; e < o.epochs; ++e) {
            for (int64_t k = 0; k < n; ++k) perm[k] = k;
            for (int64_t k = n - 1; k > 0; --k) std::swap(perm[k], perm[next() % (uint64_t)(k + 1)]);
            MLM_HIP(hipMemcpyAsync(didx, perm.data(), (size_t)n * sizeof(int64_t), hipMemcpyHostToDevice, ts));
            mlp_step_reset(tstep, lacc, false, ts);
            if (ge) MLM_HIP(hipGraphLaunch(ge, ts));
            else epoch_steps();
            double hl = 0.0;
            if (loss_per_epoch) MLM_HIP(hipMemcpyAsync(&hl, lacc, sizeof(double), hipMemcpyDeviceToHost, ts));
            MLM_HIP(hipStreamSynchronize(ts));   // perm (and hl) are reused by the next epoch
            if (loss_per_epoch) loss_per_epoch[e] = (float)(hl / (double)n);
        }
    } catch (...) {
        if (ge) (void)hipGraphExecDestroy(ge);
        throw;
    }
    if (ge) MLM_HIP(hipGraphExecDestroy(ge));
    MLM_HIP(hipStreamSynchronize(ts));
    API_END
}

mlm_status mlm_cell_samples(mlm_lens *lens, const mlm_map_request *req, const int64_t *cells, int64_t n, float *feats,
                            uint8_t *labels, int32_t device_ptrs)
{
    API_BEGIN
    if (!lens || !cells || n <= 0 || (!feats && !labels)) fail(MLM_EINVAL, "lens, cells and an output must be given");
    check_request(req);
    if (req->precision != MLM_PREC_FP64 || req->method != MLM_METHOD_FMM)
        fail(MLM_ENOTSUP, "cell samples need FP64 and the FMM");
    std::lock_guard<std::mutex> guard(lens->mu);
    Region R{};
    setup_region(lens, req, &R);
    hipStream_t st = stream_of(req);
    Tree T;
    prepare_fmm(lens, R, *req, T, st);
    Workspace &ws = lens->ws;
    const int64_t *dab = cells;
    if (!device_ptrs) {
        int64_t *d = static_cast<int64_t *>(ws.rpos.reserve((size_t)n * 2 * sizeof(int64_t)));
        MLM_HIP(hipMemcpyAsync(d, cells, (size_t)n * 2 * sizeof(int64_t), hipMemcpyHostToDevice, st));
        dab = d;
    }
    const MapGeom g = map_geom(*req, R);
    const LensConst lc = lens_const(lens, R);
    if (feats) {
        float *df = device_ptrs ? feats : static_cast<float *>(ws.rfeat.reserve((size_t)n * 12 * sizeof(float)));
        launch_sample_features(T, R, lc, g, n, dab, df, st);
        if (!device_ptrs) MLM_HIP(hipMemcpyAsync(feats, df, (size_t)n * 12 * sizeof(float), hipMemcpyDeviceToHost, st));
    }
    if (labels) {
        uint8_t *dl = device_ptrs ? labels : static_cast<uint8_t *>(ws.rlabel.reserve((size_t)n));
        launch_sample_labels(T, R, lc, g, req->refine_tau, req->refine_window, n, dab, dl, st);
        if (!device_ptrs) MLM_HIP(hipMemcpyAsync(labels, dl, (size_t)n, hipMemcpyDeviceToHost, st));
    }
    MLM_HIP(hipStreamSynchronize(st));
    API_END
}

mlm_status mlm_deflect(mlm_lens *lens, const mlm_map_request *req, const double *z_xy, int64_t n, double *w_xy)
{
    API_BEGIN
    if (!lens || (n > 0 && (!z_xy || !w_xy))) fail(MLM_EINVAL, "lens, z and w must not be NULL");
    if (n < 0) fail(MLM_EINVAL, "n must be >= 0");
    check_request(req);
    std::lock_guard<std::mutex> guard(lens->mu);
    Region R{};
    setup_region(lens, req, &R);
    hipStream_t st = stream_of(req);
    Workspace &ws = lens->ws;
    const double *zd = z_xy;
    double *wd = w_xy;
    if (!req->device_out && n > 0) {
        double *buf = static_cast<double *>(ws.pts.reserve((size_t)n * 4 * sizeof(double)));
        MLM_HIP(hipMemcpyAsync(buf, z_xy, n * 2 * sizeof(double), hipMemcpyHostToDevice, st));
        zd = buf;
        wd = buf + 2 * n;
    }
    if (n > 0) {
        // every point must lie in the root square
        std::vector<double> hz(2 * n);
        MLM_HIP(hipMemcpyAsync(hz.data(), zd, n * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        MLM_HIP(hipStreamSynchronize(st));
        for (int64_t i = 0; i < 2 * n; ++i)
            if (!(std::fabs(hz[i]) < R.L0)) fail(MLM_ERANGE, "point %lld lies outside the root square", (long long)(i / 2));
    }
    LensConst lc = lens_const(lens, R);
    Tree T;
    if (req->method == MLM_METHOD_FMM) {
        prepare_fmm(lens, R, *req, T, st);
        launch_deflect_points(lens, &T, lc, zd, n, wd, st);
    } else {
        launch_deflect_points(lens, nullptr, lc, zd, n, wd, st);
    }
    if (!req->device_out && n > 0) MLM_HIP(hipMemcpyAsync(w_xy, wd, n * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    API_END
}

mlm_status mlm_fmm_export(mlm_lens *lens, const mlm_map_request *req, mlm_tree_info *info, int32_t *level,
                          int64_t *ix, int64_t *iy, int32_t *leaf, int64_t *nstars, int64_t *block, double *mult,
                          double *local, int64_t cap)
{
    API_BEGIN
    if (!lens || !info) fail(MLM_EINVAL, "lens and info must not be NULL");
    check_request(req);
    std::lock_guard<std::mutex> guard(lens->mu);
    Region R{};
    setup_region(lens, req, &R);
    hipStream_t st = stream_of(req);
    Tree T;
    prepare_fmm(lens, R, *req, T, st);
    MLM_HIP(hipStreamSynchronize(st));
    mlm_tree_info I{};
    I.n_nodes = T.nnodes;
    I.n_leaves = T.nleaves;
    I.n_levels = T.nlevels;
    I.order = T.p;
    I.L0 = T.L0;
    *info = I;
    if (T.nnodes > cap) fail(MLM_ERANGE, "tree has %lld nodes, capacity %lld", (long long)T.nnodes, (long long)cap);
    int64_t N = T.nnodes, P1 = T.p + 1;
    std::vector<uint64_t> code(N);
    std::vector<int32_t> lv(N), lf(N), lo(N), hi(N), bk(N);
    MLM_HIP(hipMemcpy(code.data(), T.code, N * 8, hipMemcpyDeviceToHost));
    MLM_HIP(hipMemcpy(lv.data(), T.level, N * 4, hipMemcpyDeviceToHost));
    MLM_HIP(hipMemcpy(lf.data(), T.leaf, N * 4, hipMemcpyDeviceToHost));
    MLM_HIP(hipMemcpy(lo.data(), T.slo, N * 4, hipMemcpyDeviceToHost));
    MLM_HIP(hipMemcpy(hi.data(), T.shi, N * 4, hipMemcpyDeviceToHost));
    MLM_HIP(hipMemcpy(bk.data(), T.block, N * 4, hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < N; ++k) {
        if (level) level[k] = lv[k];
        if (ix) ix[k] = compact_bits(code[k]);
        if (iy) iy[k] = compact_bits(code[k] >> 1);
        if (leaf) leaf[k] = lf[k];
        if (nstars) nstars[k] = hi[k] - lo[k];
        if (block) block[k] = bk[k];
    }
    if (mult) MLM_HIP(hipMemcpy(mult, T.mult, N * P1 * sizeof(double2), hipMemcpyDeviceToHost));
    if (local) MLM_HIP(hipMemcpy(local, T.local, N * P1 * sizeof(double2), hipMemcpyDeviceToHost));
    API_END
}

}  // extern "C"
