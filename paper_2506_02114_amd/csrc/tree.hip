// Quadtree of the FMM (sec. 3.3, app. C.1), built on the device.
//
// Stars are sorted by their Morton key at the finest level (24 bits per axis),
// so the stars of any square of any level are one contiguous range of the
// sorted array.  The tree is then built level by level from the root: a node
// is divided into four children when the stars of its 3x3 block of
// same-level squares (the node and its neighbours) exceed nmax.  Counting the
// block needs only binary searches in the sorted keys.
#include <hipcub/hipcub.hpp>

#include "dev.hpp"

namespace mlm {

namespace {

constexpr int BLK = 256;

inline unsigned nblocks(int64_t n, int b = BLK) { return (unsigned)((n + b - 1) / b); }

__global__ void k_keys(const double *__restrict__ x, const double *__restrict__ y, int32_t n,
                       double L0, double scale, uint64_t *__restrict__ key, int32_t *__restrict__ idx)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    key[s] = morton2(fine_cell(x[s], L0, scale), fine_cell(y[s], L0, scale));
    idx[s] = s;
}

__global__ void k_gather(const int32_t *__restrict__ idx, const double *__restrict__ x,
                         const double *__restrict__ y, const double *__restrict__ m, int32_t n,
                         double *__restrict__ sx, double *__restrict__ sy, double *__restrict__ sm)
{
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n) return;
    int32_t k = idx[s];
    sx[s] = x[k];
    sy[s] = y[k];
    sm[s] = m[k];
}

__global__ void k_root(uint64_t *code, int32_t *level, int32_t *parent)
{
    code[0] = 0;
    level[0] = 0;
    parent[0] = -1;
}

// star range of the node's square and the star count of its 3x3 block
__global__ void k_level(int64_t lo, int64_t hi, int lev, int lmax, int nmax,
                        const uint64_t *__restrict__ code, const uint64_t *__restrict__ keys, int32_t n,
                        int32_t *__restrict__ slo, int32_t *__restrict__ shi, int32_t *__restrict__ block,
                        int32_t *__restrict__ split)
{
    int64_t q = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= hi) return;
    uint64_t c = code[q];
    uint32_t i = compact_bits(c), j = compact_bits(c >> 1);
    int sh = 2 * (KEY_BITS - lev);
    slo[q] = lower_bound_u64(keys, n, c << sh);
    shi[q] = lower_bound_u64(keys, n, (c + 1) << sh);
    int64_t side = 1ll << lev;
    int32_t blk = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            int64_t a = (int64_t)i + di, b = (int64_t)j + dj;
            if (a < 0 || b < 0 || a >= side || b >= side) continue;
            uint64_t cc = morton2((uint32_t)a, (uint32_t)b);
            blk += lower_bound_u64(keys, n, (cc + 1) << sh) - lower_bound_u64(keys, n, cc << sh);
        }
    block[q] = blk;
    split[q - lo] = (blk > nmax && lev < lmax) ? 1 : 0;
}

// children of the split nodes of a level, in Morton order
__global__ void k_emit(int64_t lo, int64_t hi, int64_t base, const int32_t *__restrict__ split,
                       const int32_t *__restrict__ offs, uint64_t *__restrict__ code,
                       int32_t *__restrict__ level, int32_t *__restrict__ parent,
                       int32_t *__restrict__ child0, int32_t *__restrict__ leaf, int next_level)
{
    int64_t q = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= hi) return;
    int32_t s = split[q - lo];
    leaf[q] = s ? 0 : 1;
    if (!s) {
        child0[q] = -1;
        return;
    }
    int64_t cb = base + 4 * (int64_t)offs[q - lo];
    child0[q] = (int32_t)cb;
    uint64_t c = code[q] << 2;
    for (int quad = 0; quad < 4; ++quad) {
        code[cb + quad] = c | (uint64_t)quad;
        parent[cb + quad] = (int32_t)q;
        level[cb + quad] = next_level;
    }
}

__global__ void k_leaf_index(int64_t nnodes, const int32_t *__restrict__ leaf,
                             const int32_t *__restrict__ offs, int32_t *__restrict__ node_leaf,
                             int32_t *__restrict__ leaf_node)
{
    int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnodes) return;
    if (leaf[q]) {
        node_leaf[q] = offs[q];
        leaf_node[offs[q]] = (int32_t)q;
    } else {
        node_leaf[q] = -1;
    }
}

__global__ void k_zero_first(int64_t *p) { p[0] = 0; }

struct LevelRanges {
    int64_t lo[KEY_BITS + 2], hi[KEY_BITS + 2];
};

__device__ inline int64_t find_code(const uint64_t *code, int64_t lo, int64_t hi, uint64_t v)
{
    int64_t a = lo, b = hi;
    while (a < b) {
        int64_t mid = (a + b) >> 1;
        if (code[mid] < v) a = mid + 1;
        else b = mid;
    }
    return (a < hi && code[a] == v) ? a : -1;
}

// interaction squares of every node of level >= 2: the children of the
// parent's 3x3 block that are outside the node's own 3x3 block (27 of them)
__global__ void k_ilist(int64_t lo, int64_t hi, LevelRanges lr, const uint64_t *__restrict__ code,
                        const int32_t *__restrict__ level, const uint64_t *__restrict__ keys,
                        int32_t n, IEntry *__restrict__ list)
{
    int64_t q = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= hi) return;
    int lev = level[q];
    uint64_t c = code[q];
    int64_t i = compact_bits(c), j = compact_bits(c >> 1);
    int64_t pi = i >> 1, pj = j >> 1, side = 1ll << lev;
    int sh = 2 * (KEY_BITS - lev);
    int e = 0;
    for (int64_t qj = pj - 1; qj <= pj + 1; ++qj)
        for (int64_t qi = pi - 1; qi <= pi + 1; ++qi)
            for (int cj = 0; cj < 2; ++cj)
                for (int ci = 0; ci < 2; ++ci) {
                    int64_t si = 2 * qi + ci, sj = 2 * qj + cj;
                    int64_t dx = si - i, dy = sj - j;
                    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
                    IEntry en;
                    en.off = (int32_t)((dx + 3) + 7 * (dy + 3));
                    en.src = -2;
                    en.slo = en.shi = 0;
                    if (si >= 0 && sj >= 0 && si < side && sj < side) {
                        uint64_t sc = morton2((uint32_t)si, (uint32_t)sj);
                        int64_t s = find_code(code, lr.lo[lev], lr.hi[lev], sc);
                        if (s >= 0) {
                            en.src = (int32_t)s;
                        } else {
                            int32_t a = lower_bound_u64(keys, n, sc << sh);
                            int32_t b = lower_bound_u64(keys, n, (sc + 1) << sh);
                            if (b > a) {
                                en.src = -1;
                                en.slo = a;
                                en.shi = b;
                            }
                        }
                    }
                    list[(q - lo) * NLIST + e++] = en;
                }
}

template <class T>
T *grow_keep(DevBuf &b, size_t used_elems, size_t need_elems, hipStream_t st)
{
    size_t need = need_elems * sizeof(T);
    if (need <= b.cap) return b.as<T>();
    size_t cap = b.cap ? b.cap : 4096;
    while (cap < need) cap *= 2;
    void *p = nullptr;
    MLM_HIP(hipMalloc(&p, cap));
    if (b.p && used_elems) MLM_HIP(hipMemcpyAsync(p, b.p, used_elems * sizeof(T), hipMemcpyDeviceToDevice, st));
    MLM_HIP(hipStreamSynchronize(st));
    if (b.p) MLM_HIP(hipFree(b.p));
    b.p = p;
    b.cap = cap;
    return static_cast<T *>(p);
}

void *cub_tmp(Workspace &ws, size_t bytes) { return ws.cub_tmp.reserve(bytes ? bytes : 1); }

// exclusive prefix sum of n int32 flags; returns the total
int64_t scan_total(mlm_lens *lens, const int32_t *in, int32_t *out, int64_t n, hipStream_t st)
{
    Workspace &ws = lens->ws;
    if (n == 0) return 0;
    size_t tb = 0;
    MLM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, st));
    void *tmp = cub_tmp(ws, tb);
    MLM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, st));
    int32_t *h = static_cast<int32_t *>(pinned(lens, 2 * sizeof(int32_t)));
    MLM_HIP(hipMemcpyAsync(h, out + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipMemcpyAsync(h + 1, in + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    return (int64_t)h[0] + h[1];
}

}  // namespace

int64_t scan_total_public(mlm_lens *lens, const int32_t *in, int32_t *out, int64_t n, hipStream_t st)
{
    return scan_total(lens, in, out, n, st);
}

// exclusive prefix sum of n int32 counts into n + 1 int64 offsets (the last
// one is the total, which is returned)
int64_t scan_i32_to_i64(mlm_lens *lens, const int32_t *in, int64_t *out, int64_t n, hipStream_t st)
{
    Workspace &ws = lens->ws;
    if (n == 0) return 0;
    size_t tb = 0;
    MLM_HIP(hipcub::DeviceScan::InclusiveSum(nullptr, tb, in, out + 1, (int)n, st));
    void *tmp = cub_tmp(ws, tb);
    hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, st, out);
    MLM_HIP(hipcub::DeviceScan::InclusiveSum(tmp, tb, in, out + 1, (int)n, st));
    int64_t *h = static_cast<int64_t *>(pinned(lens, sizeof(int64_t)));
    MLM_HIP(hipMemcpyAsync(h, out + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    return h[0];
}

// exclusive prefix sum of n int32 counts into n + 1 uint64 offsets; returns the total
int64_t scan_i32_to_u64(mlm_lens *lens, const int32_t *in, unsigned long long *out, int64_t n, hipStream_t st)
{
    return scan_i32_to_i64(lens, in, reinterpret_cast<int64_t *>(out), n, st);
}

// exclusive prefix sum of n int64 values; returns the total
int64_t scan_total_i64(mlm_lens *lens, const int64_t *in, int64_t *out, int64_t n, hipStream_t st)
{
    Workspace &ws = lens->ws;
    if (n == 0) return 0;
    size_t tb = 0;
    MLM_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, in, out, (int)n, st));
    void *tmp = cub_tmp(ws, tb);
    MLM_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, tb, in, out, (int)n, st));
    int64_t *h = static_cast<int64_t *>(pinned(lens, 2 * sizeof(int64_t)));
    MLM_HIP(hipMemcpyAsync(h, out + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipMemcpyAsync(h + 1, in + n - 1, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    MLM_HIP(hipStreamSynchronize(st));
    return h[0] + h[1];
}

void build_tree(mlm_lens *lens, const Region &R, const mlm_map_request &req, Tree &T, hipStream_t st)
{
    Workspace &ws = lens->ws;
    const int32_t n = (int32_t)lens->n;
    T.L0 = R.L0;
    T.L0_exp = R.L0_exp;
    T.nmax = req.leaf_max > 0 ? req.leaf_max : 32;
    T.lmax = (req.max_level > 0 && req.max_level < KEY_BITS) ? req.max_level : KEY_BITS;
    T.n = n;

    // 1. Morton keys of the stars at the finest level, radix sort, gather
    size_t nn = (size_t)(n > 0 ? n : 1);
    uint64_t *kin = static_cast<uint64_t *>(ws.keys_in.reserve(nn * 8));
    uint64_t *kout = static_cast<uint64_t *>(ws.keys.reserve(nn * 8));
    int32_t *iin = static_cast<int32_t *>(ws.idx_in.reserve(nn * 4));
    int32_t *iout = static_cast<int32_t *>(ws.idx.reserve(nn * 4));
    T.x = static_cast<double *>(ws.sx.reserve(nn * 8));
    T.y = static_cast<double *>(ws.sy.reserve(nn * 8));
    T.m = static_cast<double *>(ws.sm.reserve(nn * 8));
    T.keys = kout;
    if (n > 0) {
        double scale = std::ldexp(1.0, KEY_BITS - R.L0_exp);   // 2^24 / (2 L0)
        hipLaunchKernelGGL(k_keys, dim3(nblocks(n)), dim3(BLK), 0, st, lens->d_x, lens->d_y, n, R.L0,
                           scale, kin, iin);
        size_t tb = 0;
        MLM_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, kin, kout, iin, iout, n, 0, 2 * KEY_BITS, st));
        void *tmp = cub_tmp(ws, tb);
        MLM_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, tb, kin, kout, iin, iout, n, 0, 2 * KEY_BITS, st));
        hipLaunchKernelGGL(k_gather, dim3(nblocks(n)), dim3(BLK), 0, st, iout, lens->d_x, lens->d_y,
                           lens->d_m, n, T.x, T.y, T.m);
    }

    // 2. levels, top down
    T.level_lo.assign(1, 0);
    T.level_hi.assign(1, 1);
    size_t used = 0;
    auto ensure = [&](size_t need) {
        T.code = grow_keep<uint64_t>(ws.code, used, need, st);
        T.level = grow_keep<int32_t>(ws.level, used, need, st);
        T.leaf = grow_keep<int32_t>(ws.leaf, used, need, st);
        T.slo = grow_keep<int32_t>(ws.slo, used, need, st);
        T.shi = grow_keep<int32_t>(ws.shi, used, need, st);
        T.block = grow_keep<int32_t>(ws.block, used, need, st);
        T.parent = grow_keep<int32_t>(ws.parent, used, need, st);
        T.child0 = grow_keep<int32_t>(ws.child0, used, need, st);
    };
    ensure(1024);
    hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, st, T.code, T.level, T.parent);
    used = 1;
    for (int lev = 0;; ++lev) {
        int64_t lo = T.level_lo[lev], hi = T.level_hi[lev], nl = hi - lo;
        int32_t *flags = static_cast<int32_t *>(ws.flags.reserve(nl * 4));
        int32_t *offs = static_cast<int32_t *>(ws.offs.reserve(nl * 4));
        hipLaunchKernelGGL(k_level, dim3(nblocks(nl)), dim3(BLK), 0, st, lo, hi, lev, T.lmax, T.nmax,
                           T.code, T.keys, n, T.slo, T.shi, T.block, flags);
        int64_t nsplit = scan_total(lens, flags, offs, nl, st);
        if (hi + 4 * nsplit > (int64_t)INT32_MAX) fail(MLM_ERANGE, "tree too large");
        ensure((size_t)(hi + 4 * nsplit));
        hipLaunchKernelGGL(k_emit, dim3(nblocks(nl)), dim3(BLK), 0, st, lo, hi, hi, flags, offs, T.code,
                           T.level, T.parent, T.child0, T.leaf, lev + 1);
        used = (size_t)(hi + 4 * nsplit);
        if (nsplit == 0) {
            T.nlevels = lev + 1;
            break;
        }
        T.level_lo.push_back(hi);
        T.level_hi.push_back(hi + 4 * nsplit);
    }
    T.nnodes = T.level_hi.back();

    // 3. leaf numbering
    int32_t *offs = static_cast<int32_t *>(ws.offs.reserve(T.nnodes * 4));
    T.node_leaf = static_cast<int32_t *>(ws.node_leaf.reserve(T.nnodes * 4));
    T.nleaves = scan_total(lens, T.leaf, offs, T.nnodes, st);
    T.leaf_node = static_cast<int32_t *>(ws.leaf_node.reserve(T.nleaves * 4));
    hipLaunchKernelGGL(k_leaf_index, dim3(nblocks(T.nnodes)), dim3(BLK), 0, st, T.nnodes, T.leaf, offs,
                       T.node_leaf, T.leaf_node);

    // 4. interaction lists of the nodes of levels >= 2
    T.ilist = static_cast<IEntry *>(ws.ilist.reserve((size_t)T.nnodes * NLIST * sizeof(IEntry)));
    if (T.nlevels > 2) {
        LevelRanges lr{};
        for (int l = 0; l < T.nlevels; ++l) {
            lr.lo[l] = T.level_lo[l];
            lr.hi[l] = T.level_hi[l];
        }
        int64_t lo = T.level_lo[2], hi = T.nnodes;
        hipLaunchKernelGGL(k_ilist, dim3(nblocks(hi - lo)), dim3(BLK), 0, st, lo, hi, lr, T.code,
                           T.level, T.keys, n, T.ilist + lo * NLIST);
    }
}

}  // namespace mlm
