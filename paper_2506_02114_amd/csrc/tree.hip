// Quadtree of the FMM (sec. 3.3, app. C.1), built on the device.
//
// Stars are sorted by their Morton key at the finest level (24 bits per axis),
// so the stars of any square of any level are one contiguous range of the
// sorted array.  The tree is then built level by level from the root: a node
// is divided into four children when the stars of its 3x3 block of
// same-level squares (the node and its neighbours) exceed nmax.  A divided
// node always gets all four children, so every square of a level inside the
// root is a node or lies inside a leaf of a coarser level; each node keeps its
// 3x3 neighbourhood as such references ("colleagues"), found from its
// parent's in O(1), and the block count and the interaction lists follow
// from them without searching the whole key array.
#include <atomic>
#include <chrono>

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

// star range of each node's square: a sub-range of its parent's
__global__ void k_level(int64_t lo, int64_t hi, int lev, const uint64_t *__restrict__ code,
                        const int32_t *__restrict__ parent, const uint64_t *__restrict__ keys, int32_t n,
                        int32_t *__restrict__ slo, int32_t *__restrict__ shi)
{
    const int64_t q = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= hi) return;
    if (lev == 0) {
        slo[q] = 0;
        shi[q] = n;
        return;
    }
    const uint64_t c = code[q];
    const int sh = 2 * (KEY_BITS - lev);
    const int32_t pq = parent[q], a = slo[pq], b = shi[pq];
    const int32_t s0 = a + lower_bound_u64(keys + a, b - a, c << sh);
    slo[q] = s0;
    shi[q] = s0 + lower_bound_u64(keys + s0, b - s0, (c + 1) << sh);
}

// A colleague reference: >= 0 a node of the same level, -1 nothing (outside
// the root), <= -2 the leaf -(ref + 2) of a coarser level containing the square.
// Stars of square `sc` (level shift sh) inside the reference's range.
__device__ inline void ref_stars(int32_t ref, uint64_t sc, int sh, const int32_t *__restrict__ slo,
                                 const int32_t *__restrict__ shi, const uint64_t *__restrict__ keys, int32_t &s0,
                                 int32_t &s1)
{
    s0 = s1 = 0;
    if (ref >= 0) {
        s0 = slo[ref];
        s1 = shi[ref];
    } else if (ref <= -2) {
        const int32_t L = -ref - 2, a = slo[L], b = shi[L];
        s0 = a + lower_bound_u64(keys + a, b - a, sc << sh);
        s1 = s0 + lower_bound_u64(keys + s0, b - s0, (sc + 1) << sh);
    }
}

// square (a, b) of level lev, one of the children of the parent-level
// reference pc: its own reference
__device__ inline int32_t child_ref(int32_t pc, uint32_t a, uint32_t b, const int32_t *__restrict__ child0)
{
    if (pc == -1) return -1;
    if (pc <= -2) return pc;
    const int32_t c0 = child0[pc];
    return c0 >= 0 ? c0 + (int32_t)((a & 1u) | ((b & 1u) << 1)) : -(pc + 2);
}

// colleagues of each node (from its parent's), the star count of its 3x3
// block and whether it is divided
__global__ void k_block(int64_t lo, int64_t hi, int lev, int lmax, int nmax, const uint64_t *__restrict__ code,
                        const int32_t *__restrict__ parent, const int32_t *__restrict__ child0,
                        const int32_t *__restrict__ slo, const int32_t *__restrict__ shi,
                        const uint64_t *__restrict__ keys, int32_t *__restrict__ coll,
                        int32_t *__restrict__ block, int32_t *__restrict__ split)
{
    const int64_t q = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= hi) return;
    const uint64_t c = code[q];
    const int64_t i = compact_bits(c), j = compact_bits(c >> 1), side = 1ll << lev;
    const int sh = 2 * (KEY_BITS - lev);
    const int32_t pq = lev > 0 ? parent[q] : -1;
    int32_t blk = 0;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            const int64_t a = i + di, b = j + dj;
            int32_t ref = -1;
            if (a >= 0 && b >= 0 && a < side && b < side) {
                if (lev == 0) {
                    ref = (int32_t)q;
                } else {
                    const int k = (int)((b >> 1) - (j >> 1) + 1) * 3 + (int)((a >> 1) - (i >> 1) + 1);
                    ref = child_ref(coll[(int64_t)pq * 9 + k], (uint32_t)a, (uint32_t)b, child0);
                }
            }
            coll[q * 9 + (dj + 1) * 3 + (di + 1)] = ref;
            int32_t s0, s1;
            ref_stars(ref, morton2((uint32_t)(a < 0 ? 0 : a), (uint32_t)(b < 0 ? 0 : b)), sh, slo, shi, keys, s0,
                      s1);
            blk += s1 - s0;
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

// interaction squares of every node of level >= 2: the children of the
// parent's 3x3 block that are outside the node's own 3x3 block (27 of them),
// read from the parent's colleagues: a node (M2L), a part of a leaf (P2L from
// its stars in the square) or nothing
__global__ void k_ilist(int64_t lo, int64_t hi, const uint64_t *__restrict__ code,
                        const int32_t *__restrict__ level, const int32_t *__restrict__ parent,
                        const int32_t *__restrict__ child0, const int32_t *__restrict__ slo,
                        const int32_t *__restrict__ shi, const uint64_t *__restrict__ keys,
                        const int32_t *__restrict__ coll, IEntry *__restrict__ list)
{
    const int64_t q = lo + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= hi) return;
    const int lev = level[q];
    const uint64_t c = code[q];
    const int64_t i = compact_bits(c), j = compact_bits(c >> 1);
    const int64_t pi = i >> 1, pj = j >> 1;
    const int sh = 2 * (KEY_BITS - lev);
    const int32_t *pc = coll + (int64_t)parent[q] * 9;
    int e = 0;
    for (int qj = -1; qj <= 1; ++qj)
        for (int qi = -1; qi <= 1; ++qi) {
            const int32_t pref = pc[(qj + 1) * 3 + (qi + 1)];
            for (int cj = 0; cj < 2; ++cj)
                for (int ci = 0; ci < 2; ++ci) {
                    const int64_t si = 2 * (pi + qi) + ci, sj = 2 * (pj + qj) + cj;
                    const int64_t dx = si - i, dy = sj - j;
                    if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1) continue;
                    IEntry en;
                    en.off = (int32_t)((dx + 3) + 7 * (dy + 3));
                    en.src = -2;
                    en.slo = en.shi = 0;
                    const int32_t ref = child_ref(pref, (uint32_t)si, (uint32_t)sj, child0);
                    if (ref >= 0) {
                        en.src = ref;
                    } else if (ref <= -2) {
                        int32_t s0, s1;
                        ref_stars(ref, morton2((uint32_t)si, (uint32_t)sj), sh, slo, shi, keys, s0, s1);
                        if (s1 > s0) {
                            en.src = -1;
                            en.slo = s0;
                            en.shi = s1;
                        }
                    }
                    list[(q - lo) * NLIST + e++] = en;
                }
        }
}

template <class T>
T *grow_keep(DevBuf &b, size_t used_elems, size_t need_elems, hipStream_t st)
{
    return static_cast<T *>(b.grow_keep(used_elems * sizeof(T), need_elems * sizeof(T), st));
}

void *scan_tmp(Workspace &ws, size_t bytes) { return ws.scan_tmp.reserve(bytes ? bytes : 1); }

// A scan's total, read back to the host: the scan stores it straight into a
// coherent pinned slot with a sequence number behind it, and the host spins
// until that number appears instead of synchronising the stream (whose
// wake-up would add its latency to every tree level and count).  After a
// short spin it blocks on the stream instead, which also reports any error
// of the queued work.  Inside a scratch arena (no pinned slot) the total goes
// to a scratch slot that is copied, after a synchronisation.
struct TotalSlot {
    int64_t *dev = nullptr, *host = nullptr;
    int64_t seq = 0;
};

TotalSlot total_slot(mlm_lens *lens)
{
    TotalSlot t;
    if (Arena *a = thread_arena()) {
        t.dev = static_cast<int64_t *>(a->take(sizeof(int64_t)));
        return t;
    }
    Workspace &ws = lens->ws;
    if (!ws.spin) ws.spin = static_cast<int64_t *>(coherent_pinned(2 * sizeof(int64_t)));
    t.host = ws.spin;
    t.seq = ++ws.spin_seq;
    return t;
}

int64_t read_total(const TotalSlot &t, hipStream_t st)
{
    if (t.dev) {
        int64_t v = 0;
        MLM_HIP(hipMemcpyAsync(&v, t.dev, sizeof v, hipMemcpyDeviceToHost, st));
        MLM_HIP(hipStreamSynchronize(st));
        return v;
    }
    const volatile int64_t *h = t.host;
    const auto t0 = std::chrono::steady_clock::now();
    for (int k = 1; h[1] != t.seq; ++k) {
        if ((k & 255) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(200)) {
            MLM_HIP(hipStreamSynchronize(st));
            if (h[1] != t.seq) fail(MLM_EDEVICE, "a scan's total did not arrive");
            break;
        }
        __builtin_ia32_pause();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    return h[0];
}

// exclusive prefix sum of n int32 flags; returns the total
int64_t scan_total(mlm_lens *lens, const int32_t *in, int32_t *out, int64_t n, hipStream_t st)
{
    if (n == 0) return 0;
    const TotalSlot t = total_slot(lens);
    dev_scan_i32(in, out, n, false, scan_tmp(lens->ws, scan_tmp_bytes(n)), t.dev, t.host, t.seq, st);
    return read_total(t, st);
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
    if (n == 0) return 0;
    const TotalSlot t = total_slot(lens);
    hipLaunchKernelGGL(k_zero_first, dim3(1), dim3(1), 0, st, out);
    dev_scan_i32_i64(in, out + 1, n, true, scan_tmp(lens->ws, scan_tmp_bytes(n)), t.dev, t.host, t.seq, st);
    return read_total(t, st);
}

// exclusive prefix sum of n int32 counts into n + 1 uint64 offsets; returns the total
int64_t scan_i32_to_u64(mlm_lens *lens, const int32_t *in, unsigned long long *out, int64_t n, hipStream_t st)
{
    return scan_i32_to_i64(lens, in, reinterpret_cast<int64_t *>(out), n, st);
}

// exclusive prefix sum of n int64 values; returns the total
int64_t scan_total_i64(mlm_lens *lens, const int64_t *in, int64_t *out, int64_t n, hipStream_t st)
{
    if (n == 0) return 0;
    const TotalSlot t = total_slot(lens);
    dev_scan_i64(in, out, n, false, scan_tmp(lens->ws, scan_tmp_bytes(n)), t.dev, t.host, t.seq, st);
    return read_total(t, st);
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
        radix_sort_pairs(kin, iin, kout, iout, n, 2 * KEY_BITS, scan_tmp(ws, radix_sort_tmp_bytes(n)), st);
        hipLaunchKernelGGL(k_gather, dim3(nblocks(n)), dim3(BLK), 0, st, iout, lens->d_x, lens->d_y,
                           lens->d_m, n, T.x, T.y, T.m);
    }

    // 2. levels, top down
    T.level_lo.assign(1, 0);
    T.level_hi.assign(1, 1);
    size_t used = 0;
    int32_t *coll = nullptr;   // 9 colleague references per node
    auto ensure = [&](size_t need) {
        T.code = grow_keep<uint64_t>(ws.code, used, need, st);
        T.level = grow_keep<int32_t>(ws.level, used, need, st);
        T.leaf = grow_keep<int32_t>(ws.leaf, used, need, st);
        T.slo = grow_keep<int32_t>(ws.slo, used, need, st);
        T.shi = grow_keep<int32_t>(ws.shi, used, need, st);
        T.block = grow_keep<int32_t>(ws.block, used, need, st);
        T.parent = grow_keep<int32_t>(ws.parent, used, need, st);
        T.child0 = grow_keep<int32_t>(ws.child0, used, need, st);
        coll = grow_keep<int32_t>(ws.coll, 9 * used, 9 * need, st);
    };
    ensure(1024);
    hipLaunchKernelGGL(k_root, dim3(1), dim3(1), 0, st, T.code, T.level, T.parent);
    used = 1;
    for (int lev = 0;; ++lev) {
        int64_t lo = T.level_lo[lev], hi = T.level_hi[lev], nl = hi - lo;
        int32_t *flags = static_cast<int32_t *>(ws.flags.reserve(nl * 4));
        int32_t *offs = static_cast<int32_t *>(ws.offs.reserve(nl * 4));
        hipLaunchKernelGGL(k_level, dim3(nblocks(nl)), dim3(BLK), 0, st, lo, hi, lev, T.code, T.parent, T.keys, n,
                           T.slo, T.shi);
        hipLaunchKernelGGL(k_block, dim3(nblocks(nl)), dim3(BLK), 0, st, lo, hi, lev, T.lmax, T.nmax, T.code,
                           T.parent, T.child0, T.slo, T.shi, T.keys, coll, T.block, flags);
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
        int64_t lo = T.level_lo[2], hi = T.nnodes;
        hipLaunchKernelGGL(k_ilist, dim3(nblocks(hi - lo)), dim3(BLK), 0, st, lo, hi, T.code, T.level, T.parent,
                           T.child0, T.slo, T.shi, T.keys, coll, T.ilist + lo * NLIST);
    }
}

}  // namespace mlm
