// Device-wide prefix sums and the radix sort of the stars' Morton keys,
// written for CDNA wavefronts (64 lanes) and launched with sizes known on the
// host, so no hidden fills or host reads are made: every launch is a plain
// kernel on the caller's stream.
//
// Scan: a tile of 2048 items per 256-thread workgroup.  Pass 1 sums each tile,
// pass 2 (one workgroup) scans the tile sums in place and stores the total
// where asked, pass 3 scans each tile again with its offset.  A single tile
// needs pass 3 only.
//
// Sort: least-significant-digit radix sort of (64-bit key, 32-bit value) pairs,
// 8-bit digits.  Per digit: a 256-bin histogram per tile, stored digit-major
// (so one exclusive scan of the whole table gives every (digit, tile) its
// output offset), then a stable scatter: items are ranked in tile order, one
// round of 256 at a time; inside a wavefront, lanes with the same digit are
// found with eight ballots, and earlier wavefronts' counts come from LDS.
#include "dev.hpp"

namespace mlm {

namespace {

constexpr int SC_THREADS = 256;
constexpr int SC_ITEMS = 8;
constexpr int64_t SC_TILE = SC_THREADS * SC_ITEMS;   // 2048

inline unsigned sc_tiles(int64_t n) { return (unsigned)((n + SC_TILE - 1) / SC_TILE); }

// exclusive scan of one value per thread over the workgroup (256 threads);
// part: 4 LDS slots; returns the workgroup total in `total`
template <class T>
__device__ inline T block_excl_scan(T v, T *part, T &total)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    T incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const T o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) part[wave] = incl;
    __syncthreads();
    T before = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < SC_THREADS / 64; ++w) {
        const T p = part[w];
        if (w < wave) before += p;
        total += p;
    }
    __syncthreads();   // part may be reused
    return before + incl - v;
}

template <class TI, class TO>
__global__ __launch_bounds__(SC_THREADS) void k_tile_sums(const TI *__restrict__ in, int64_t n, TO *__restrict__ sums)
{
    __shared__ TO part[SC_THREADS / 64];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    TO s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        const int64_t i = base + k * SC_THREADS + threadIdx.x;   // coalesced; the order inside a tile is free here
        if (i < n) s += (TO)in[i];
    }
    TO total;
    (void)block_excl_scan(s, part, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// exclusive scan of the nt tile sums in place (one workgroup); the total goes
// to total_dev and/or total_host when given
// the total to the host: the value, then its sequence number behind a
// system-scope fence, so a host thread that sees the number sees the value
__device__ inline void store_host_total(int64_t *total_host, int64_t v, int64_t seq)
{
    total_host[0] = v;
    __threadfence_system();
    __hip_atomic_store(total_host + 1, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

template <class TO>
__global__ __launch_bounds__(SC_THREADS) void k_scan_sums(TO *__restrict__ sums, int64_t nt, int64_t *total_dev,
                                                         int64_t *total_host, int64_t seq)
{
    __shared__ TO part[SC_THREADS / 64];
    TO carry = 0;
    for (int64_t b = 0; b < nt; b += SC_THREADS) {
        const int64_t i = b + threadIdx.x;
        const TO v = i < nt ? sums[i] : (TO)0;
        TO total;
        const TO e = block_excl_scan(v, part, total);
        if (i < nt) sums[i] = carry + e;
        carry += total;
    }
    if (threadIdx.x == 0) {
        if (total_dev) *total_dev = (int64_t)carry;
        if (total_host) store_host_total(total_host, (int64_t)carry, seq);
    }
}

// each tile scanned with its offset (offs: the scanned tile sums, or null for
// a single tile); thread t takes the consecutive items t*8 .. t*8+7 of the
// tile.  Exclusive or inclusive; out may not alias in.  With one tile the
// total is stored here.
template <class TI, class TO>
__global__ __launch_bounds__(SC_THREADS) void k_tile_scan(const TI *__restrict__ in, int64_t n,
                                                         const TO *__restrict__ offs, TO *__restrict__ out,
                                                         int inclusive, int64_t *total_dev, int64_t *total_host,
                                                         int64_t seq)
{
    __shared__ TO part[SC_THREADS / 64];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + (int64_t)threadIdx.x * SC_ITEMS;
    TO v[SC_ITEMS];
    TO s = 0;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        v[k] = base + k < n ? (TO)in[base + k] : (TO)0;
        s += v[k];
    }
    TO total;
    TO run = block_excl_scan(s, part, total) + (offs ? offs[blockIdx.x] : (TO)0);
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        if (base + k < n) out[base + k] = inclusive ? run + v[k] : run;
        run += v[k];
    }
    if (!offs && threadIdx.x == 0) {
        if (total_dev) *total_dev = (int64_t)total;
        if (total_host) store_host_total(total_host, (int64_t)total, seq);
    }
}

// ---------------------------------------------------------------------------
// radix sort
// ---------------------------------------------------------------------------
constexpr int RS_BINS = 256;

__global__ __launch_bounds__(SC_THREADS) void k_rs_hist(const uint64_t *__restrict__ key, int64_t n, int shift,
                                                       int32_t *__restrict__ hist, int64_t ntiles)
{
    __shared__ int32_t h[RS_BINS];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
#pragma unroll
    for (int k = 0; k < SC_ITEMS; ++k) {
        const int64_t i = base + k * SC_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(int)((key[i] >> shift) & 0xff)], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];   // digit-major
}

// stable scatter of one tile: items in tile order, 256 per round (item
// r * 256 + t in thread t); offs is the scanned digit-major histogram
__global__ __launch_bounds__(SC_THREADS) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                          const int32_t *__restrict__ vin, int64_t n, int shift,
                                                          const int32_t *__restrict__ offs, int64_t ntiles,
                                                          uint64_t *__restrict__ kout, int32_t *__restrict__ vout)
{
    __shared__ int32_t dbase[RS_BINS];              // next output slot of each digit in this tile
    __shared__ int32_t wcnt[SC_THREADS / 64][RS_BINS];   // this round's count per wavefront and digit
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    dbase[t] = offs[(int64_t)t * ntiles + blockIdx.x];
    for (int w = 0; w < SC_THREADS / 64; ++w) wcnt[w][t] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SC_TILE;
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int r = 0; r < SC_ITEMS; ++r) {
        const int64_t i = base + r * SC_THREADS + t;
        const bool valid = i < n;
        uint64_t k = 0;
        int32_t v = 0;
        int d = 0;
        if (valid) {
            k = kin[i];
            v = vin[i];
            d = (int)((k >> shift) & 0xff);
        }
        // lanes of this wavefront holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int rank = __popcll(same & lt);
        const bool leader = valid && rank == 0;
        if (leader) wcnt[wave][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int32_t pos = dbase[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        // thread t owns digit t (as many threads as digits): advance its base by
        // the round's count and clear the round's table
        int32_t s = 0;
#pragma unroll
        for (int w = 0; w < SC_THREADS / 64; ++w) {
            s += wcnt[w][t];
            wcnt[w][t] = 0;
        }
        dbase[t] += s;
        __syncthreads();
    }
}

template <class TI, class TO>
void scan_launch(const TI *in, TO *out, int64_t n, bool inclusive, TO *tile_sums, int64_t *total_dev,
                 int64_t *total_host, int64_t seq, hipStream_t st)
{
    const unsigned nt = sc_tiles(n);
    if (nt <= 1) {
        hipLaunchKernelGGL((k_tile_scan<TI, TO>), dim3(1), dim3(SC_THREADS), 0, st, in, n, (const TO *)nullptr, out,
                           inclusive ? 1 : 0, total_dev, total_host, seq);
        return;
    }
    hipLaunchKernelGGL((k_tile_sums<TI, TO>), dim3(nt), dim3(SC_THREADS), 0, st, in, n, tile_sums);
    hipLaunchKernelGGL((k_scan_sums<TO>), dim3(1), dim3(SC_THREADS), 0, st, tile_sums, (int64_t)nt, total_dev,
                       total_host, seq);
    hipLaunchKernelGGL((k_tile_scan<TI, TO>), dim3(nt), dim3(SC_THREADS), 0, st, in, n, (const TO *)tile_sums, out,
                       inclusive ? 1 : 0, (int64_t *)nullptr, (int64_t *)nullptr, (int64_t)0);
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return (size_t)(sc_tiles(n) + 1) * sizeof(int64_t); }

void dev_scan_i32(const int32_t *in, int32_t *out, int64_t n, bool inclusive, void *tmp, int64_t *total_dev,
                  int64_t *total_host, int64_t seq, hipStream_t st)
{
    if (n > 0)
        scan_launch<int32_t, int32_t>(in, out, n, inclusive, static_cast<int32_t *>(tmp), total_dev, total_host, seq, st);
}

void dev_scan_i32_i64(const int32_t *in, int64_t *out, int64_t n, bool inclusive, void *tmp, int64_t *total_dev,
                      int64_t *total_host, int64_t seq, hipStream_t st)
{
    if (n > 0)
        scan_launch<int32_t, int64_t>(in, out, n, inclusive, static_cast<int64_t *>(tmp), total_dev, total_host, seq, st);
}

void dev_scan_i64(const int64_t *in, int64_t *out, int64_t n, bool inclusive, void *tmp, int64_t *total_dev,
                  int64_t *total_host, int64_t seq, hipStream_t st)
{
    if (n > 0)
        scan_launch<int64_t, int64_t>(in, out, n, inclusive, static_cast<int64_t *>(tmp), total_dev, total_host, seq, st);
}

size_t radix_sort_tmp_bytes(int64_t n)
{
    const int64_t nt = sc_tiles(n);
    // digit-major histogram, its scan, the scan's tile sums
    return (size_t)(2 * RS_BINS * nt) * sizeof(int32_t) + scan_tmp_bytes(RS_BINS * nt) + 256;
}

// Stable sort of (key, value) pairs by bits [0, bits) of the key; the result
// ends in kout/vout.  kin/vin are overwritten (ping-pong buffers).
void radix_sort_pairs(uint64_t *kin, int32_t *vin, uint64_t *kout, int32_t *vout, int64_t n, int bits, void *tmp,
                      hipStream_t st)
{
    if (n <= 0) return;
    const int64_t nt = sc_tiles(n);
    int32_t *hist = static_cast<int32_t *>(tmp);
    int32_t *offs = hist + RS_BINS * nt;
    void *stmp = offs + RS_BINS * nt;
    const int passes = (bits + 7) / 8;
    uint64_t *ka = kin, *kb = kout;
    int32_t *va = vin, *vb = vout;
    for (int p = 0; p < passes; ++p) {
        // the last pass must land in kout: with an even number of passes the
        // first one writes into kin's partner so the ping-pong ends right
        uint64_t *ks = ka, *kd = kb;
        int32_t *vs = va, *vd = vb;
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)nt), dim3(SC_THREADS), 0, st, ks, n, 8 * p, hist, nt);
        scan_launch<int32_t, int32_t>(hist, offs, RS_BINS * nt, false, static_cast<int32_t *>(stmp), nullptr, nullptr,
                                      0, st);
        hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)nt), dim3(SC_THREADS), 0, st, ks, vs, n, 8 * p, offs, nt, kd,
                           vd);
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != kout) {   // odd number of passes: the result is in kin's buffers
        MLM_HIP(hipMemcpyAsync(kout, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        MLM_HIP(hipMemcpyAsync(vout, va, (size_t)n * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    }
}

}  // namespace mlm
