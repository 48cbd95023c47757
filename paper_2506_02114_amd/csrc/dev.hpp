// Device helpers shared by the library's kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.hpp"

namespace mlm {

// 2-D Morton interleave: bit b of i goes to bit 2b, bit b of j to bit 2b+1
__device__ __host__ inline uint64_t spread_bits(uint32_t v)
{
    uint64_t x = v;
    x = (x | (x << 16)) & 0x0000FFFF0000FFFFull;
    x = (x | (x << 8)) & 0x00FF00FF00FF00FFull;
    x = (x | (x << 4)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x << 2)) & 0x3333333333333333ull;
    x = (x | (x << 1)) & 0x5555555555555555ull;
    return x;
}

__device__ __host__ inline uint32_t compact_bits(uint64_t x)
{
    x &= 0x5555555555555555ull;
    x = (x | (x >> 1)) & 0x3333333333333333ull;
    x = (x | (x >> 2)) & 0x0F0F0F0F0F0F0F0Full;
    x = (x | (x >> 4)) & 0x00FF00FF00FF00FFull;
    x = (x | (x >> 8)) & 0x0000FFFF0000FFFFull;
    x = (x | (x >> 16)) & 0x00000000FFFFFFFFull;
    return (uint32_t)x;
}

__device__ __host__ inline uint64_t morton2(uint32_t i, uint32_t j)
{
    return spread_bits(i) | (spread_bits(j) << 1);
}

// square index of coordinate t at the finest level: floor((t + L0) * 2^KEY_BITS / (2 L0)),
// where scale = 2^KEY_BITS / (2 L0) is a power of two (exact product of the rounded sum)
__device__ inline uint32_t fine_cell(double t, double L0, double scale)
{
    double u = floor((t + L0) * scale);
    const double top = (double)((1u << KEY_BITS) - 1);
    u = u < 0.0 ? 0.0 : (u > top ? top : u);
    return (uint32_t)u;
}

// first index in sorted a[0, n) with a[k] >= v
__device__ inline int32_t lower_bound_u64(const uint64_t *a, int32_t n, uint64_t v)
{
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <class T>
__device__ inline int64_t upper_bound_i64(const T *a, int64_t n, T v)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// complex helpers on double2 (x = real, y = imaginary)
__device__ __host__ inline double2 cmul(double2 a, double2 b)
{
    return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __host__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __host__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 cinv(double2 a)
{
    double r = 1.0 / (a.x * a.x + a.y * a.y);
    return make_double2(a.x * r, -a.y * r);
}
// z^n for n >= 0 by binary powering
__device__ inline double2 cpowi(double2 z, int n)
{
    double2 r = make_double2(1.0, 0.0);
    while (n) {
        if (n & 1) r = cmul(r, z);
        z = cmul(z, z);
        n >>= 1;
    }
    return r;
}

// the same on float2, and the complex type of a real type
__device__ __host__ inline float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __host__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ inline float2 cinv(float2 a)
{
    float r = __builtin_amdgcn_rcpf(a.x * a.x + a.y * a.y);
    return make_float2(a.x * r, -a.y * r);
}
__device__ inline float2 cpowi(float2 z, int n)
{
    float2 r = make_float2(1.0f, 0.0f);
    while (n) {
        if (n & 1) r = cmul(r, z);
        z = cmul(z, z);
        n >>= 1;
    }
    return r;
}

// wavefront-level load balancing: a wavefront owns 64 segments (cells, large
// triangles or rows) with v items each; the exclusive scan of v over the
// lanes numbers the items, and an item finds its segment by binary lifting
// over the lanes' scan values (lane shuffles, no global memory)
__device__ inline int wave_excl_scan(int v, int lane, int &total)
{
    int incl = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    total = __shfl(incl, 63, 64);
    return incl - v;
}

// largest lane L with excl(L) <= x (excl non-decreasing over the lanes); the
// segment of item x has at least one item since excl(L + 1) > x
__device__ inline int wave_find(int excl, int x)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const int e = __shfl(excl, lo + step, 64);
        if (e <= x) lo += step;
    }
    return lo;
}

template <class R> struct Cx;
template <> struct Cx<double> {
    using c2 = double2;
    using v4 = double4;
    __device__ __host__ static c2 make(double a, double b) { return make_double2(a, b); }
    __device__ __host__ static v4 make4(double a, double b, double c) { return make_double4(a, b, c, 0.0); }
};
template <> struct Cx<float> {
    using c2 = float2;
    using v4 = float4;
    __device__ __host__ static c2 make(float a, float b) { return make_float2(a, b); }
    __device__ __host__ static v4 make4(float a, float b, float c) { return make_float4(a, b, c, 0.0f); }
};

// a / b: FP64 division, or a times the FP32 hardware reciprocal (1 ulp)
__device__ inline double qdiv(double a, double b) { return a / b; }

// a / b for the near-field sum: the hardware reciprocal estimate refined by
// two Newton steps y <- y + y (1 - b y) (each doubles the correct bits), then
// one product; within a few ulp of the correctly rounded quotient, and
// non-finite (as the quotient) when b is 0
__device__ inline double near_div(double a, double b)
{
    double y = __builtin_amdgcn_rcp(b);
    y = fma(fma(-b, y, 1.0), y, y);
    y = fma(fma(-b, y, 1.0), y, y);
    return a * y;
}
__device__ inline float near_div(float a, float b) { return qdiv(a, b); }
__device__ inline float qdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

}  // namespace mlm
