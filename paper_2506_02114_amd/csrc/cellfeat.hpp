// Per-cell inputs of the refinement network: the mapped corners of a ray-grid
// cell reduced to 12 features, and whether the cell is folded (its mapped ears
// disagree in orientation: a critical curve crosses it).  Shared by the
// refinement kernels and the fused inference that flags a strip's cells.
#pragma once

#include "dev.hpp"

namespace mlm {

__device__ inline double sgn(double x) { return (double)((x > 0.0) - (x < 0.0)); }

// twice the signed area of (a, b, c), evaluated as written
__device__ inline double area2(double ua, double va, double ub, double vb, double uc, double vc)
{
#pragma clang fp contract(off)
    return (ub - ua) * (vc - va) - (uc - ua) * (vb - va);
}

// 12 features of a mapped cell (corners 00, 10, 11, 01 in pixel units):
// sign(d) log(1 + |d|) of the corners' offsets from the corner of the pixel
// holding their mean, then the signs of the mapped ears at the corners.
// Half h of them: features 4h .. 4h + 3 (corners 2h, 2h + 1) to f[0 .. 4),
// ear signs 2h, 2h + 1 to f[4], f[5].
__device__ inline void cell_features_half(const double *u4, const double *v4, int h, float *f)
{
    const double cu = floor(0.25 * (u4[0] + u4[1] + u4[2] + u4[3]));
    const double cv = floor(0.25 * (v4[0] + v4[1] + v4[2] + v4[3]));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = 2 * h + j;
        const double du = u4[k] - cu, dv = v4[k] - cv;
        f[2 * j] = (float)(sgn(du) * log1p(fabs(du)));
        f[2 * j + 1] = (float)(sgn(dv) * log1p(fabs(dv)));
        const int p = (k + 3) & 3, q = (k + 1) & 3;
        f[4 + j] = (float)sgn(area2(u4[k], v4[k], u4[q], v4[q], u4[p], v4[p]));
    }
}

// log(1 + x) for x >= 0 in FP32 from the hardware base-2 logarithm, with the
// correction of Goldberg's theorem 4 ("What every computer scientist should
// know about floating-point arithmetic", 1991): for u = fl(1 + x) != 1,
// log(u) x / (u - 1) keeps the relative error within a few units of the last
// place even where 1 + x rounds, and for u = 1 the value is x itself
__device__ inline float log1p_hw(float x)
{
    const float u = 1.0f + x;
    const float l = __builtin_amdgcn_logf(u) * 0.693147180559945309f;
    return u == 1.0f ? x : l * (x * __builtin_amdgcn_rcpf(u - 1.0f));
}

// The same half of the features with the logarithms in FP32, for the fused
// inference, which rounds its inputs to bf16 (8 significant bits) anyway: the
// offsets and the ear signs are still formed in FP64, and the logarithm is
// within a few FP32 units of its last place, far inside the bf16 rounding.
__device__ inline void cell_features_half_f32(const double *u4, const double *v4, int h, float *f)
{
    const double cu = floor(0.25 * (u4[0] + u4[1] + u4[2] + u4[3]));
    const double cv = floor(0.25 * (v4[0] + v4[1] + v4[2] + v4[3]));
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int k = 2 * h + j;
        const double du = u4[k] - cu, dv = v4[k] - cv;
        f[2 * j] = (float)sgn(du) * log1p_hw((float)fabs(du));
        f[2 * j + 1] = (float)sgn(dv) * log1p_hw((float)fabs(dv));
        const int p = (k + 3) & 3, q = (k + 1) & 3;
        f[4 + j] = (float)sgn(area2(u4[k], v4[k], u4[q], v4[q], u4[p], v4[p]));
    }
}

__device__ inline void cell_features(const double *u4, const double *v4, float *f)
{
    float a[6], b[6];
    cell_features_half(u4, v4, 0, a);
    cell_features_half(u4, v4, 1, b);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        f[k] = a[k];
        f[4 + k] = b[k];
    }
    f[8] = a[4];
    f[9] = a[5];
    f[10] = b[4];
    f[11] = b[5];
}

__device__ inline bool folded(const float *f) { return !(f[8] == f[9] && f[9] == f[10] && f[10] == f[11]); }

}  // namespace mlm
