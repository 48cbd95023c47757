// The refinement network: 12 -> 64 -> 64 -> 1 with ReLU between layers and a
// logit out, BF16 weights and activations on the matrix cores with FP32
// accumulation (v_mfma_f32_32x32x8_bf16), FP32 master weights and Adam.  The
// hidden activations feeding the second layer are carried as two bf16 parts
// (value and residual, two products each): one bf16 rounding there moves
// pre-activations across the ReLU kink often enough to change gradients by
// percents, while the rounding of weights and back-propagated gradients
// costs about 2^-9.
//
// Parameters (FP32, 5057): W1 [12][64], b1 [64], W2 [64][64], b2 [64],
// W3 [64], b3; layer l computes h_l = relu(h_{l-1} W_l + b_l).
// Loss: mean_i [ w+ y_i softplus(-z_i) + (1 - y_i) softplus(z_i) ].
//
// One wavefront takes 32 samples; a workgroup of four wavefronts takes 128.
// Every product is a 32 x 32 block tile (one MFMA per 8 of the reduced
// dimension) whose operands are read from LDS or global memory with the
// strides that make the transposes of the backward pass free.
#include <algorithm>

#include "cellfeat.hpp"
#include "dev.hpp"

namespace mlm {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int NP = 5057;
constexpr int OW1 = 0, OB1 = 768, OW2 = 832, OB2 = 4928, OW3 = 4992, OB3 = 5056;
constexpr int MB = 128;   // samples per workgroup (4 wavefronts x 32)

// float -> bf16, round to nearest even (finite inputs): one hardware
// conversion (v_cvt_pk_bf16_f32) in the default rounding mode
__device__ inline uint16_t f2bf(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// C (32 x 32 tile) += A (32 x K) B (K x 32); A(m, k) = a[m * sam + k * sak],
// B(k, n) = b[k * sbk + n * sbn] (bf16); K a multiple of 8.  Operand layout
// of the instruction: lane l holds A(l % 32, 4 (l / 32) + t) and
// B(4 (l / 32) + t, l % 32), t < 4.
__device__ inline f32x16 tile_mma(const uint16_t *a, int sam, int sak, const uint16_t *b, int sbk, int sbn, int K,
                                  f32x16 acc, int lane)
{
    const int r = lane & 31, h = (lane >> 5) * 4;
    for (int k0 = 0; k0 < K; k0 += 8) {
        bf16x4 av, bv;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            av[t] = (short)a[r * sam + (k0 + h + t) * sak];
            bv[t] = (short)b[(k0 + h + t) * sbk + r * sbn];
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// row and column of accumulator element j of lane `lane` in a 32 x 32 tile
__device__ inline int acc_row(int j, int lane) { return 8 * (j >> 2) + 4 * (lane >> 5) + (j & 3); }
__device__ inline int acc_col(int lane) { return lane & 31; }

struct WaveLds {
    uint16_t x[32 * 16];     // inputs, 12 features + 4 zero columns
    uint16_t h1[32 * 64];    // layer-1 activations, bf16 part
    uint16_t h1lo[32 * 64];  // and the bf16 residual: h1 + h1lo carries 16 bits
    float h2[32 * 64];       // layer-2 activations
    uint16_t d2[32 * 64];    // gradient at layer-2 pre-activations
    uint16_t d1[32 * 64];    // gradient at layer-1 pre-activations
    float z[32], dz[32];
};

// forward pass of the wavefront's 32 samples [s0, s0 + 32) (rows past n
// are zero); W1b is [16][64] (rows 12..15 zero), W2b [64][64], bf16
__device__ inline void forward(const float *__restrict__ feats, int64_t s0, int64_t n, const uint16_t *__restrict__ W1b,
                               const uint16_t *__restrict__ W2b, const float *__restrict__ P, WaveLds &L, int lane)
{
    for (int e = lane; e < 32 * 16; e += 64) {
        const int m = e >> 4, k = e & 15;
        const int64_t s = s0 + m;
        L.x[e] = (k < 12 && s < n) ? f2bf(feats[s * 12 + k]) : (uint16_t)0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int nh = 0; nh < 2; ++nh) {
        f32x16 acc = {};
        acc = tile_mma(L.x, 16, 1, W1b + nh * 32, 64, 1, 16, acc, lane);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int m = acc_row(j, lane), c = nh * 32 + acc_col(lane);
            const float h = fmaxf(acc[j] + P[OB1 + c], 0.0f);
            const uint16_t hi = f2bf(h);
            L.h1[m * 64 + c] = hi;
            L.h1lo[m * 64 + c] = f2bf(h - bf2f(hi));
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int nh = 0; nh < 2; ++nh) {
        f32x16 acc = {};
        acc = tile_mma(L.h1, 64, 1, W2b + nh * 32, 64, 1, 64, acc, lane);
        acc = tile_mma(L.h1lo, 64, 1, W2b + nh * 32, 64, 1, 64, acc, lane);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int m = acc_row(j, lane), c = nh * 32 + acc_col(lane);
            L.h2[m * 64 + c] = fmaxf(acc[j] + P[OB2 + c], 0.0f);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 32) {
        float z = P[OB3];
        for (int c = 0; c < 64; ++c) z += L.h2[lane * 64 + c] * bf2f(f2bf(P[OW3 + c]));
        L.z[lane] = z;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inference only: the weights are staged once per workgroup in LDS, rows of
// every operand are stored so that the four consecutive values of the
// reduced dimension that a lane feeds one MFMA are one 8-byte LDS read, and
// each wavefront loops over tiles of 32 samples (a grid sized to the device,
// not to the samples).  Same arithmetic as `forward` (bf16 inputs, two-part
// bf16 hidden layer, FP32 accumulation); the final 64-term sum runs in
// another order.
constexpr int PS = 68;    // padded row stride (bf16) of the 64-wide operands: 136 B, so rows fall in other banks
constexpr int XS = 20;    // and of the 16-wide input rows: 40 B

struct PredictLds {
    uint16_t w1t[64 * XS];   // W1 transposed: w1t[n][k] = W1[k][n], k < 16
    uint16_t w2t[64 * PS];   // W2 transposed: w2t[n][k] = W2[k][n]
    float b1[64], b2[64], w3[64];
    struct Wave {
        uint16_t x[32 * XS];   // the tile's inputs, 12 features + 4 zero columns
        uint16_t h1[32 * PS];  // layer-1 activations, bf16 part (then the layer-3 partial sums)
        uint16_t h1lo[32 * PS];
    } w[4];
};

// C (32 x 32) += A (32 x K) B (K x 32), A(m, k) = a[m * sa + k], B(k, n) =
// bt[n * sb + k] (bf16 in LDS, rows 8-byte aligned): one 8-byte read per
// operand and MFMA
__device__ inline f32x16 tile_mma_rows(const uint16_t *a, int sa, const uint16_t *bt, int sb, int K, f32x16 acc,
                                       int lane)
{
    const int r = lane & 31, h = (lane >> 5) * 4;
    for (int k0 = 0; k0 < K; k0 += 8) {
        const bf16x4 av = *reinterpret_cast<const bf16x4 *>(a + r * sa + k0 + h);
        const bf16x4 bv = *reinterpret_cast<const bf16x4 *>(bt + r * sb + k0 + h);
        acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
    }
    return acc;
}

// the weights of the inference into the workgroup's LDS
__device__ inline void stage_weights(PredictLds &S, const uint16_t *__restrict__ W1b, const uint16_t *__restrict__ W2b,
                                     const float *__restrict__ P)
{
    for (int e = threadIdx.x; e < 64 * 64; e += blockDim.x) {
        const int k = e >> 6, c = e & 63;   // W2b[k][c]
        S.w2t[c * PS + k] = W2b[e];
        if (k < 16) S.w1t[c * XS + k] = W1b[e];
    }
    if (threadIdx.x < 64) {
        S.b1[threadIdx.x] = P[OB1 + threadIdx.x];
        S.b2[threadIdx.x] = P[OB2 + threadIdx.x];
        S.w3[threadIdx.x] = bf2f(f2bf(P[OW3 + threadIdx.x]));
    }
}

__device__ inline void wave_sync_lds()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// the logit of sample `lane` (lanes < 32) of the tile whose inputs the wavefront
// has staged in L.x
__device__ __forceinline__ float tile_logit(const PredictLds &S, PredictLds::Wave &L, float b3, int lane)
{
    for (int nh = 0; nh < 2; ++nh) {
        f32x16 acc = {};
        acc = tile_mma_rows(L.x, XS, S.w1t + nh * 32 * XS, XS, 16, acc, lane);
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int m = acc_row(j, lane), c = nh * 32 + acc_col(lane);
            const float h = fmaxf(acc[j] + S.b1[c], 0.0f);
            const uint16_t hi = f2bf(h);
            L.h1[m * PS + c] = hi;
            L.h1lo[m * PS + c] = f2bf(h - bf2f(hi));
        }
    }
    wave_sync_lds();
    // layer 2 and each lane's share of layer 3: sum over its two columns
    float part[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) part[j] = 0.0f;
    for (int nh = 0; nh < 2; ++nh) {
        f32x16 acc = {};
        acc = tile_mma_rows(L.h1, PS, S.w2t + nh * 32 * PS, PS, 64, acc, lane);
        acc = tile_mma_rows(L.h1lo, PS, S.w2t + nh * 32 * PS, PS, 64, acc, lane);
        const int c = nh * 32 + acc_col(lane);
#pragma unroll
        for (int j = 0; j < 16; ++j) part[j] += fmaxf(acc[j] + S.b2[c], 0.0f) * S.w3[c];
    }
    wave_sync_lds();
    // the 32 partial sums of each sample, through LDS (h1 is free now)
    float *zb = reinterpret_cast<float *>(L.h1);   // [32 samples][32 lanes]
#pragma unroll
    for (int j = 0; j < 16; ++j) zb[acc_row(j, lane) * 32 + acc_col(lane)] = part[j];
    wave_sync_lds();
    float z = b3;
    if (lane < 32)
        for (int q = 0; q < 32; ++q) z += zb[lane * 32 + ((q + lane) & 31)];
    wave_sync_lds();   // the next tile overwrites the LDS
    return z;
}

__global__ __launch_bounds__(256) void k_mlp_predict(const float *__restrict__ feats, int64_t n,
                                                     const uint16_t *__restrict__ W1b, const uint16_t *__restrict__ W2b,
                                                     const float *__restrict__ P, float *__restrict__ logits)
{
    __shared__ PredictLds S;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    stage_weights(S, W1b, W2b, P);
    const float b3 = P[OB3];
    __syncthreads();
    PredictLds::Wave &L = S.w[wave];
    const int64_t ntiles = (n + 31) / 32, nwaves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += nwaves) {
        const int64_t s0 = tile * 32;
        for (int e = lane; e < 32 * 16; e += 64) {
            const int m = e >> 4, k = e & 15;
            const int64_t s = s0 + m;
            L.x[m * XS + k] = (k < 12 && s < n) ? f2bf(feats[s * 12 + k]) : (uint16_t)0;
        }
        wave_sync_lds();
        const float z = tile_logit(S, L, b3, lane);
        if (lane < 32 && s0 + lane < n) logits[s0 + lane] = z;
    }
}

// The cells of a strip (cells [cb0, cb0 + ncells / (nr1 - 1)) of the grid,
// vertex rows from vb0 in `verts`) that the refinement tests: the network's
// logit above thr, or folded.  Features are formed from the mapped corners
// in the tile that uses them (zero for a cell with a non-finite corner, which
// the test then leaves alone), so nothing per cell goes through memory but
// the flag.
__global__ __launch_bounds__(256) void k_mlp_flag_cells(int64_t nr1, int64_t cb0, int64_t ncells, int64_t vb0,
                                                        const double2 *__restrict__ verts,
                                                        const uint16_t *__restrict__ W1b,
                                                        const uint16_t *__restrict__ W2b, const float *__restrict__ P,
                                                        float thr, int32_t *__restrict__ flag)
{
    __shared__ PredictLds S;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    stage_weights(S, W1b, W2b, P);
    const float b3 = P[OB3];
    __syncthreads();
    PredictLds::Wave &L = S.w[wave];
    const int64_t ntiles = (ncells + 31) / 32, nwaves = (int64_t)gridDim.x * 4;
    for (int64_t tile = (int64_t)blockIdx.x * 4 + wave; tile < ntiles; tile += nwaves) {
        // cell m of the tile, half h of its features on this lane
        const int m = lane & 31, h = lane >> 5;
        const int64_t t = tile * 32 + m;
        float f[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) f[k] = 0.0f;
        if (t < ncells) {
            const int64_t a = t % (nr1 - 1), b = cb0 + t / (nr1 - 1);
            const double2 *r0 = verts + (b - vb0) * nr1, *r1 = r0 + nr1;
            const double2 q[4] = {r0[a], r0[a + 1], r1[a + 1], r1[a]};
            const double u4[4] = {q[0].x, q[1].x, q[2].x, q[3].x}, v4[4] = {q[0].y, q[1].y, q[2].y, q[3].y};
            if (isfinite(u4[0]) && isfinite(u4[1]) && isfinite(u4[2]) && isfinite(u4[3]) && isfinite(v4[0]) &&
                isfinite(v4[1]) && isfinite(v4[2]) && isfinite(v4[3]))
                cell_features_half_f32(u4, v4, h, f);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) L.x[m * XS + 4 * h + k] = f2bf(f[k]);
        L.x[m * XS + 8 + 2 * h] = f2bf(f[4]);
        L.x[m * XS + 9 + 2 * h] = f2bf(f[5]);
        L.x[m * XS + 12 + 2 * h] = 0;
        L.x[m * XS + 13 + 2 * h] = 0;
        wave_sync_lds();
        // folded: the four ear signs (0 or +-1, exact in bf16) of the staged row
        bool fold = false;
        if (lane < 32) {
            const uint16_t *e = L.x + m * XS + 8;
            fold = !(e[0] == e[1] && e[1] == e[2] && e[2] == e[3]);
        }
        const float z = tile_logit(S, L, b3, lane);
        if (lane < 32 && t < ncells) flag[t] = (z > thr || fold) ? 1 : 0;
    }
}

__device__ inline float softplus(float x) { return x > 0.0f ? x + log1pf(expf(-x)) : log1pf(expf(x)); }

// forward and backward of samples idx[s] (s in [0, n)); each wavefront (32
// samples) writes its whole gradient (FP32) and its part of the loss (at
// [NP]; the loss is divided by `norm`, the batch size) to its own row
// part[w * (NP + 1) ..], w = 4 blockIdx.x + wave, with no atomics: k_grad_sum
// adds the rows in a fixed order, so a batch's gradient is the same bits on
// every run
__global__ __launch_bounds__(256) void k_mlp_train(const float *__restrict__ feats_all, const uint8_t *__restrict__ y_all,
                                                   const int64_t *__restrict__ idx, int64_t n,
                                                   const uint16_t *__restrict__ W1b,
                                                   const uint16_t *__restrict__ W2b, const float *__restrict__ P,
                                                   float pos_weight, float norm, float *__restrict__ part,
                                                   float *__restrict__ xbuf)
{
    __shared__ WaveLds lds[4];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    WaveLds &L = lds[wave];
    const int64_t s0 = (int64_t)blockIdx.x * MB + wave * 32;
    float *g = part + ((int64_t)blockIdx.x * 4 + wave) * (NP + 1);
    // gather this wavefront's samples into a contiguous staging area
    float *xs = xbuf + ((int64_t)blockIdx.x * MB + wave * 32) * 12;
    for (int e = lane; e < 32 * 12; e += 64) {
        const int64_t s = s0 + e / 12;
        xs[e] = s < n ? feats_all[idx[s] * 12 + e % 12] : 0.0f;
    }
    __threadfence_block();
    __syncthreads();
    forward(xbuf + (int64_t)blockIdx.x * MB * 12, wave * 32, MB, W1b, W2b, P, L, lane);
    // loss and dL/dz
    {
        float l = 0.0f;
        if (lane < 32) {
            const int64_t s = s0 + lane;
            float dz = 0.0f;
            if (s < n) {
                const float z = L.z[lane], y = (float)y_all[idx[s]];
                const float sg = 1.0f / (1.0f + expf(-z));
                l = pos_weight * y * softplus(-z) + (1.0f - y) * softplus(z);
                dz = (pos_weight * y * (sg - 1.0f) + (1.0f - y) * sg) / norm;
            }
            L.dz[lane] = dz;
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) l += __shfl_xor(l, o, 64);
        if (lane == 0) g[NP] = l / norm;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 3: dW3, db3; gradient at layer-2 pre-activations
    {
        const int c = lane;   // unit 0..63
        const float w3 = bf2f(f2bf(P[OW3 + c]));
        float gw = 0.0f, gb = 0.0f;
        for (int m = 0; m < 32; ++m) {
            const float h = L.h2[m * 64 + c], dz = L.dz[m];
            gw += dz * h;
            const float d = h > 0.0f ? dz * w3 : 0.0f;
            gb += d;
            L.d2[m * 64 + c] = f2bf(d);
        }
        g[OW3 + c] = gw;
        g[OB2 + c] = gb;
        if (lane == 0) {
            float s = 0.0f;
            for (int m = 0; m < 32; ++m) s += L.dz[m];
            g[OB3] = s;
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW2 (64 x 64) = h1^T d2: A(i, m) = h1[m][i], B(m, j) = d2[m][j]
    for (int ih = 0; ih < 2; ++ih)
        for (int jh = 0; jh < 2; ++jh) {
            f32x16 acc = {};
            acc = tile_mma(L.h1 + ih * 32, 1, 64, L.d2 + jh * 32, 64, 1, 32, acc, lane);
            acc = tile_mma(L.h1lo + ih * 32, 1, 64, L.d2 + jh * 32, 64, 1, 32, acc, lane);
#pragma unroll
            for (int j = 0; j < 16; ++j) g[OW2 + (ih * 32 + acc_row(j, lane)) * 64 + jh * 32 + acc_col(lane)] = acc[j];
        }
    // gradient at layer-1 pre-activations: (d2 W2^T) masked; A(m, j) = d2[m][j], B(j, i) = W2[i][j]
    for (int ih = 0; ih < 2; ++ih) {
        f32x16 acc = {};
        acc = tile_mma(L.d2, 64, 1, W2b + ih * 32 * 64, 1, 64, 64, acc, lane);
        float b1 = 0.0f;   // db1 of unit ih * 32 + acc_col(lane): this lane's rows, then the other half's
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int m = acc_row(j, lane), c = ih * 32 + acc_col(lane);
            const float d = L.h1[m * 64 + c] != 0 ? acc[j] : 0.0f;   // relu'(pre) = [h1 > 0]
            L.d1[m * 64 + c] = f2bf(d);
            b1 += d;
        }
        b1 += __shfl_xor(b1, 32, 64);
        if (lane < 32) g[OB1 + ih * 32 + lane] = b1;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // dW1 (16 x 64, rows 12.. zero) = x^T d1: A(k, m) = x[m][k] (rows >= 16 read as zero via x's padding)
    for (int jh = 0; jh < 2; ++jh) {
        f32x16 acc = {};
        {
            const int r = lane & 31, h = (lane >> 5) * 4;
            for (int k0 = 0; k0 < 32; k0 += 8) {
                bf16x4 av, bv;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    av[t] = r < 16 ? (short)L.x[(k0 + h + t) * 16 + r] : (short)0;
                    bv[t] = (short)L.d1[(k0 + h + t) * 64 + jh * 32 + r];
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x8bf16_1k(av, bv, acc, 0, 0, 0);
            }
        }
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            const int k = acc_row(j, lane);
            if (k < 12) g[OW1 + k * 64 + jh * 32 + acc_col(lane)] = acc[j];
        }
    }
}

// grad[t] += the sum over the rows w = 0 .. nrows - 1 of part[w * (NP + 1) + t],
// in a fixed order: a workgroup takes 32 parameters; its thread (g, p) sums
// the rows g, g + GS_GROUPS, ... of parameter p in order, and the GS_GROUPS
// partial sums are then added in the order g = 0, 1, ...
constexpr int GS_GROUPS = 8;
__global__ __launch_bounds__(32 * GS_GROUPS) void k_grad_sum(const float *__restrict__ part, int64_t nrows,
                                                             float *__restrict__ grad)
{
    __shared__ float ps[GS_GROUPS][32];
    const int p = threadIdx.x & 31, g = threadIdx.x >> 5;
    const int t = blockIdx.x * 32 + p;
    float s = 0.0f;
    if (t <= NP)
        for (int64_t w = g; w < nrows; w += GS_GROUPS) s += part[w * (NP + 1) + t];
    ps[g][p] = s;
    __syncthreads();
    if (g == 0 && t <= NP) {
        float a = 0.0f;
#pragma unroll
        for (int k = 0; k < GS_GROUPS; ++k) a += ps[k][p];
        grad[t] += a;
    }
}

// bf16 copies of the weights in the layouts the kernels read
__global__ void k_mlp_pack(const float *__restrict__ P, uint16_t *__restrict__ W1b, uint16_t *__restrict__ W2b)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < 16 * 64) W1b[t] = t < 12 * 64 ? f2bf(P[OW1 + t]) : (uint16_t)0;
    if (t < 64 * 64) W2b[t] = f2bf(P[OW2 + t]);
}

// Adam step (bias-corrected) on the FP32 master weights; clears the gradient.
// The step number is read from the device (steps taken + 1), so a captured
// sequence of steps replays with the right corrections.
__global__ void k_adam(float *__restrict__ P, float *__restrict__ M, float *__restrict__ V, float *__restrict__ grad,
                       float lr, float b1, float b2, float eps, const int64_t *__restrict__ tstep)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= NP) return;
    const float s = (float)(tstep[0] + 1);
    const float c1 = 1.0f - powf(b1, s), c2 = 1.0f - powf(b2, s);
    const float gv = grad[t];
    const float m = b1 * M[t] + (1.0f - b1) * gv, v = b2 * V[t] + (1.0f - b2) * gv * gv;
    M[t] = m;
    V[t] = v;
    P[t] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
    grad[t] = 0.0f;
}

// after a step: counts it, adds the batch's loss (the mean over its nb rows,
// in G[NP]) times nb to the epoch's sum, and clears it
__global__ void k_step_end(float *__restrict__ G, int64_t *__restrict__ tstep, double *__restrict__ lacc, float nb)
{
    if (threadIdx.x == 0) {
        *lacc += (double)G[NP] * (double)nb;
        G[NP] = 0.0f;
        *tstep += 1;
    }
}

__global__ void k_step_reset(int64_t *__restrict__ tstep, double *__restrict__ lacc, int steps)
{
    if (threadIdx.x == 0) {
        if (steps) *tstep = 0;
        *lacc = 0.0;
    }
}

__global__ void k_zero_f32(float *p, int64_t n)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) p[t] = 0.0f;
}

}  // namespace

// host launchers (device pointers throughout)
void mlp_pack(const float *P, uint16_t *W1b, uint16_t *W2b, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_pack, dim3(16), dim3(256), 0, st, P, W1b, W2b);
}

// a grid the device holds at once (three workgroups per CU at this LDS
// size), each wavefront looping over tiles of 32 samples
static unsigned predict_grid(int64_t n)
{
    const int64_t tiles = (n + 31) / 32;
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((tiles + 3) / 4, 256 * 3 * 4));
}

void mlp_flag_cells(int64_t nr1, int64_t cb0, int64_t ncells, int64_t vb0, const double2 *verts, const uint16_t *W1b,
                    const uint16_t *W2b, const float *P, float thr, int32_t *flag, hipStream_t st)
{
    if (ncells > 0)
        hipLaunchKernelGGL(k_mlp_flag_cells, dim3(predict_grid(ncells)), dim3(256), 0, st, nr1, cb0, ncells, vb0, verts,
                           W1b, W2b, P, thr, flag);
}

void mlp_predict(const float *feats, int64_t n, const uint16_t *W1b, const uint16_t *W2b, const float *P,
                 float *logits, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_mlp_predict, dim3(predict_grid(n)), dim3(256), 0, st, feats, n, W1b, W2b, P, logits);
}

int64_t mlp_part_rows(int64_t n) { return (n + MB - 1) / MB * 4; }

void mlp_train_batch(const float *feats, const uint8_t *y, const int64_t *idx, int64_t n, const uint16_t *W1b,
                     const uint16_t *W2b, const float *P, float pos_weight, float norm, float *grad, float *part,
                     float *xbuf, hipStream_t st)
{
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_train, dim3((unsigned)((n + MB - 1) / MB)), dim3(256), 0, st, feats, y, idx, n, W1b, W2b,
                       P, pos_weight, norm, part, xbuf);
    hipLaunchKernelGGL(k_grad_sum, dim3((NP + 1 + 31) / 32), dim3(32 * GS_GROUPS), 0, st, part, mlp_part_rows(n), grad);
}

void mlp_adam(float *P, float *M, float *V, float *grad, float lr, const int64_t *tstep, hipStream_t st)
{
    hipLaunchKernelGGL(k_adam, dim3((NP + 255) / 256), dim3(256), 0, st, P, M, V, grad, lr, 0.9f, 0.999f, 1e-8f, tstep);
}

void mlp_step_end(float *G, int64_t *tstep, double *lacc, float nb, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_end, dim3(1), dim3(64), 0, st, G, tstep, lacc, nb);
}

void mlp_step_reset(int64_t *tstep, double *lacc, bool steps, hipStream_t st)
{
    hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(64), 0, st, tstep, lacc, steps ? 1 : 0);
}

void mlp_zero(float *p, int64_t n, hipStream_t st)
{
    if (n > 0) hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
}

}  // namespace mlm
