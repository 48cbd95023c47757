// FMM passes (sec. 3.3, app. C.2): P2M at the leaves, M2M upward, then per
// level L2L from the parent + M2L from same-level interaction nodes + P2L from
// the stars of interaction squares that lie inside coarser leaves.
//
// Coefficients are normalised to each node's half-length (app. C.2), which
// makes every translation a fixed linear operator: M2M and L2L depend only on
// the child's quadrant, M2L only on the offset between the two squares (one
// of 40 in a 7x7 stencil).  The operators are tabulated once on the host in
// extended precision.
#include <cmath>
#include <complex>
#include <vector>

#include "dev.hpp"

namespace mlm {

int64_t scan_total_public(mlm_lens *lens, const int32_t *in, int32_t *out, int64_t n, hipStream_t st);

namespace {

constexpr int BLK = 256;
inline unsigned nblocks(int64_t n, int b = BLK) { return (unsigned)((n + b - 1) / b); }

using cld = std::complex<long double>;

long double binom_ld(int n, int k)
{
    if (k < 0 || k > n) return 0.0L;
    long double r = 1.0L;
    for (int t = 1; t <= k; ++t) r = r * (long double)(n - k + t) / (long double)t;
    return r;
}

cld ipow(cld z, int n)
{
    cld r(1.0L, 0.0L);
    for (int t = 0; t < n; ++t) r *= z;
    return r;
}

// M2M, child quadrant (qi, qj): z0 = child centre - parent centre in child
// half-lengths = (2qi-1) + i(2qj-1);  b_l = z0^l [-a_0/l + sum_{k=1}^{l} a_k z0^-k C(l-1,k-1)] / 2^l
void table_m2m(int p, std::vector<double2> &out)
{
    int P1 = p + 1;
    out.assign(4 * P1 * P1, make_double2(0, 0));
    for (int quad = 0; quad < 4; ++quad) {
        cld z0((long double)(2 * (quad & 1) - 1), (long double)(2 * (quad >> 1) - 1));
        for (int l = 0; l <= p; ++l)
            for (int k = 0; k <= p; ++k) {
                cld v(0.0L, 0.0L);
                if (l == 0) {
                    if (k == 0) v = 1.0L;
                } else if (k == 0) {
                    v = -ipow(z0, l) / (long double)l;
                } else if (k <= l) {
                    v = ipow(z0, l - k) * binom_ld(l - 1, k - 1);
                }
                v /= std::ldexp(1.0L, l);
                out[(quad * P1 + l) * P1 + k] = make_double2((double)v.real(), (double)v.imag());
            }
    }
}

// M2L, offset (dx, dy) in squares: z0 = 2(dx + i dy) in half-lengths;
// c_l = z0^-l [-b_0/l + sum_{k=1}^{p} b_k (-z0)^-k C(l+k-1,k-1)], l >= 1
void table_m2l(int p, std::vector<double2> &out)
{
    int P1 = p + 1;
    out.assign(49 * P1 * P1, make_double2(0, 0));
    for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
            if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
            int off = (dx + 3) + 7 * (dy + 3);
            cld z0(2.0L * dx, 2.0L * dy);
            cld zi = 1.0L / z0, nzi = -1.0L / z0;
            for (int l = 1; l <= p; ++l) {
                cld zl = ipow(zi, l);
                for (int k = 0; k <= p; ++k) {
                    cld v = (k == 0) ? -zl / (long double)l : zl * ipow(nzi, k) * binom_ld(l + k - 1, k - 1);
                    out[(off * P1 + l) * P1 + k] = make_double2((double)v.real(), (double)v.imag());
                }
            }
        }
}

// L2L, child quadrant (qi, qj): delta = child centre - parent centre in parent
// half-lengths = ((2qi-1) + i(2qj-1)) / 2;  d_l = sum_{k>=l} c_k C(k,l) delta^(k-l) / 2^l
void table_l2l(int p, std::vector<double2> &out)
{
    int P1 = p + 1;
    out.assign(4 * P1 * P1, make_double2(0, 0));
    for (int quad = 0; quad < 4; ++quad) {
        cld delta(0.5L * (2 * (quad & 1) - 1), 0.5L * (2 * (quad >> 1) - 1));
        for (int l = 0; l <= p; ++l)
            for (int k = l; k <= p; ++k) {
                cld v = ipow(delta, k - l) * binom_ld(k, l) / std::ldexp(1.0L, l);
                out[(quad * P1 + l) * P1 + k] = make_double2((double)v.real(), (double)v.imag());
            }
    }
}

__device__ inline void node_geom(uint64_t code, int lev, double L0, double &cx, double &cy, double &L,
                                 double &invL)
{
    uint32_t i = compact_bits(code), j = compact_bits(code >> 1);
    L = ldexp(L0, -lev);
    invL = 1.0 / L;   // exact: L is a power of two
    cx = -L0 + (double)(2 * (int64_t)i + 1) * L;
    cy = -L0 + (double)(2 * (int64_t)j + 1) * L;
}

// upward pass of one level: P2M at leaves, M2M from the four children
// elsewhere.  R is the arithmetic type of the coefficients; star offsets from
// the node centre are always formed in FP64.
template <class R>
__global__ void k_upward(int64_t lo, int64_t hi, int lev, int p, double L0, const uint64_t *__restrict__ code,
                         const int32_t *__restrict__ leaf, const int32_t *__restrict__ slo,
                         const int32_t *__restrict__ shi, const int32_t *__restrict__ child0,
                         const double *__restrict__ sx, const double *__restrict__ sy,
                         const double *__restrict__ sm, const typename Cx<R>::c2 *__restrict__ m2m,
                         typename Cx<R>::c2 *__restrict__ mult)
{
    using C2 = typename Cx<R>::c2;
    const int P1 = p + 1;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t q = lo + t / P1;
    int k = (int)(t % P1);
    if (q >= hi) return;
    C2 acc = Cx<R>::make(0, 0);
    if (leaf[q]) {
        double cx, cy, L, invL;
        node_geom(code[q], lev, L0, cx, cy, L, invL);
        // a_0 = sum m_i;  a_k = -(1/k) sum m_i zeta_i^k
        for (int32_t s = slo[q]; s < shi[q]; ++s) {
            const R m = (R)sm[s];
            if (k == 0) {
                acc.x += m;
            } else {
                C2 z = Cx<R>::make((R)((sx[s] - cx) * invL), (R)((sy[s] - cy) * invL));
                C2 zk = cpowi(z, k);
                acc.x -= m * zk.x;
                acc.y -= m * zk.y;
            }
        }
        if (k > 0) acc = cscale(acc, (R)1 / (R)k);
    } else {
        int32_t c0 = child0[q];
        for (int quad = 0; quad < 4; ++quad) {
            const C2 *op = m2m + (quad * P1 + k) * P1;
            const C2 *a = mult + (int64_t)(c0 + quad) * P1;
            for (int kk = 0; kk <= k; ++kk) {
                C2 o = op[kk], v = a[kk];
                acc.x += o.x * v.x - o.y * v.y;
                acc.y += o.x * v.y + o.y * v.x;
            }
        }
    }
    mult[q * P1 + k] = acc;
}

// downward pass of one level (>= 2): Taylor coefficient l of each node
template <class R>
__global__ void k_downward(int64_t lo, int64_t hi, int lev, int p, double L0, const uint64_t *__restrict__ code,
                           const int32_t *__restrict__ parent, const IEntry *__restrict__ ilist,
                           const double *__restrict__ sx, const double *__restrict__ sy,
                           const double *__restrict__ sm, const typename Cx<R>::c2 *__restrict__ m2l,
                           const typename Cx<R>::c2 *__restrict__ l2l, const typename Cx<R>::c2 *__restrict__ mult,
                           typename Cx<R>::c2 *__restrict__ local)
{
    using C2 = typename Cx<R>::c2;
    const int P1 = p + 1;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t q = lo + t / P1;
    int l = (int)(t % P1);
    if (q >= hi) return;
    if (l == 0) {
        local[q * P1] = Cx<R>::make(0, 0);   // c_0 only shifts the potential
        return;
    }
    uint64_t c = code[q];
    C2 acc = Cx<R>::make(0, 0);
    // L2L from the parent (levels 0 and 1 have no far field)
    if (lev >= 3) {
        int quad = (int)((c & 1ull) | (((c >> 1) & 1ull) << 1));
        const C2 *op = l2l + (quad * P1 + l) * P1;
        const C2 *cp = local + (int64_t)parent[q] * P1;
        for (int k = l; k <= p; ++k) {
            C2 o = op[k], v = cp[k];
            acc.x += o.x * v.x - o.y * v.y;
            acc.y += o.x * v.y + o.y * v.x;
        }
    }
    double cx, cy, L, invL;
    node_geom(c, lev, L0, cx, cy, L, invL);
    const IEntry *list = ilist + q * NLIST;
    for (int e = 0; e < NLIST; ++e) {
        IEntry en = list[e];
        if (en.src >= 0) {
            // M2L
            const C2 *op = m2l + (en.off * P1 + l) * P1;
            const C2 *b = mult + (int64_t)en.src * P1;
            for (int k = 0; k <= p; ++k) {
                C2 o = op[k], v = b[k];
                acc.x += o.x * v.x - o.y * v.y;
                acc.y += o.x * v.y + o.y * v.x;
            }
        } else if (en.src == -1) {
            // P2L: c_l += -m_i / (l zeta_i^l)
            for (int32_t s = en.slo; s < en.shi; ++s) {
                C2 z = Cx<R>::make((R)((sx[s] - cx) * invL), (R)((sy[s] - cy) * invL));
                C2 w = cpowi(cinv(z), l);
                R f = -(R)sm[s] / (R)l;
                acc.x += f * w.x;
                acc.y += f * w.y;
            }
        }
    }
    local[q * P1 + l] = acc;
}

template <class C2>
__global__ void k_zero2(C2 *a, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = C2{0, 0};
}

// per-leaf data for the ray kernels: geometry, derivative of the Taylor
// series (in R) and the stars of the leaf's 3x3 block relative to its centre
// (FP64 in both modes: a ray's offset from a star is formed from them)
template <class R>
__global__ void k_leaf_tables(int64_t nleaves, int p, double L0, const int32_t *__restrict__ leaf_node,
                              const uint64_t *__restrict__ code, const int32_t *__restrict__ level,
                              const int32_t *__restrict__ block, const int32_t *__restrict__ near_offs,
                              const uint64_t *__restrict__ keys, int32_t n, const double *__restrict__ sx,
                              const double *__restrict__ sy, const double *__restrict__ sm,
                              const typename Cx<R>::c2 *__restrict__ local, LeafInfo *__restrict__ info,
                              typename Cx<R>::c2 *__restrict__ deriv, double4 *__restrict__ near)
{
    int64_t lf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lf >= nleaves) return;
    int32_t q = leaf_node[lf];
    int lev = level[q];
    uint64_t c = code[q];
    double cx, cy, L, invL;
    node_geom(c, lev, L0, cx, cy, L, invL);
    LeafInfo li;
    li.cx = cx;
    li.cy = cy;
    li.L = L;
    li.invL = invL;
    li.near_off = near_offs[lf];
    li.near_cnt = block[q];
    li.a_lo = li.na = li.b_lo = li.nb = li.ntx = li.pad = 0;
    info[lf] = li;
    const int P1 = p + 1;
    // d psi / dz = (1/L) sum_{l>=1} l c_l zeta^(l-1)
    for (int l = 0; l < p; ++l) deriv[lf * p + l] = cscale(local[(int64_t)q * P1 + l + 1], (R)((double)(l + 1) * invL));
    uint32_t i = compact_bits(c), j = compact_bits(c >> 1);
    int64_t side = 1ll << lev;
    int sh = 2 * (KEY_BITS - lev);
    int32_t o = li.near_off;
    for (int dj = -1; dj <= 1; ++dj)
        for (int di = -1; di <= 1; ++di) {
            int64_t a = (int64_t)i + di, b = (int64_t)j + dj;
            if (a < 0 || b < 0 || a >= side || b >= side) continue;
            uint64_t cc = morton2((uint32_t)a, (uint32_t)b);
            int32_t s0 = lower_bound_u64(keys, n, cc << sh), s1 = lower_bound_u64(keys, n, (cc + 1) << sh);
            for (int32_t s = s0; s < s1; ++s) near[o++] = make_double4(sx[s] - cx, sy[s] - cy, sm[s], 0.0);
        }
}

__global__ void k_leaf_block(int64_t nleaves, const int32_t *__restrict__ leaf_node,
                             const int32_t *__restrict__ block, int32_t *__restrict__ cnt)
{
    int64_t lf = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lf < nleaves) cnt[lf] = block[leaf_node[lf]];
}

}  // namespace

namespace {

template <class R>
void upload_ops(DevBuf &buf, const std::vector<double2> &h)
{
    using C2 = typename Cx<R>::c2;
    std::vector<C2> c(h.size());
    for (size_t k = 0; k < h.size(); ++k) c[k] = Cx<R>::make((R)h[k].x, (R)h[k].y);
    void *d = buf.reserve(c.size() * sizeof(C2));
    MLM_HIP(hipMemcpy(d, c.data(), c.size() * sizeof(C2), hipMemcpyHostToDevice));
}

template <class R>
void run_fmm_t(mlm_lens *lens, Tree &T, int p, hipStream_t st, typename Cx<R>::c2 *&mult,
               typename Cx<R>::c2 *&local)
{
    using C2 = typename Cx<R>::c2;
    Workspace &ws = lens->ws;
    const int P1 = p + 1;
    const int key = 2 * p + (sizeof(R) == 4 ? 1 : 0);
    if (ws.ops_p != key) {
        std::vector<double2> h;
        table_m2m(p, h);
        upload_ops<R>(ws.ops_m2m, h);
        table_m2l(p, h);
        upload_ops<R>(ws.ops_m2l, h);
        table_l2l(p, h);
        upload_ops<R>(ws.ops_l2l, h);
        ws.ops_p = key;
    }
    mult = static_cast<C2 *>(ws.mult.reserve((size_t)T.nnodes * P1 * sizeof(C2)));
    local = static_cast<C2 *>(ws.local.reserve((size_t)T.nnodes * P1 * sizeof(C2)));
    // upward
    for (int lev = T.nlevels - 1; lev >= 0; --lev) {
        int64_t lo = T.level_lo[lev], hi = T.level_hi[lev], nt = (hi - lo) * P1;
        hipLaunchKernelGGL(k_upward<R>, dim3(nblocks(nt)), dim3(BLK), 0, st, lo, hi, lev, p, T.L0, T.code, T.leaf,
                           T.slo, T.shi, T.child0, T.x, T.y, T.m, ws.ops_m2m.as<C2>(), mult);
    }
    // downward: levels 0, 1 have no far field
    int64_t top = T.nlevels > 2 ? T.level_lo[2] : T.nnodes;
    hipLaunchKernelGGL(k_zero2<C2>, dim3(nblocks(top * P1)), dim3(BLK), 0, st, local, top * P1);
    for (int lev = 2; lev < T.nlevels; ++lev) {
        int64_t lo = T.level_lo[lev], hi = T.level_hi[lev], nt = (hi - lo) * P1;
        hipLaunchKernelGGL(k_downward<R>, dim3(nblocks(nt)), dim3(BLK), 0, st, lo, hi, lev, p, T.L0, T.code,
                           T.parent, T.ilist, T.x, T.y, T.m, ws.ops_m2l.as<C2>(), ws.ops_l2l.as<C2>(), mult, local);
    }
}

}  // namespace

void run_fmm(mlm_lens *lens, Tree &T, int p, hipStream_t st)
{
    if (p < 1 || p > MAX_ORDER) fail(MLM_EINVAL, "expansion order %d outside [1, %d]", p, MAX_ORDER);
    T.p = p;
    if (T.mixed) run_fmm_t<float>(lens, T, p, st, T.mult_f, T.local_f);
    else run_fmm_t<double>(lens, T, p, st, T.mult, T.local);
}

void build_leaf_tables(mlm_lens *lens, Tree &T, hipStream_t st)
{
    Workspace &ws = lens->ws;
    int64_t nl = T.nleaves;
    int32_t *cnt = static_cast<int32_t *>(ws.flags.reserve(nl * 4));
    int32_t *offs = static_cast<int32_t *>(ws.near_offs.reserve(nl * 4));
    hipLaunchKernelGGL(k_leaf_block, dim3(nblocks(nl)), dim3(BLK), 0, st, nl, T.leaf_node, T.block, cnt);
    T.near_total = scan_total_public(lens, cnt, offs, nl, st);
    T.leaves = static_cast<LeafInfo *>(ws.leaves.reserve(nl * sizeof(LeafInfo)));
    const size_t nn = (size_t)(T.near_total > 0 ? T.near_total : 1);
    T.near = static_cast<double4 *>(ws.near.reserve(nn * sizeof(double4)));
    if (T.mixed) {
        T.deriv_f = static_cast<float2 *>(ws.deriv.reserve((size_t)nl * T.p * sizeof(float2)));
        hipLaunchKernelGGL(k_leaf_tables<float>, dim3(nblocks(nl, 64)), dim3(64), 0, st, nl, T.p, T.L0, T.leaf_node,
                           T.code, T.level, T.block, offs, T.keys, (int32_t)T.n, T.x, T.y, T.m, T.local_f,
                           T.leaves, T.deriv_f, T.near);
    } else {
        T.deriv = static_cast<double2 *>(ws.deriv.reserve((size_t)nl * T.p * sizeof(double2)));
        hipLaunchKernelGGL(k_leaf_tables<double>, dim3(nblocks(nl, 64)), dim3(64), 0, st, nl, T.p, T.L0,
                           T.leaf_node, T.code, T.level, T.block, offs, T.keys, (int32_t)T.n, T.x, T.y, T.m, T.local,
                           T.leaves, T.deriv, T.near);
    }
}

}  // namespace mlm
