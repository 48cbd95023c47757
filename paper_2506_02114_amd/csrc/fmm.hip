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

// The M2L operator factorised: with z0 the source-to-target offset (in
// half-lengths) and b' = b_k (-z0)^-k,
//   c_l = z0^-l [ sum_{k>=1} C(l+k-1, k-1) b'_k - b_0 / l ],
// so every offset shares one real matrix P[l-1][k-1] = C(l+k-1, k-1) and
// differs only by the diagonal scalings S[off][k] = (-z0)^-k (sources) and
// T[off][l] = z0^-l (targets).  Tables of 32 entries per offset (p <= 31);
// P is 32 x 32, zero beyond p.
void table_m2l_factors(int p, std::vector<double2> &S, std::vector<double2> &T, std::vector<double> &P)
{
    S.assign(49 * 32, make_double2(0, 0));
    T.assign(49 * 32, make_double2(0, 0));
    P.assign(32 * 32, 0.0);
    for (int dy = -3; dy <= 3; ++dy)
        for (int dx = -3; dx <= 3; ++dx) {
            if (std::abs(dx) <= 1 && std::abs(dy) <= 1) continue;
            int off = (dx + 3) + 7 * (dy + 3);
            cld z0(2.0L * dx, 2.0L * dy);
            for (int k = 0; k <= p; ++k) {
                cld sv = ipow(-1.0L / z0, k), tv = ipow(1.0L / z0, k);
                S[off * 32 + k] = make_double2((double)sv.real(), (double)sv.imag());
                T[off * 32 + k] = make_double2((double)tv.real(), (double)tv.imag());
            }
        }
    for (int l = 1; l <= p; ++l)
        for (int k = 1; k <= p; ++k) P[(l - 1) * 32 + (k - 1)] = (double)binom_ld(l + k - 1, k - 1);
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

// Matrix-core product of the factorised M2L: Y (32 x 64) = P (32 x 32) B
// (32 x 64), as 16 x 16 x 4 FP64 tiles; lane l holds A(l % 16, l / 16) and
// B(l / 16, l % 16); its four results are D(4 i + l / 16, l % 16), i < 4.
// (The coefficient passes run in FP64 in both precision modes.)
typedef double f64x4 __attribute__((ext_vector_type(4)));
__device__ inline f64x4 mma16(double a, double b, f64x4 c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
template <class R> struct V4T;
template <> struct V4T<double> {
    using t = f64x4;
    __device__ static int row(int i, int g4) { return 4 * i + g4; }
};

// The sources of a node go through the matrix cores in groups of GS: a
// group's scaled coefficients fill a 32 x 2 GS block of LDS (row stride BRS,
// one more than its columns so the rows of a column fall in other banks), so
// a node's wavefront needs 9 KB of LDS, not the 17 KB that all 27 sources at
// once would take, and more wavefronts fit a CU.
constexpr int GS = 16;
constexpr int BRS = 2 * GS + 1;
template <class R> struct DownLds {
    R B[32 * BRS];         // a group's scaled source coefficients: row k - 1, columns (2 s, 2 s + 1) =
                           // (re, im) of source s of the group; then, in place, P B
    typename Cx<R>::c2 b0[32];
    int off[32], src[32];
};

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// downward pass of one level (>= 2), one wavefront per node: L2L from the
// parent (lane l: coefficient l), M2L from the same-level interaction nodes
// through the factorised operator (the shared real matrix on the matrix
// cores, the scalings on the vector units), P2L from the stars of
// interaction squares inside coarser leaves
template <class R>
__global__ __launch_bounds__(64) void k_downward(int64_t lo, int64_t hi, int lev, int p, double L0,
                                                  const uint64_t *__restrict__ code, const int32_t *__restrict__ parent,
                                                  const IEntry *__restrict__ ilist, const double *__restrict__ sx,
                                                  const double *__restrict__ sy, const double *__restrict__ sm,
                                                  const typename Cx<R>::c2 *__restrict__ Sf,
                                                  const typename Cx<R>::c2 *__restrict__ Tf, const R *__restrict__ Pm,
                                                  const typename Cx<R>::c2 *__restrict__ l2l,
                                                  const typename Cx<R>::c2 *__restrict__ mult,
                                                  typename Cx<R>::c2 *__restrict__ local)
{
    using C2 = typename Cx<R>::c2;
    using V4 = typename V4T<R>::t;
    __shared__ DownLds<R> L;   // one wavefront per workgroup and node
    const int lane = threadIdx.x;
    const int64_t q = lo + (int64_t)blockIdx.x;
    if (q >= hi) return;
    const int P1 = p + 1;
    const uint64_t c = code[q];
    // the node's M2L sources into slots 0 .. ns-1 (lanes 0..26 hold the entries)
    const IEntry *list = ilist + q * NLIST;
    IEntry en{-2, 0, 0, 0};
    if (lane < NLIST) en = list[lane];
    const uint64_t mask = __ballot(lane < NLIST && en.src >= 0);
    const int ns = __popcll(mask);
    const int slot = __popcll(mask & ((1ull << lane) - 1ull));
    if (lane < NLIST && en.src >= 0) {
        L.off[slot] = en.off;
        L.src[slot] = en.src;
        L.b0[slot] = mult[(int64_t)en.src * P1];
    }
    wave_sync();
    // M2L, coefficient l = lane: sum over the sources of z0^-l (y_l - b_0 / l),
    // y = P B with B the coefficients b_k (-z0)^-k (rows k - 1 = 0 .. p - 1;
    // only the rows the products read: 16 for p <= 16, else 32)
    const int l = lane;
    const R il = l > 0 ? (R)1 / (R)l : (R)0;
    C2 acc = Cx<R>::make(0, 0);
    const int lgr = p <= 16 ? 4 : 5;
    const int mt_n = (p + 15) / 16, kt_n = (p + 3) / 4;
    const int r = lane & 15, g4 = lane >> 4;
    // this lane's operands of P for every product below, loaded once: P is the
    // same for every node and group, and reading it inside the product loop
    // made each matrix-core step wait for a global load
    constexpr int KTMAX = (MAX_ORDER + 4) / 4;
    R pa[KTMAX], pb[KTMAX];
#pragma unroll
    for (int ks = 0; ks < KTMAX; ++ks) {
        pa[ks] = ks < kt_n ? Pm[r * 32 + ks * 4 + g4] : (R)0;
        pb[ks] = ks < kt_n && mt_n > 1 ? Pm[(16 + r) * 32 + ks * 4 + g4] : (R)0;
    }
    for (int g0 = 0; g0 < ns; g0 += GS) {
        const int gn = min(GS, ns - g0);
        const int ncol = ((2 * gn + 15) / 16) * 16;
        for (int e = lane; e < (ncol / 2) << lgr; e += 64) {
            const int k1 = e & ((1 << lgr) - 1), s2 = e >> lgr;   // row k1 = k - 1, source g0 + s2
            R re = 0, im = 0;
            if (s2 < gn && k1 < p) {
                const C2 b = mult[(int64_t)L.src[g0 + s2] * P1 + k1 + 1], f = Sf[L.off[g0 + s2] * 32 + k1 + 1];
                re = b.x * f.x - b.y * f.y;
                im = b.x * f.y + b.y * f.x;
            }
            L.B[k1 * BRS + 2 * s2] = re;
            L.B[k1 * BRS + 2 * s2 + 1] = im;
        }
        wave_sync();
        // Y = P B on the matrix cores, in place: a 16-column block of B is read
        // whole (both 16-row tiles of P) before Y's block overwrites it
        for (int nt = 0; nt < ncol / 16; ++nt) {
            V4 acc0 = {}, acc1 = {};
#pragma unroll
            for (int ks = 0; ks < KTMAX; ++ks) {
                if (ks < kt_n) {
                    const R b = L.B[(ks * 4 + g4) * BRS + nt * 16 + r];
                    acc0 = mma16(pa[ks], b, acc0);
                    if (mt_n > 1) acc1 = mma16(pb[ks], b, acc1);
                }
            }
            wave_sync();
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                L.B[V4T<R>::row(i, g4) * BRS + nt * 16 + r] = acc0[i];
                if (mt_n > 1) L.B[(16 + V4T<R>::row(i, g4)) * BRS + nt * 16 + r] = acc1[i];
            }
        }
        wave_sync();
        if (l >= 1 && l <= p)
            for (int s2 = 0; s2 < gn; ++s2) {
                const C2 t = Tf[L.off[g0 + s2] * 32 + l];
                const R yr = L.B[(l - 1) * BRS + 2 * s2] - L.b0[g0 + s2].x * il;
                const R yi = L.B[(l - 1) * BRS + 2 * s2 + 1] - L.b0[g0 + s2].y * il;
                acc.x += t.x * yr - t.y * yi;
                acc.y += t.x * yi + t.y * yr;
            }
        wave_sync();   // the next group overwrites B
    }
    // P2L from the stars of interaction squares that are not nodes (parts of
    // coarser leaves): c_l += -m / (l zeta^l).  Lanes take the stars, the
    // powers zeta^-l follow by one product per order, and each order's sum
    // over the wavefront lands in lane l.
    double cx, cy, Lh, invL;
    node_geom(c, lev, L0, cx, cy, Lh, invL);
    C2 p2l = Cx<R>::make(0, 0);
    {
        const int cnt = (lane < NLIST && en.src == -1) ? en.shi - en.slo : 0;
        int total;
        const int excl = wave_excl_scan(cnt, lane, total);
        for (int base = 0; base < total; base += 64) {
            const int item = base + lane;
            const int E = wave_find(excl, item);
            const int s = __shfl(en.slo, E, 64) + item - __shfl(excl, E, 64);
            C2 w = Cx<R>::make(0, 0);
            R mq = 0;
            if (item < total) {
                w = cinv(Cx<R>::make((R)((sx[s] - cx) * invL), (R)((sy[s] - cy) * invL)));
                mq = -(R)sm[s];
            }
            C2 t = cscale(w, mq);   // -m zeta^-1
            for (int k = 1; k <= p; ++k) {
                R vx = t.x, vy = t.y;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    vx += __shfl_xor(vx, o, 64);
                    vy += __shfl_xor(vy, o, 64);
                }
                if (lane == k) {
                    p2l.x += vx;
                    p2l.y += vy;
                }
                t = cmul(t, w);
            }
        }
    }
    // coefficient l = lane
    if (l > p) return;
    if (l == 0) {
        local[q * P1] = Cx<R>::make(0, 0);   // c_0 only shifts the potential
        return;
    }
    // L2L from the parent (levels 0 and 1 have no far field)
    if (lev >= 3) {
        const int quad = (int)((c & 1ull) | (((c >> 1) & 1ull) << 1));
        const C2 *op = l2l + (quad * P1 + l) * P1;
        const C2 *cp = local + (int64_t)parent[q] * P1;
        for (int k = l; k <= p; ++k) {
            const C2 o = op[k], v = cp[k];
            acc.x += o.x * v.x - o.y * v.y;
            acc.y += o.x * v.y + o.y * v.x;
        }
    }
    acc.x += p2l.x * il;
    acc.y += p2l.y * il;
    local[q * P1 + l] = acc;
}

template <class C2>
__global__ void k_zero2(C2 *a, int64_t n)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) a[t] = C2{0, 0};
}

// per-leaf data for the ray kernels: geometry, the far field at the centre
// (FP64), derivative of the Taylor series (rounded to R) and the stars of the
// leaf's 3x3 block relative to its centre (FP64 in both modes: a ray's offset
// from a star is formed from them)
template <class R>
__global__ void k_leaf_tables(int64_t nleaves, int p, double L0, const int32_t *__restrict__ leaf_node,
                              const uint64_t *__restrict__ code, const int32_t *__restrict__ level,
                              const int32_t *__restrict__ block, const int32_t *__restrict__ near_offs,
                              const uint64_t *__restrict__ keys, int32_t n, const double *__restrict__ sx,
                              const double *__restrict__ sy, const double *__restrict__ sm,
                              const double2 *__restrict__ local, LeafInfo *__restrict__ info,
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
    const int P1 = p + 1;
    // d psi / dz = (1/L) sum_{l>=1} l c_l zeta^(l-1); its value at the centre
    // (l = 1) is the whole field of the far stars, kept in FP64
    const double2 d0 = cscale(local[(int64_t)q * P1 + 1], invL);
    li.f0x = d0.x;
    li.f0y = d0.y;
    info[lf] = li;
    for (int l = 0; l < p; ++l) {
        const double2 d = cscale(local[(int64_t)q * P1 + l + 1], (double)(l + 1) * invL);
        deriv[lf * p + l] = Cx<R>::make((R)d.x, (R)d.y);
    }
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
    const int key = p;
    if (ws.ops_p != key) {
        std::vector<double2> h, S, T;
        std::vector<double> Pm;
        table_m2m(p, h);
        upload_ops<R>(ws.ops_m2m, h);
        table_l2l(p, h);
        upload_ops<R>(ws.ops_l2l, h);
        table_m2l_factors(p, S, T, Pm);
        // one buffer: S (49 x 32 complex), T (49 x 32 complex), P (32 x 32 real)
        std::vector<C2> st(2 * 49 * 32);
        for (size_t k = 0; k < S.size(); ++k) {
            st[k] = Cx<R>::make((R)S[k].x, (R)S[k].y);
            st[S.size() + k] = Cx<R>::make((R)T[k].x, (R)T[k].y);
        }
        std::vector<R> pr(Pm.size());
        for (size_t k = 0; k < Pm.size(); ++k) pr[k] = (R)Pm[k];
        char *d = static_cast<char *>(ws.ops_m2l.reserve(st.size() * sizeof(C2) + pr.size() * sizeof(R)));
        MLM_HIP(hipMemcpy(d, st.data(), st.size() * sizeof(C2), hipMemcpyHostToDevice));
        MLM_HIP(hipMemcpy(d + st.size() * sizeof(C2), pr.data(), pr.size() * sizeof(R), hipMemcpyHostToDevice));
        ws.ops_p = key;
    }
    const C2 *Sf = ws.ops_m2l.as<C2>(), *Tf = Sf + 49 * 32;
    const R *Pm = reinterpret_cast<const R *>(Sf + 2 * 49 * 32);
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
        const int64_t lo = T.level_lo[lev], hi = T.level_hi[lev];
        hipLaunchKernelGGL(k_downward<R>, dim3((unsigned)(hi - lo)), dim3(64), 0, st, lo, hi, lev, p, T.L0,
                           T.code, T.parent, T.ilist, T.x, T.y, T.m, Sf, Tf, Pm, ws.ops_l2l.as<C2>(), mult, local);
    }
}

}  // namespace

void run_fmm(mlm_lens *lens, Tree &T, int p, hipStream_t st)
{
    if (p < 1 || p > MAX_ORDER) fail(MLM_EINVAL, "expansion order %d outside [1, %d]", p, MAX_ORDER);
    T.p = p;
    // FP64 in both modes: the low-order Taylor coefficients carry the field of
    // the whole star disc (about kappa_* |z|), far above what FP32 translation
    // chains could hold to a fraction of a pixel
    run_fmm_t<double>(lens, T, p, st, T.mult, T.local);
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
                           T.code, T.level, T.block, offs, T.keys, (int32_t)T.n, T.x, T.y, T.m, T.local,
                           T.leaves, T.deriv_f, T.near);
    } else {
        T.deriv = static_cast<double2 *>(ws.deriv.reserve((size_t)nl * T.p * sizeof(double2)));
        hipLaunchKernelGGL(k_leaf_tables<double>, dim3(nblocks(nl, 64)), dim3(64), 0, st, nl, T.p, T.L0,
                           T.leaf_node, T.code, T.level, T.block, offs, T.keys, (int32_t)T.n, T.x, T.y, T.m, T.local,
                           T.leaves, T.deriv, T.near);
    }
}

}  // namespace mlm
