// Closed-form pixel areas of a triangle by pixel columns (the apportioning of
// sec. 3.2: a mapped triangle's share of a source pixel is their overlap over
// the triangle's area), shared by the IPM's cell pass and the cell
// refinement.  Inside a strip of pixel columns the area of a triangle below
// the line v = r is H(r) = sum_e du_e I(r - va_e, r - vb_e) over its edges
// clipped to the strip (du_e the clipped edge's extent along u, I the
// integral over [0, 1] of a clamped linear function), signed like the
// triangle; the area of the pixel between rows r and r + 1 is
// H(r + 1) - H(r).  Templated on the arithmetic type (FP64, or FP32 for the
// mixed mode's well-conditioned triangles).
#pragma once

#include "dev.hpp"

namespace mlm {

template <class R> struct Pt {
    R u, v;
};
using P2 = Pt<double>;

// a / b for slopes and weights: the hardware reciprocal estimate, two Newton
// steps and a corrected product (within an ulp or two of the rounded
// quotient, for finite normal b); FP32: the reciprocal times a
__device__ inline double fdiv(double a, double b)
{
    double y = __builtin_amdgcn_rcp(b);
    y = fma(fma(-b, y, 1.0), y, y);
    y = fma(fma(-b, y, 1.0), y, y);
    const double r = a * y;
    return fma(fma(-b, r, a), y, r);
}
__device__ inline float fdiv(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }

// edge slopes of a triangle: sv = dv/du (for clips along u), su = du/dv (along v);
// a slope that overflows (an edge whose extent along one axis is below the
// other's over the largest double) is taken as 0, as for an edge exactly
// along that axis, so that both stay finite
template <class R>
__device__ inline void tri_slopes(const Pt<R> (&T)[3], R (&sv)[3], R (&su)[3])
{
    const R big = sizeof(R) == 4 ? R(3e38f) : R(1e308);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R du = T[(k + 1) % 3].u - T[k].u, dv = T[(k + 1) % 3].v - T[k].v;
        const R a = du != R(0) ? fdiv(dv, du) : R(0), b = dv != R(0) ? fdiv(du, dv) : R(0);
        sv[k] = fabs(a) <= big ? a : R(0);
        su[k] = fabs(b) <= big ? b : R(0);
    }
}

// A strip of pixel columns lo <= u <= hi, divide-free: for an edge with slope
// sv = dv/du clipped to the strip, |b - a| = |sv| |d|, so where the clamped
// function changes sign d I = sign(d) m^2 / (2 |sv|) = m^2 c with
// c = sign(d) |du/dv| / 2 fixed per edge.
template <class R> struct ColSeg {
    R lo, hi;           // v range of the clipped edge
    R mid;              // (lo + hi) / 2
    R d;                // du of the clipped edge
    R c;                // sign(du) |du/dv| / 2 (0 if du = 0)
    bool any;           // the edge crosses the column with some extent
};
template <class R> struct ColSegs {
    ColSeg<R> e0, e1, e2;
};

// edge P->Q clipped to the column lo <= u <= hi, without branches: its ends
// are clamped into the column (an end inside keeps its exact v: for P the
// clip's own product is then an exact zero, the slope being finite); an edge
// that misses the column clamps to a single point, where d = 0 and lo = hi
// make its term below zero at every r
template <class R>
__device__ inline ColSeg<R> col_seg(Pt<R> P, Pt<R> Q, R lo, R hi, R sv, R su)
{
    ColSeg<R> s;
    const R eu = fmin(fmax(P.u, lo), hi), xu = fmin(fmax(Q.u, lo), hi);
    const R ev = fma(eu - P.u, sv, P.v);
    const R xv = xu == Q.u ? Q.v : fma(xu - P.u, sv, P.v);
    s.d = xu - eu;
    s.any = s.d != R(0) || ev != xv;
    s.lo = fmin(ev, xv);
    s.hi = fmax(ev, xv);
    s.mid = R(0.5) * (s.lo + s.hi);
    s.c = s.d != R(0) ? copysign(R(0.5) * fabs(su), s.d) : R(0);
    return s;
}

template <class R>
__device__ inline void col_segments(const Pt<R> (&T)[3], const R (&sv)[3], const R (&su)[3], R lo, R hi,
                                    ColSegs<R> &S)
{
    S.e0 = col_seg(T[0], T[1], lo, hi, sv[0], su[0]);
    S.e1 = col_seg(T[1], T[2], lo, hi, sv[1], su[1]);
    S.e2 = col_seg(T[2], T[0], lo, hi, sv[2], su[2]);
}

// d I(r - a, r - b) without case branches: below the edge's v range the
// crossing form (r - lo)^2 c is 0 once r - lo is clamped at 0; above it the
// linear form d (r - (lo + hi) / 2) applies
template <class R>
__device__ inline R col_term(const ColSeg<R> &e, R r)
{
    const R t = fmax(r - e.lo, R(0));
    const R cross = t * t * e.c;
    const R full = e.d * (r - e.mid);
    return r >= e.hi ? full : cross;
}

// area below v = r inside the column: sum_e d_e I(r - a_e, r - b_e)
template <class R>
__device__ inline R col_cumulative(const ColSegs<R> &S, R r)
{
    return col_term(S.e0, r) + col_term(S.e1, r) + col_term(S.e2, r);
}

// widen [lo, hi] to the v range of a clipped edge (if it has one)
template <class R>
__device__ inline void col_range(const ColSeg<R> &e, R &lo, R &hi)
{
    if (e.any) {
        lo = fmin(lo, e.lo);
        hi = fmax(hi, e.hi);
    }
}

}  // namespace mlm
