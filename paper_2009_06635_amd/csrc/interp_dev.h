// Device functions of the interpolation (shared by the interpolation,
// batched and surrogate kernels): knot search, Hermite stencil weights,
// point location, in-grid stencil sum and the extrapolation formulas.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdfmi_dev.h"

namespace pdfmi {

// Largest i in [0, n-2] with t[i] <= v, 0 if t[0] > v (t strictly increasing).
__device__ __forceinline__ int find_cell(const double* __restrict__ t, int n, double v) {
  const int last = n - 2;
  int i = 0;
  int step = last > 0 ? (1 << (31 - __builtin_clz((unsigned)last))) : 0;
  for (; step > 0; step >>= 1) {
    const int j = i + step;
    if (j <= last && t[j] <= v) i = j;
  }
  return i;
}

// Same index as find_cell, from the table's bucket hints (see HintAxis):
// one hint read, then two independent knot comparisons.  v > 0.
__device__ __forceinline__ int find_cell_hint(const double* __restrict__ t, int n, double v, const HintAxis& h,
                                              const short* __restrict__ hints) {
  if (h.off < 0) return find_cell(t, n, v);
  const int last = n - 2;
  const unsigned key = (unsigned)((unsigned long long)__double_as_longlong(v) >> h.shift);
  const int b = min(max((int)(key - h.key0), 0), h.n - 1);
  const int i = hints[h.off + b];
  const int i1 = min(i + 1, last), i2 = min(i + 2, last);
  return i + ((i + 1 <= last && t[i1] <= v) ? 1 : 0) + ((i + 2 <= last && t[i2] <= v) ? 1 : 0);
}

// Point-location tables as a kernel reads them: from LDS (staged copy of the
// member's table block) or from global memory.
struct Tables {
  const double* knots;
  const CellCoef* cells;
  const short* hints;
  const SubDesc* subs;
};

__device__ __forceinline__ Tables tables_at(const unsigned char* base, const MemberDev& m) {
  return Tables{reinterpret_cast<const double*>(base), reinterpret_cast<const CellCoef*>(base + m.cells_off),
                reinterpret_cast<const short*>(base + m.hints_off), reinterpret_cast<const SubDesc*>(base + m.subs_off)};
}

// Hermite weights of knots i-1..i+2 re-based onto the stencil that starts at
// knot i - d (d = 0 left edge, 1 interior, 2 right edge).
template <typename T>
__device__ __forceinline__ void stencil_weights(double u64, const CellCoef& c, int d, T out[4]) {
  // the Hermite basis in factored form: 1 - u is exact, so every basis value
  // keeps its relative precision near u = 0 and u = 1 (the expanded forms
  // cancel there, leaving absolute errors of one ulp that the large weights
  // of a cell next to a much narrower one magnify)
  const T u = (T)u64;
  const T w = (T)1 - u;
  const T u2 = u * u, w2 = w * w;
  const T h00 = w2 * ((T)1 + (T)2 * u);
  const T h10 = u * w2;
  const T h01 = ((T)3 - (T)2 * u) * u2;
  const T h11 = -(w * u2);
  const bool L = c.hl >= 0.0, R = c.hr >= 0.0;
  const double am1 = L ? -c.hl : 0.0, a0 = L ? c.hl - 0.5 : -1.0, a1 = L ? 0.5 : 1.0;
  const double b0 = R ? -0.5 : -1.0, b1 = R ? 0.5 - c.hr : 1.0, b2 = R ? c.hr : 0.0;
  T r[4];
  r[0] = h10 * (T)am1;
  r[1] = h00 + h10 * (T)a0 + h11 * (T)b0;
  r[2] = h01 + h10 * (T)a1 + h11 * (T)b1;
  r[3] = h11 * (T)b2;
  out[0] = d == 0 ? r[1] : (d == 1 ? r[0] : (T)0);
  out[1] = d == 0 ? r[2] : (d == 1 ? r[1] : r[0]);
  out[2] = d == 0 ? r[3] : (d == 1 ? r[2] : r[1]);
  out[3] = d == 1 ? r[3] : (d == 2 ? r[2] : (T)0);
}

// Cell parameter with exact 0 / 1 at the cell's knots.
__device__ __forceinline__ double cell_u(double v, const CellCoef& c) {
  return v == c.t0 ? 0.0 : (v == c.t1 ? 1.0 : log(v * c.inv_t0) * c.invD);
}

// alpha_s at one Q^2 from the table (knots sk, values sv, cells sc); NaN for
// Q^2 <= 0 or non-finite.
__device__ __forceinline__ double alphas_point(const AlphasDev& A, const double* sk, const double* sv,
                                               const CellCoef* sc, const short* sh, double q2) {
  const bool valid = q2 > 0.0 && q2 < INFINITY;
  if (!valid) return NAN;
  if (q2 < sk[0]) return sv[0];
  if (q2 > sk[A.n - 1]) return sv[A.n - 1];
  int s = 0;
  for (int j = 1; j < A.nseg; ++j)
    if (A.seg_first[j] <= q2) s = j;
  const int lo = A.seg_lo[s], hi = A.seg_hi[s];
  const int m = hi - lo + 1;
  const int c = lo + find_cell_hint(sk + lo, m, q2, A.seg_hint[s], sh);
  const CellCoef cc = sc[c];
  const int m4 = m < 4 ? m : 4;
  const int st = min(max(c - 1, lo), hi - m4 + 1);
  double w[4];
  stencil_weights<double>(cell_u(q2, cc), cc, c - st, w);
  double acc = w[0] * sv[st];
  for (int a = 1; a < m4; ++a) acc = fma(w[a], sv[st + a], acc);
  return acc;
}


// The alpha_s table as a kernel reads it (staged in LDS) and where a fused
// evaluation writes alpha_s: out == nullptr means no alpha_s output.
struct AsView {
  const double* k;
  const double* v;
  const CellCoef* c;
  const short* h;
  double* out;
};

struct PointLoc {
  int mode;      // region bits | kXHigh | (anchor row << 8) for high Q^2
  int k, ix, iq;
  int sx, sq;    // stencil origin (first x and Q^2 knot of the 4x4 stencil)
  int base;      // element offset of f[sx][sq][0]
  int sa;        // element stride between x knots
  double p0, p1; // extrapolation parameters
};

// Phase 1: everything that depends on the point only.
template <typename T>
__device__ __forceinline__ PointLoc locate_point(const MemberDev& m, const Tables& tb, double x, double q2, T w[4],
                                                 T v[4]) {
  PointLoc L;
  L.p0 = 0.0;
  L.p1 = 0.0;
  const bool valid = (x > 0.0) && (x <= m.xmax) && (q2 > 0.0) && (q2 < INFINITY);
  if (!valid) {
    L.mode = kInvalid;
    L.k = L.ix = L.iq = -1;
    L.sx = L.sq = 0;
    L.base = 0;
    L.sa = 0;
    for (int a = 0; a < 4; ++a) w[a] = v[a] = (T)0;
    return L;
  }
  int mode = 0;
  if (x < m.xmin) mode |= kLowX;
  if (q2 < m.qmin) mode |= kLowQ;
  if (q2 > m.qmax) mode |= kHighQ;
  int k = 0;
  for (int j = 1; j < m.K; ++j)
    if (m.sub[j].qfirst <= q2) k = j;
  const SubDesc S = tb.subs[k];
  const int ix = find_cell_hint(tb.knots + S.xk_off, S.nx, x, S.xh, tb.hints);
  const int iq = find_cell_hint(tb.knots + S.qk_off, S.nq, q2, S.qh, tb.hints);
  const CellCoef cx = tb.cells[S.xc_off + ix];
  const CellCoef cq = tb.cells[S.qc_off + iq];
  const int sx = min(max(ix - 1, 0), S.nxp - 4);
  const int sq = min(max(iq - 1, 0), S.nqp - 4);
  // one logarithm per axis whatever the region: below x_0 the cell is the
  // first one and ux = ln(x/x_0) / ln(x_1/x_0) is the continuation parameter
  // itself; above the last Q^2 knot uq - 1 = ln(Q^2/q_n-1) / ln(q_n-1/q_n-2)
  const double ux = cell_u(x, cx);
  const double uq = cell_u(q2, cq);
  if (!(mode & kLowX)) {
    stencil_weights<T>(ux, cx, ix - sx, w);
  } else {
    for (int a = 0; a < 4; ++a) w[a] = (T)0;
    if (mode & (kLowQ | kHighQ)) L.p1 = ux; else L.p0 = ux;
  }
  if (!(mode & (kLowQ | kHighQ))) {
    stencil_weights<T>(uq, cq, iq - sq, v);
  } else {
    for (int b = 0; b < 4; ++b) v[b] = (T)0;
    if (mode & kLowQ) {
      L.p0 = q2 * cq.inv_t0;                       // r = Q^2 / Q^2_0
    } else {
      L.p0 = uq - 1.0;                             // s = ln(Q^2/q_n-1) / ln(q_n-1/q_n-2)
      mode |= (S.nq - 2 - sq) << 8;                // stencil row of q_n-2
    }
  }
  if (x > 0.9) mode |= kXHigh;
  L.mode = mode;
  L.k = k;
  L.ix = ix;
  L.iq = iq;
  L.sx = sx;
  L.sq = sq;
  const int Pp = sizeof(T) == 8 ? m.P64 : m.P32;
  L.sa = S.nqp * Pp;
  L.base = (int)((sizeof(T) == 8 ? S.val_off64 : S.val_off32) + (int64_t)(sx * S.nqp + sq) * Pp);
  return L;
}

// The same location in two halves, for points that share Q^2 (the two
// lookups of a Monte-Carlo point): the Q^2 half (validity of Q^2, region bits,
// sub-grid, Q^2 cell and weights) is computed once, the x half completes each
// location.  locate_x(locate_q(q2), x) equals locate_point(x, q2) field by
// field (the fused Monte-Carlo sum, which uses the halves, is compared bit
// for bit with the unfused one, which uses locate_point); locate_point stays
// one function because the split form compiles to a slower schedule in the
// fused x*f + alpha_s kernel.
template <typename T>
struct QLoc {
  int mode;      // kInvalid (Q^2 <= 0 or not finite), else kLowQ | kHighQ | (anchor row << 8)
  int k, iq, sq;
  double p0;     // Q^2 continuation parameter (below Q^2_min: r; above Q^2_max: s)
  T v[4];
};

template <typename T>
__device__ __forceinline__ QLoc<T> locate_q(const MemberDev& m, const Tables& tb, double q2) {
  QLoc<T> Q;
  Q.p0 = 0.0;
  for (int b = 0; b < 4; ++b) Q.v[b] = (T)0;
  if (!((q2 > 0.0) && (q2 < INFINITY))) {
    Q.mode = kInvalid;
    Q.k = Q.iq = -1;
    Q.sq = 0;
    return Q;
  }
  int mode = 0;
  if (q2 < m.qmin) mode |= kLowQ;
  if (q2 > m.qmax) mode |= kHighQ;
  int k = 0;
  for (int j = 1; j < m.K; ++j)
    if (m.sub[j].qfirst <= q2) k = j;
  const SubDesc S = tb.subs[k];
  const int iq = find_cell_hint(tb.knots + S.qk_off, S.nq, q2, S.qh, tb.hints);
  const CellCoef cq = tb.cells[S.qc_off + iq];
  const int sq = min(max(iq - 1, 0), S.nqp - 4);
  // one logarithm whatever the region: above the last knot
  // uq - 1 = ln(Q^2/q_n-1) / ln(q_n-1/q_n-2)
  const double uq = cell_u(q2, cq);
  if (!(mode & (kLowQ | kHighQ))) {
    stencil_weights<T>(uq, cq, iq - sq, Q.v);
  } else if (mode & kLowQ) {
    Q.p0 = q2 * cq.inv_t0;                         // r = Q^2 / Q^2_0
  } else {
    Q.p0 = uq - 1.0;                               // s = ln(Q^2/q_n-1) / ln(q_n-1/q_n-2)
    mode |= (S.nq - 2 - sq) << 8;                  // stencil row of q_n-2
  }
  Q.mode = mode;
  Q.k = k;
  Q.iq = iq;
  Q.sq = sq;
  return Q;
}

template <typename T>
__device__ __forceinline__ PointLoc locate_x(const MemberDev& m, const Tables& tb, const QLoc<T>& Q, double x, T w[4],
                                             T v[4]) {
  PointLoc L;
  L.p0 = 0.0;
  L.p1 = 0.0;
  if ((Q.mode & kInvalid) || !((x > 0.0) && (x <= m.xmax))) {
    L.mode = kInvalid;
    L.k = L.ix = L.iq = -1;
    L.sx = L.sq = 0;
    L.base = 0;
    L.sa = 0;
    for (int a = 0; a < 4; ++a) w[a] = v[a] = (T)0;
    return L;
  }
  int mode = Q.mode;
  const bool qout = mode & (kLowQ | kHighQ);
  const SubDesc S = tb.subs[Q.k];
  const int ix = find_cell_hint(tb.knots + S.xk_off, S.nx, x, S.xh, tb.hints);
  const CellCoef cx = tb.cells[S.xc_off + ix];
  const int sx = min(max(ix - 1, 0), S.nxp - 4);
  // below x_0 the cell is the first one and ux = ln(x/x_0) / ln(x_1/x_0) is
  // the continuation parameter itself
  const double ux = cell_u(x, cx);
  if (!(x < m.xmin)) {
    stencil_weights<T>(ux, cx, ix - sx, w);
  } else {
    mode |= kLowX;
    for (int a = 0; a < 4; ++a) w[a] = (T)0;
    if (qout) L.p1 = ux; else L.p0 = ux;
  }
  if (qout) L.p0 = Q.p0;
  for (int b = 0; b < 4; ++b) v[b] = Q.v[b];
  if (x > 0.9) mode |= kXHigh;
  L.mode = mode;
  L.k = Q.k;
  L.ix = ix;
  L.iq = Q.iq;
  L.sx = sx;
  L.sq = Q.sq;
  const int Pp = sizeof(T) == 8 ? m.P64 : m.P32;
  L.sa = S.nqp * Pp;
  L.base = (int)((sizeof(T) == 8 ? S.val_off64 : S.val_off32) + (int64_t)(sx * S.nqp + Q.sq) * Pp);
  return L;
}

// a^b for a > 0 as exp(b ln a): the bases here are positive ratios, and a
// few ulps of exp and log stay far inside the FP64 parity bound, at a
// fraction of the general pow's cost (the extrapolated points of a tile run
// these formulas on a few of the wave's lanes).
__device__ __forceinline__ double pos_pow(double a, double b) { return exp(b * log(a)); }
// Two-anchor continuation (log-linear when both anchors exceed 1e-3).
__device__ __forceinline__ double cont_low(double f0, double f1, double s) {
  return (f0 > 1e-3 && f1 > 1e-3) ? f0 * pos_pow(f1 / f0, s) : f0 + s * (f1 - f0);
}
__device__ __forceinline__ double cont_high(double f0, double f1, double s) {
  return (f0 > 1e-3 && f1 > 1e-3) ? f1 * pos_pow(f1 / f0, s) : f1 + s * (f1 - f0);
}
// Below Q^2_min: f0 * r^(gamma r + 1 - r), gamma from the first two Q^2 knots.
__device__ __forceinline__ double low_q(double f0, double f1, double r, double invL01, bool xhigh) {
  const bool use_gamma = f0 > 1e-5 && f1 > 1e-5 && !xhigh;
  if (!use_gamma) return f0 * r;
  const double lr = log(r);
  const double gamma = log(f1 / f0) * invL01;
  return f0 * exp((gamma * r + 1.0 - r) * lr);
}

// Extrapolated value from anchor values (rare path, FP64 combination):
//   x below x_min only:      a0, a1 = rows x_0, x_1 interpolated in Q^2
//   Q^2 outside, x inside:   a0, a1 = anchor Q^2 rows interpolated in x
//   corners:                 a0, a1 (x_0, x_1 on the lower anchor row),
//                            a2, a3 (x_0, x_1 on the upper anchor row)
static __device__ __noinline__ double extrapolate(int mode, double a0, double a1, double a2, double a3, double p0,
                                           double p1, double invL01) {
  const bool lowx = mode & kLowX, lowq = mode & kLowQ, highq = mode & kHighQ;
  const bool xhigh = mode & kXHigh;
  if (lowx && !(lowq || highq)) return cont_low(a0, a1, p0);
  if (!lowx) return lowq ? low_q(a0, a1, p0, invL01, xhigh) : cont_high(a0, a1, p0);
  // corners: continue in x on the two anchor rows first, then in Q^2
  const double g0 = cont_low(a0, a1, p1);
  const double g1 = cont_low(a2, a3, p1);
  return lowq ? low_q(g0, g1, p0, invL01, xhigh) : cont_high(g0, g1, p0);
}

template <typename T>
__device__ __forceinline__ const T* member_values(const MemberDev& m);
template <>
__device__ __forceinline__ const double* member_values<double>(const MemberDev& m) { return m.v64; }
template <>
__device__ __forceinline__ const float* member_values<float>(const MemberDev& m) { return m.v32; }

// In-grid value of one column from its gathered 4x4 stencil: the x-direction
// weights on each of the four Q^2 rows, then the Q^2-direction weights.
// stencil_step adds Q^2 row b (its four x-knot values f0..f3) to the running
// sum acc; interp_stencil is the four steps in order, and a caller that
// gathers the stencil row by row may take the steps itself with the same
// result.
template <typename T>
__device__ __forceinline__ T stencil_step(int b, T acc, T f0, T f1, T f2, T f3, const T w[4], const T v[4]) {
  T g = w[0] * f0;
  g = fma(w[1], f1, g);
  g = fma(w[2], f2, g);
  g = fma(w[3], f3, g);
  return b == 0 ? v[0] * g : fma(v[b], g, acc);
}

template <typename T>
__device__ __forceinline__ T interp_stencil(const T F[4][4], const T w[4], const T v[4]) {
  T acc = (T)0;
#pragma unroll
  for (int b = 0; b < 4; ++b) acc = stencil_step<T>(b, acc, F[0][b], F[1][b], F[2][b], F[3][b], w, v);
  return acc;
}

// Extrapolated value of one column (rare path).  f points at the column's
// entry of the stencil origin; only the anchor knots the formula needs are
// read:
//   x below x_min only:     rows x_0, x_1 interpolated in Q^2
//   Q^2 outside, x inside:  the two anchor Q^2 rows interpolated in x
//   corners:                the four anchor knot values
struct Wts {
  double w0, w1, w2, w3, v0, v1, v2, v3;
};

template <typename T>
__device__ __noinline__ double extrap_entry(const T* f, int sa, int Pp, int mode, Wts wt, double p0, double p1,
                                            double invL01) {
  const double w[4] = {wt.w0, wt.w1, wt.w2, wt.w3};
  const double v[4] = {wt.v0, wt.v1, wt.v2, wt.v3};
  const bool lowx = mode & kLowX, lowq = mode & kLowQ, highq = mode & kHighQ;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  if (lowx && !(lowq || highq)) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      a0 += v[b] * (double)f[b * Pp];
      a1 += v[b] * (double)f[sa + b * Pp];
    }
  } else {
    const int ra = lowq ? 0 : (mode >> 8) & 3;
    if (!lowx) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        a0 += w[a] * (double)f[a * sa + ra * Pp];
        a1 += w[a] * (double)f[a * sa + (ra + 1) * Pp];
      }
    } else {
      a0 = (double)f[ra * Pp];
      a1 = (double)f[sa + ra * Pp];
      a2 = (double)f[(ra + 1) * Pp];
      a3 = (double)f[sa + (ra + 1) * Pp];
    }
  }
  return extrapolate(mode, a0, a1, a2, a3, p0, p1, invL01);
}


// Value of one stored column at one point (location, weights, stencil and,
// outside the grid, the extrapolation formula); NaN for an invalid point.
template <typename T>
__device__ __forceinline__ T interp_point(const MemberDev& m, const Tables& tb, double x, double q2, int col,
                                          double invL01) {
  T w[4], v[4];
  const PointLoc L = locate_point<T>(m, tb, x, q2, w, v);
  if (L.mode & kInvalid) return (T)NAN;
  const int Pp = sizeof(T) == 8 ? m.P64 : m.P32;
  const T* f = member_values<T>(m) + L.base + col;
  if (!(L.mode & (kLowX | kLowQ | kHighQ))) {
    T F[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) F[a][b] = f[a * L.sa + b * Pp];
    return interp_stencil<T>(F, w, v);
  }
  const Wts wt{(double)w[0], (double)w[1], (double)w[2], (double)w[3],
               (double)v[0], (double)v[1], (double)v[2], (double)v[3]};
  return (T)extrap_entry<T>(f, L.sa, Pp, L.mode, wt, L.p0, L.p1, invL01);
}

}  // namespace pdfmi
