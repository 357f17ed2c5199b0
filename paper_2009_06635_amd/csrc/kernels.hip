// HIP kernels for gfx950: x*f(x,Q^2) log-bicubic interpolation, point
// location, and alpha_s(Q^2) log-cubic interpolation.
//
// Interpolation (paper section 2.2): cubic Hermite in ln x then in ln Q^2 with
// finite-difference slopes, written as a separable 4x4 weighted sum
//   xf = sum_b v_b * sum_a w_a * f[sx+a][sq+b][col]
// where w (x direction) and v (Q^2 direction) are the Hermite weights of the
// point's cell, re-based onto a 4-knot stencil that stays inside the sub-grid
// (one-sided slopes at sub-grid edges give zero weight outside it).
// Extrapolation (figure 1 EXTRAPOLATE) uses anchor values on the edge rows or
// columns of the same stencil, combined in FP64.
//
// Work split per tile of 256 points:
//   phase 1, one lane per point: validate, region, sub-grid, FP64 knot search
//     (raw FP64 comparisons), FP64 log transform, Hermite weights -> LDS;
//   phase 2, one lane per (point, flavour), consecutive lanes on consecutive
//     output elements (coalesced point-major stores): 16 grid reads from LDS
//     (grid staged once per workgroup when it fits) or from L2-resident
//     global memory, 20 FMAs.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pdfmi_dev.h"

namespace pdfmi {

constexpr int kTile = 256;  // points per tile == threads per workgroup

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

// Hermite weights of knots i-1..i+2 re-based onto the stencil that starts at
// knot i - d (d = 0 left edge, 1 interior, 2 right edge).
template <typename T>
__device__ __forceinline__ void stencil_weights(double u64, const CellCoef& c, int d, T out[4]) {
  const T u = (T)u64;
  const T u2 = u * u;
  const T h00 = ((T)2 * u - (T)3) * u2 + (T)1;
  const T h10 = ((u - (T)2) * u + (T)1) * u;
  const T h01 = ((T)3 - (T)2 * u) * u2;
  const T h11 = (u - (T)1) * u2;
  T r[4];
  r[0] = h10 * (T)c.am1;
  r[1] = h00 + h10 * (T)c.a0 + h11 * (T)c.b0;
  r[2] = h01 + h10 * (T)c.a1 + h11 * (T)c.b1;
  r[3] = h11 * (T)c.b2;
  out[0] = d == 0 ? r[1] : (d == 1 ? r[0] : (T)0);
  out[1] = d == 0 ? r[2] : (d == 1 ? r[1] : r[0]);
  out[2] = d == 0 ? r[3] : (d == 1 ? r[2] : r[1]);
  out[3] = d == 1 ? r[3] : (d == 2 ? r[2] : (T)0);
}

// Cell parameter with exact 0 / 1 at the cell's knots.
__device__ __forceinline__ double cell_u(double v, const CellCoef& c) {
  return v == c.t0 ? 0.0 : (v == c.t1 ? 1.0 : log(v * c.inv_t0) * c.invD);
}

struct PointLoc {
  int mode;      // region bits | kXHigh | (anchor row << 8) for high Q^2
  int k, ix, iq;
  int base;      // element offset of f[sx][sq][0]
  int sa;        // element stride between x knots
  double p0, p1; // extrapolation parameters
};

// Phase 1: everything that depends on the point only.
template <typename T>
__device__ __forceinline__ PointLoc locate_point(const MemberDev& m, double x, double q2, T w[4], T v[4]) {
  PointLoc L;
  L.p0 = 0.0;
  L.p1 = 0.0;
  const bool valid = (x > 0.0) && (x <= m.xmax) && (q2 > 0.0) && (q2 < INFINITY);
  if (!valid) {
    L.mode = kInvalid;
    L.k = L.ix = L.iq = -1;
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
  const SubDesc& S = m.sub[k];
  const int ix = find_cell(m.knots + S.xk_off, S.nx, x);
  const int iq = find_cell(m.knots + S.qk_off, S.nq, q2);
  const CellCoef cx = m.cells[S.xc_off + ix];
  const CellCoef cq = m.cells[S.qc_off + iq];
  const int sx = min(max(ix - 1, 0), S.nxp - 4);
  const int sq = min(max(iq - 1, 0), S.nqp - 4);
  if (!(mode & kLowX)) {
    stencil_weights<T>(cell_u(x, cx), cx, ix - sx, w);
  } else {
    for (int a = 0; a < 4; ++a) w[a] = (T)0;
    // continuation in ln x from knots 0 and 1: s = ln(x/x_0) / ln(x_1/x_0)
    const double sx_par = log(x * cx.inv_t0) * cx.invD;
    if (mode & (kLowQ | kHighQ)) L.p1 = sx_par; else L.p0 = sx_par;
  }
  if (!(mode & (kLowQ | kHighQ))) {
    stencil_weights<T>(cell_u(q2, cq), cq, iq - sq, v);
  } else {
    for (int b = 0; b < 4; ++b) v[b] = (T)0;
    if (mode & kLowQ) {
      L.p0 = q2 / cq.t0;                          // r = Q^2 / Q^2_0
    } else {
      L.p0 = log(q2 / cq.t1) * cq.invD;            // s = ln(Q^2/q_n-1) / ln(q_n-1/q_n-2)
      mode |= (S.nq - 2 - sq) << 8;                // stencil row of q_n-2
    }
  }
  if (x > 0.9) mode |= kXHigh;
  L.mode = mode;
  L.k = k;
  L.ix = ix;
  L.iq = iq;
  L.sa = S.nqp * m.P;
  L.base = (int)(S.val_off + (int64_t)(sx * S.nqp + sq) * m.P);
  return L;
}

// Two-anchor continuation (log-linear when both anchors exceed 1e-3).
__device__ __forceinline__ double cont_low(double f0, double f1, double s) {
  return (f0 > 1e-3 && f1 > 1e-3) ? f0 * pow(f1 / f0, s) : f0 + s * (f1 - f0);
}
__device__ __forceinline__ double cont_high(double f0, double f1, double s) {
  return (f0 > 1e-3 && f1 > 1e-3) ? f1 * pow(f1 / f0, s) : f1 + s * (f1 - f0);
}
// Below Q^2_min: f0 * r^(gamma r + 1 - r), gamma from the first two Q^2 knots.
__device__ __forceinline__ double low_q(double f0, double f1, double r, double invL01, bool xhigh) {
  const bool use_gamma = f0 > 1e-5 && f1 > 1e-5 && !xhigh;
  if (!use_gamma) return f0 * r;
  const double gamma = log(f1 / f0) * invL01;
  return f0 * pow(r, gamma * r + 1.0 - r);
}

// Extrapolated value from the 4x4 stencil F (rare path, FP64 combination).
template <typename T>
__device__ __noinline__ double extrapolate(const T F[4][4], int mode, const T w[4], const T v[4],
                                           double p0, double p1, double invL01) {
  const bool lowx = mode & kLowX, lowq = mode & kLowQ, highq = mode & kHighQ;
  const bool xhigh = mode & kXHigh;
  const int r0 = (mode >> 8) & 3;
  if (lowx && !(lowq || highq)) {
    double f0 = 0.0, f1 = 0.0;
    for (int b = 0; b < 4; ++b) {
      f0 += (double)v[b] * (double)F[0][b];
      f1 += (double)v[b] * (double)F[1][b];
    }
    return cont_low(f0, f1, p0);
  }
  if (!lowx) {
    const int ra = lowq ? 0 : r0;
    double f0 = 0.0, f1 = 0.0;
    for (int a = 0; a < 4; ++a) {
      f0 += (double)w[a] * (double)F[a][ra];
      f1 += (double)w[a] * (double)F[a][ra + 1];
    }
    return lowq ? low_q(f0, f1, p0, invL01, xhigh) : cont_high(f0, f1, p0);
  }
  // corners: continue in x on the two anchor rows first, then in Q^2
  const int ra = lowq ? 0 : r0;
  const double g0 = cont_low((double)F[0][ra], (double)F[1][ra], p1);
  const double g1 = cont_low((double)F[0][ra + 1], (double)F[1][ra + 1], p1);
  return lowq ? low_q(g0, g1, p0, invL01, xhigh) : cont_high(g0, g1, p0);
}

template <typename T>
__device__ __forceinline__ const T* member_values(const MemberDev& m);
template <>
__device__ __forceinline__ const double* member_values<double>(const MemberDev& m) { return m.v64; }
template <>
__device__ __forceinline__ const float* member_values<float>(const MemberDev& m) { return m.v32; }

// One (point, flavour) output from its stencil.
template <typename T>
__device__ __forceinline__ T eval_entry(const T* __restrict__ f, int sa, int P, int mode,
                                        const T w[4], const T v[4], double p0, double p1,
                                        double invL01) {
  T F[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) F[a][b] = f[a * sa + b * P];
  if ((mode & (kLowX | kLowQ | kHighQ)) == 0) {
    T acc;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      T g = w[0] * F[0][b];
      g = fma(w[1], F[1][b], g);
      g = fma(w[2], F[2][b], g);
      g = fma(w[3], F[3][b], g);
      acc = b == 0 ? v[0] * g : fma(v[b], g, acc);
    }
    return acc;
  }
  return (T)extrapolate<T>(F, mode, w, v, p0, p1, invL01);
}

// x*f for a set of flavours; see file header.  out is point-major [n][R].
template <typename T, bool kLdsGrid>
__global__ __launch_bounds__(kTile) void k_xfxq2(MemberDev m, ReqCols rc, const double* __restrict__ X,
                                                  const double* __restrict__ Q2, int64_t n, T* __restrict__ out,
                                                  unsigned long long* __restrict__ nerr, int lds_grid_elems,
                                                  double invL01) {
  extern __shared__ __align__(16) unsigned char smem[];
  T* sw = reinterpret_cast<T*>(smem);                 // [kTile][4]
  T* sv = sw + kTile * 4;                             // [kTile][4]
  double* sp = reinterpret_cast<double*>(sv + kTile * 4);  // [kTile][2]
  int* sbase = reinterpret_cast<int*>(sp + 2 * kTile);
  int* ssa = sbase + kTile;
  int* smode = ssa + kTile;
  T* sgrid = reinterpret_cast<T*>(smode + kTile);      // 16-byte aligned (kTile multiple of 4)

  const T* gvals = member_values<T>(m);
  if constexpr (kLdsGrid) {
    for (int i = threadIdx.x; i < lds_grid_elems; i += kTile) sgrid[i] = gvals[i];
    __syncthreads();
  }
  const int R = rc.n;
  const int t = threadIdx.x;
  const int64_t ntiles = (n + kTile - 1) / kTile;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    const int64_t pbeg = tile * kTile;
    const int tp = (int)min((int64_t)kTile, n - pbeg);
    bool bad = false;
    if (t < tp) {
      T w[4], v[4];
      const PointLoc L = locate_point<T>(m, X[pbeg + t], Q2[pbeg + t], w, v);
      bad = L.mode & kInvalid;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        sw[t * 4 + a] = w[a];
        sv[t * 4 + a] = v[a];
      }
      sp[2 * t] = L.p0;
      sp[2 * t + 1] = L.p1;
      sbase[t] = L.base;
      ssa[t] = L.sa;
      smode[t] = L.mode;
    }
    const unsigned long long bal = __ballot(bad);
    if (bal && (t & 63) == 0) atomicAdd(nerr, (unsigned long long)__popcll(bal));
    __syncthreads();
    const int nev = tp * R;
    T* obase = out + pbeg * R;
    int p = t / R, j = t - (t / R) * R;
    const int dp = kTile / R, dj = kTile - (kTile / R) * R;
    for (int e = t; e < nev; e += kTile) {
      const int mode = smode[p];
      const int col = rc.col[j];
      T val;
      if (mode & kInvalid) {
        val = (T)NAN;
      } else if (col < 0) {
        val = (T)0;
      } else {
        T w[4], v[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          w[a] = sw[p * 4 + a];
          v[a] = sv[p * 4 + a];
        }
        const int off = sbase[p] + col;
        if constexpr (kLdsGrid)
          val = eval_entry<T>(sgrid + off, ssa[p], m.P, mode, w, v, sp[2 * p], sp[2 * p + 1], invL01);
        else
          val = eval_entry<T>(gvals + off, ssa[p], m.P, mode, w, v, sp[2 * p], sp[2 * p + 1], invL01);
      }
      obase[e] = val;
      p += dp;
      j += dj;
      if (j >= R) {
        j -= R;
        ++p;
      }
    }
    __syncthreads();
  }
}

// Location only (sub-grid, cells, region), one lane per point.
__global__ __launch_bounds__(256) void k_locate(MemberDev m, const double* __restrict__ X,
                                                const double* __restrict__ Q2, int64_t n,
                                                int32_t* __restrict__ ko, int32_t* __restrict__ ixo,
                                                int32_t* __restrict__ iqo, int8_t* __restrict__ rego) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double w[4], v[4];
    const PointLoc L = locate_point<double>(m, X[i], Q2[i], w, v);
    ko[i] = L.k;
    ixo[i] = L.ix;
    iqo[i] = L.iq;
    rego[i] = (int8_t)(L.mode & (kLowX | kLowQ | kHighQ | kInvalid));
  }
}

// alpha_s(Q^2) (paper section 2.3): segment (repeated knot = threshold, the
// upper segment owns it), FP64 knot search, cubic Hermite in ln Q^2 with
// one-sided slopes at segment ends, constant outside the knots.
__global__ __launch_bounds__(256) void k_alphas(AlphasDev A, const double* __restrict__ Q2, int64_t n,
                                                double* __restrict__ out, unsigned long long* __restrict__ nerr) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double q2 = Q2[i];
    const bool valid = q2 > 0.0 && q2 < INFINITY;
    double r;
    if (!valid) {
      r = NAN;
    } else if (q2 < A.knots[0]) {
      r = A.vals[0];
    } else if (q2 > A.knots[A.n - 1]) {
      r = A.vals[A.n - 1];
    } else {
      int s = 0;
      for (int j = 1; j < A.nseg; ++j)
        if (A.seg_first[j] <= q2) s = j;
      const int lo = A.seg_lo[s], hi = A.seg_hi[s];
      const int m = hi - lo + 1;
      const int c = lo + find_cell(A.knots + lo, m, q2);
      const CellCoef cc = A.cells[c];
      const int m4 = m < 4 ? m : 4;
      const int st = min(max(c - 1, lo), hi - m4 + 1);
      double w[4];
      stencil_weights<double>(cell_u(q2, cc), cc, c - st, w);
      double acc = w[0] * A.vals[st];
      for (int a = 1; a < m4; ++a) acc = fma(w[a], A.vals[st + a], acc);
      r = acc;
    }
    const unsigned long long bal = __ballot(!valid);
    if (bal && (threadIdx.x & 63) == 0) atomicAdd(nerr, (unsigned long long)__popcll(bal));
    out[i] = r;
  }
}

// ---------------------------------------------------------------------------------------
// Launchers (host side, called by pdfmi.cpp)

size_t xfxq2_record_bytes(bool f32) { return (size_t)kTile * (8 * (f32 ? 4 : 8) + 16 + 12); }

template <typename T>
static hipError_t launch_xfxq2_t(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2,
                                 int64_t n, T* out, unsigned long long* nerr, int lds_grid_elems,
                                 double invL01, int n_cu, hipStream_t s) {
  const size_t rec = xfxq2_record_bytes(sizeof(T) == 4);
  const int64_t ntiles = (n + kTile - 1) / kTile;
  if (lds_grid_elems > 0) {
    const size_t shm = rec + (size_t)lds_grid_elems * sizeof(T);
    const int per_cu = (int)(160 * 1024 / shm) > 0 ? (int)(160 * 1024 / shm) : 1;
    const int64_t nb = min(ntiles, (int64_t)n_cu * per_cu);
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_xfxq2<T, true>),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_xfxq2<T, true>), dim3((unsigned)nb), dim3(kTile), shm, s, m, rc, x, q2, n, out, nerr,
                       lds_grid_elems, invL01);
  } else {
    const int64_t nb = min(ntiles, (int64_t)n_cu * 8);
    hipLaunchKernelGGL((k_xfxq2<T, false>), dim3((unsigned)nb), dim3(kTile), rec, s, m, rc, x, q2, n, out, nerr,
                       0, invL01);
  }
  return hipGetLastError();
}

hipError_t launch_xfxq2_f64(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2, int64_t n,
                            double* out, unsigned long long* nerr, int lds_grid_elems, double invL01, int n_cu,
                            hipStream_t s) {
  return launch_xfxq2_t<double>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, n_cu, s);
}

hipError_t launch_xfxq2_f32(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2, int64_t n,
                            float* out, unsigned long long* nerr, int lds_grid_elems, double invL01, int n_cu,
                            hipStream_t s) {
  return launch_xfxq2_t<float>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, n_cu, s);
}

hipError_t launch_locate(const MemberDev& m, const double* x, const double* q2, int64_t n, int32_t* k, int32_t* ix,
                         int32_t* iq, int8_t* reg, int n_cu, hipStream_t s) {
  const int64_t nb = min((n + 255) / 256, (int64_t)n_cu * 16);
  hipLaunchKernelGGL(k_locate, dim3((unsigned)nb), dim3(256), 0, s, m, x, q2, n, k, ix, iq, reg);
  return hipGetLastError();
}

hipError_t launch_alphas(const AlphasDev& A, const double* q2, int64_t n, double* out, unsigned long long* nerr,
                         int n_cu, hipStream_t s) {
  const int64_t nb = min((n + 255) / 256, (int64_t)n_cu * 16);
  hipLaunchKernelGGL(k_alphas, dim3((unsigned)nb), dim3(256), 0, s, A, q2, n, out, nerr);
  return hipGetLastError();
}

}  // namespace pdfmi
