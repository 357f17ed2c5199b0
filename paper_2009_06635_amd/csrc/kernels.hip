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

#include "interp_dev.h"
#include "pdfmi_dev.h"

namespace pdfmi {


// 16-byte column groups of the vectorised path.
template <typename T, int G>
struct VecOf;
template <>
struct VecOf<double, 2> { using type = double2; };
template <>
struct VecOf<float, 4> { using type = float4; };
template <>
struct VecOf<double, 1> { using type = double; };
template <>
struct VecOf<float, 1> { using type = float; };

// Buffer resource over [base, base + bytes): loads and stores through it take
// a 32-bit per-lane byte offset plus a uniform (scalar) byte offset, so the
// stencil gathers need no 64-bit address arithmetic; the hardware returns
// zero for loads past `bytes` and drops stores past it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, 0x00020000);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// G consecutive elements of T (G * sizeof(T) in {4, 8, 16} bytes).
template <typename T, int G>
__device__ __forceinline__ void buf_load(__amdgpu_buffer_rsrc_t r, int voff, int soff, T* dst) {
  constexpr int kBytes = G * (int)sizeof(T);
  if constexpr (kBytes == 16) {
    const u32x4 q = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    const unsigned int u[4] = {q.x, q.y, q.z, q.w};
    __builtin_memcpy(dst, u, 16);
  } else if constexpr (kBytes == 8) {
    const u32x2 q = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    const unsigned int u[2] = {q.x, q.y};
    __builtin_memcpy(dst, u, 8);
  } else {
    static_assert(kBytes == 4, "unsupported gather width");
    const unsigned int u = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    __builtin_memcpy(dst, &u, 4);
  }
}

// Cache policy of the output stores: 0 (default) or kStoreStream, the
// non-temporal hint.  While the grid is gathered through L2, the streamed
// output rows then displace fewer grid lines (measured 5-9 % faster for 1e7
// points); with the grid staged in LDS the hint made the same call slower
// (0.31 -> 0.55 ms in FP32), so those kernels keep the default.
constexpr int kStoreStream = 2;

template <typename T, int G, int kPolicy = 0>
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t r, int voff, const T* src) {
  constexpr int kBytes = G * (int)sizeof(T);
  if constexpr (kBytes == 16) {
    unsigned int u[4];
    __builtin_memcpy(u, src, 16);
    __builtin_amdgcn_raw_buffer_store_b128(u32x4{u[0], u[1], u[2], u[3]}, r, voff, 0, kPolicy);
  } else if constexpr (kBytes == 8) {
    unsigned int u[2];
    __builtin_memcpy(u, src, 8);
    __builtin_amdgcn_raw_buffer_store_b64(u32x2{u[0], u[1]}, r, voff, 0, kPolicy);
  } else {
    static_assert(kBytes == 4, "unsupported store width");
    unsigned int u;
    __builtin_memcpy(&u, src, 4);
    __builtin_amdgcn_raw_buffer_store_b32(u, r, voff, 0, kPolicy);
  }
}

// Workgroup copy of `bytes` (a multiple of 4; both pointers 16-byte
// aligned) from global memory to LDS.  Each thread issues eight 16-byte loads
// before it stores them: a loop of dependent load-store pairs waits out the
// memory latency once per element (a 72 KB grid: 18 round trips per thread).
template <int BS>
__device__ __forceinline__ void stage_copy(void* dst, const void* src, int64_t bytes) {
  const u32x4* s = static_cast<const u32x4*>(src);
  u32x4* d = static_cast<u32x4*>(dst);
  const int64_t nv = bytes >> 4;
  for (int64_t i0 = threadIdx.x; i0 < nv; i0 += 8 * BS) {
    u32x4 r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) r[k] = s[min(i0 + k * BS, nv - 1)];  // clamped: every load in bounds
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + k * BS < nv) d[i0 + k * BS] = r[k];
  }
  const int tail = (int)((bytes & 15) >> 2);  // trailing 4-byte words
  if ((int)threadIdx.x < tail)
    reinterpret_cast<unsigned*>(d + nv)[threadIdx.x] = reinterpret_cast<const unsigned*>(s + nv)[threadIdx.x];
}

// Workgroup copy of rows x P elements from rows of stride Ps (global) into
// rows of stride P (LDS), eight loads in flight per thread.
template <int BS, typename T>
__device__ __forceinline__ void stage_rows(T* dst, const T* src, int rows, int P, int Ps) {
  const int ne = rows * P;
  for (int e0 = threadIdx.x; e0 < ne; e0 += 8 * BS) {
    T r[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = min(e0 + k * BS, ne - 1);  // clamped: every load in bounds
      const int row = e / P;
      r[k] = src[(int64_t)row * Ps + (e - row * P)];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int e = e0 + k * BS;
      if (e < ne) dst[e] = r[k];
    }
  }
}

// x*f for a set of flavours; see file header.  out is point-major [n][R].
// Each wave works on its own 64-point tiles with no workgroup barrier after
// the initial staging, so the knot searches and log transforms of some waves
// overlap the stencil gathers of others.  In-grid entries run a branch-free
// gather + FMA loop; the rare extrapolated points of a tile are finished
// afterwards, one point at a time across the wave.
constexpr int kWave = 64;

// Per-point record of phase 1, read back by the wave's own lanes in phase 2.
struct PointInfo {
  int boff;  // byte offset of the stencil origin f[sx][sq][0] in the member's values
  int sab;   // byte stride between consecutive x knots
  int mode;  // region bits (see locate_point)
  int pad;
};

__device__ constexpr AlphasDev kNoAlphas{};

// A point's record: weights and location side by side (80 bytes in FP64,
// 48 in FP32), so that the 9-16 different records one phase-2 load
// instruction reads fall in different LDS banks.
template <typename T>
struct PointRec {
  T w[4];
  T v[4];
  PointInfo info;
};

template <typename T>
__host__ __device__ constexpr size_t wave_record_bytes() {
  return (size_t)kWave * (sizeof(PointRec<T>) + 16);
}

// One wave's 64-point tile [pbeg, pbeg + tp): phase 1 (one lane per point,
// (xv, qv) = this lane's point) into the wave's LDS record, then the in-grid
// outputs, then the extrapolated points.  obase = output row of point pbeg.
//
// Phase 2 walks the tile's outputs with consecutive lanes on consecutive
// output addresses: one lane per (point, flavour) for a flavour subset
// (G = 1), or per (point, group of G stored columns) when every stored column
// is requested in order (G * sizeof(T) = 16 bytes).  Reading the grid from
// global memory, groups start at min(G*j, R - G): the last group of a point
// overlaps the one before it and every store is full width (the shared
// column gets the same value twice).  Reading it from LDS, groups start at
// G*j (16-byte aligned LDS reads; rows are zero-padded to a multiple of G)
// and the last group stores only the columns below R.
template <typename T, bool kLdsGrid, int G, bool kAlphas = false, bool kOverlap = !kLdsGrid, int kRowB = 0>
__device__ __forceinline__ void wave_tile(const MemberDev& m, const Tables& tb, const int* scol, int R,
                                          const T* sgrid, const T* __restrict__ gvals, uint32_t gbytes,
                                          double xv, double qv, int tp, T* __restrict__ obase,
                                          unsigned long long* __restrict__ nerr, double invL01,
                                          unsigned char* rec, int lane, const AlphasDev& A, const AsView& av) {
  PointRec<T>* srec = reinterpret_cast<PointRec<T>*>(rec);        // [64]
  double* sp = reinterpret_cast<double*>(srec + kWave);           // [64][2] extrapolation parameters
  const int Pp = sizeof(T) == 8 ? m.P64 : m.P32;
  // bytes between consecutive Q^2 knots; a compile-time kRowB (the caller has
  // checked it) lets the four Q^2 rows of an LDS gather use immediate offsets
  const int rowb = kRowB ? kRowB : Pp * (int)sizeof(T);
  constexpr int kSlow = kLowX | kLowQ | kHighQ;
  // lane -> (point, flavour) or (point, column group) walk of the tile's outputs
  const int NE = G == 1 ? R : (R + G - 1) / G;
  const int e_p0 = lane / NE, e_j0 = lane - (lane / NE) * NE;
  const int e_dp = kWave / NE, e_dj = kWave - (kWave / NE) * NE;
  if constexpr (kAlphas) {  // alpha_s at the same points (fused evaluation), counted like pdf_alphas_q2
    const bool qbad = lane < tp && !(qv > 0.0 && qv < INFINITY);
    if (lane < tp) av.out[lane] = alphas_point(A, av.k, av.v, av.c, av.h, qv);
    const unsigned long long qb = __ballot(qbad);
    if (qb && lane == 0) atomicAdd(nerr, (unsigned long long)__popcll(qb));
  }
  bool bad = false, slow = false;
  if (lane < tp) {
    T w[4], v[4];
    const PointLoc L = locate_point<T>(m, tb, xv, qv, w, v);
    bad = L.mode & kInvalid;
    slow = L.mode & kSlow;
    PointRec<T> r;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      r.w[a] = w[a];
      r.v[a] = v[a];
    }
    r.info = PointInfo{L.base * (int)sizeof(T), L.sa * (int)sizeof(T), L.mode, 0};
    srec[lane] = r;
    sp[2 * lane] = L.p0;
    sp[2 * lane + 1] = L.p1;
  }
  const unsigned long long bal = __ballot(bad);
  if (bal && lane == 0) atomicAdd(nerr, (unsigned long long)__popcll(bal));
  unsigned long long slow_mask = __ballot(slow);
  // records written by this wave are read back by other lanes of the same wave
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  const __amdgpu_buffer_rsrc_t gr = buffer_rsrc(gvals, gbytes);
  const __amdgpu_buffer_rsrc_t orr = buffer_rsrc(obase, (uint32_t)(tp * R * (int)sizeof(T)));
  const int nev = tp * NE;
  int p = e_p0, j = e_j0;
  for (int e = lane; e < nev; e += kWave) {
    const PointInfo pi = srec[p].info;
    if (!(pi.mode & kSlow)) {
      T w[4], v[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        w[a] = srec[p].w[a];
        v[a] = srec[p].v[a];
      }
      const bool inv = pi.mode & kInvalid;
      int c0;       // first output column of this entry
      int ccol;     // its stored column (-1: flavour absent from the grid)
      if constexpr (G == 1) {
        c0 = j;
        ccol = scol[j];
      } else {
        c0 = kOverlap ? min(G * j, R - G) : G * j;
        ccol = c0;
      }
      T res[G];
      if (inv) {
#pragma unroll
        for (int i = 0; i < G; ++i) res[i] = (T)NAN;
      } else if (G == 1 && ccol < 0) {
#pragma unroll
        for (int i = 0; i < G; ++i) res[i] = (T)0;
      } else {
        const int o0 = pi.boff + ccol * (int)sizeof(T);
        T F[G][4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int oa = o0 + a * pi.sab;
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            T q[G];
            if constexpr (kLdsGrid) {
              const T* s = reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(sgrid) + oa + b * rowb);
              if constexpr (G > 1) {
                using V = typename VecOf<T, G>::type;  // 16-byte aligned: groups start at multiples of G
                const V vq = *reinterpret_cast<const V*>(s);
                __builtin_memcpy(q, &vq, sizeof(V));
              } else {
                q[0] = s[0];
              }
            } else {
              buf_load<T, G>(gr, oa, b * rowb, q);
            }
#pragma unroll
            for (int i = 0; i < G; ++i) F[i][a][b] = q[i];
          }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) res[i] = interp_stencil<T>(F[i], w, v);
      }
      const int ob = (p * R + c0) * (int)sizeof(T);
      if (kOverlap || G * j + G <= R) {
        buf_store<T, G, kLdsGrid ? 0 : kStoreStream>(orr, ob, res);
      } else {
        // last group of a point without overlap: only the columns below R
        for (int i = 0; i < R - G * j; ++i)
          buf_store<T, 1, kLdsGrid ? 0 : kStoreStream>(orr, ob + i * (int)sizeof(T), res + i);
      }
    }
    p += e_dp;
    j += e_dj;
    if (j >= NE) {
      j -= NE;
      ++p;
    }
  }
  // extrapolated points of the tile, one at a time across the wave
  while (slow_mask) {
    const int q = __builtin_ctzll(slow_mask);
    slow_mask &= slow_mask - 1;
    const PointInfo pi = srec[q].info;
    const PointRec<T>& rq = srec[q];
    const Wts wt{(double)rq.w[0], (double)rq.w[1], (double)rq.w[2], (double)rq.w[3],
                 (double)rq.v[0], (double)rq.v[1], (double)rq.v[2], (double)rq.v[3]};
    for (int jj = lane; jj < R; jj += kWave) {
      const int col = G == 1 ? scol[jj] : jj;
      T val = (T)0;
      if (col >= 0) {
        const T* f = reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(kLdsGrid ? sgrid : gvals) +
                                                pi.boff) + col;
        val = (T)extrap_entry<T>(f, pi.sab / (int)sizeof(T), Pp, pi.mode, wt, sp[2 * q], sp[2 * q + 1], invL01);
      }
      obase[q * R + jj] = val;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#ifndef PDFMI_WAVES_PER_EU
#define PDFMI_WAVES_PER_EU 1
#endif

// LDS layout of k_xfxq2 and k_batched: [location tables][column map][per-wave
// records][grid values], the tables only when they are staged (kLdsTables)
// and the grid only when it is staged (kLdsGrid, which implies kLdsTables).
template <typename T, bool kLdsGrid, int G, int BS, bool kLdsTables, bool kAlphas>
__global__ __launch_bounds__(BS) __attribute__((amdgpu_waves_per_eu(kAlphas ? 4 : PDFMI_WAVES_PER_EU)))
void k_xfxq2(MemberDev m, ReqCols rc, const double* __restrict__ X, const double* __restrict__ Q2, int64_t n,
             T* __restrict__ out, unsigned long long* __restrict__ nerr, int lds_grid_elems, double invL01,
             AlphasDev A, double* __restrict__ aout) {
  static_assert(kLdsTables || !kLdsGrid, "a staged grid needs staged tables");
  constexpr int kWaves = BS / kWave;
  extern __shared__ __align__(16) unsigned char smem[];
  unsigned char* stbl = smem;
  int* scol = reinterpret_cast<int*>(smem + (kLdsTables ? m.tbl_bytes : 0));
  unsigned char* srec = reinterpret_cast<unsigned char*>(scol + kMaxReq);
  T* sgrid = reinterpret_cast<T*>(srec + kWaves * wave_record_bytes<T>());
  // alpha_s table (fused alpha_s output only), after the staged grid
  unsigned char* sas = reinterpret_cast<unsigned char*>(sgrid) + (kLdsGrid ? (size_t)lds_grid_elems * sizeof(T) : 0);
  const int an2 = (A.n + 1) & ~1;
  AsView av{reinterpret_cast<const double*>(sas), reinterpret_cast<const double*>(sas) + an2,
            reinterpret_cast<const CellCoef*>(reinterpret_cast<const double*>(sas) + 2 * an2),
            reinterpret_cast<const short*>(reinterpret_cast<const CellCoef*>(reinterpret_cast<const double*>(sas) +
                                                                               2 * an2) + an2),
            nullptr};
  if constexpr (kAlphas) {
    double* k = const_cast<double*>(av.k);
    double* v = const_cast<double*>(av.v);
    CellCoef* c = const_cast<CellCoef*>(av.c);
    short* h = const_cast<short*>(av.h);
    for (int i = threadIdx.x; i < A.n; i += BS) {
      k[i] = A.knots[i];
      v[i] = A.vals[i];
      c[i] = A.cells[i];
    }
    for (int i = threadIdx.x; i < A.nhints; i += BS) h[i] = A.hints[i];
  }

  if constexpr (kLdsTables) stage_copy<BS>(stbl, m.tables, m.tbl_bytes);
  for (int i = threadIdx.x; i < rc.n; i += BS) scol[i] = rc.col[i];
  const T* __restrict__ gvals = member_values<T>(m);
  const uint32_t gbytes = (uint32_t)((sizeof(T) == 8 ? m.elems64 : m.elems32) * (int64_t)sizeof(T));
  if constexpr (kLdsGrid) stage_copy<BS>(sgrid, gvals, (int64_t)lds_grid_elems * (int64_t)sizeof(T));
  __syncthreads();
  const Tables tb = kLdsTables ? tables_at(stbl, m) : Tables{m.knots, m.cells, m.hints, m.subs};

  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  unsigned char* rec = srec + wv * wave_record_bytes<T>();
  const int R = rc.n;
  const int64_t ntiles = (n + kWave - 1) / kWave;
  const int64_t stride = (int64_t)gridDim.x * kWaves;
  int64_t tile = (int64_t)blockIdx.x * kWaves + wv;
  // the next tile's (x, Q^2) are loaded before the current tile is processed
  double xc = 0.0, qc = 0.0;
  if (tile < ntiles && tile * kWave + lane < n) {
    xc = X[tile * kWave + lane];
    qc = Q2[tile * kWave + lane];
  }
  for (; tile < ntiles; tile += stride) {
    const int64_t pbeg = tile * kWave;
    const int tp = (int)min((int64_t)kWave, n - pbeg);
    const int64_t nxt = pbeg + stride * kWave + lane;
    double xn = 0.0, qn = 0.0;
    if (nxt < n) {
      xn = X[nxt];
      qn = Q2[nxt];
    }
    if constexpr (kAlphas) av.out = aout + pbeg;
    wave_tile<T, kLdsGrid, G, kAlphas>(m, tb, scol, R, sgrid, gvals, gbytes, xc, qc, tp, out + pbeg * R, nerr, invL01, rec,
                              lane, A, av);
    xc = xn;
    qc = qn;
  }
}

// Location only (sub-grid, cells, region), one lane per point.
__global__ __launch_bounds__(256) void k_locate(MemberDev m, const double* __restrict__ X,
                                                const double* __restrict__ Q2, int64_t n,
                                                int32_t* __restrict__ ko, int32_t* __restrict__ ixo,
                                                int32_t* __restrict__ iqo, int8_t* __restrict__ rego) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    double w[4], v[4];
    const PointLoc L = locate_point<double>(m, Tables{m.knots, m.cells, m.hints, m.subs}, X[i], Q2[i], w, v);
    ko[i] = L.k;
    ixo[i] = L.ix;
    iqo[i] = L.iq;
    rego[i] = (int8_t)(L.mode & (kLowX | kLowQ | kHighQ | kInvalid));
  }
}

// alpha_s(Q^2) (paper section 2.3): segment (repeated knot = threshold, the
// upper segment owns it), FP64 knot search, cubic Hermite in ln Q^2 with
// one-sided slopes at segment ends, constant outside the knots.  The table
// (knots, values, cell coefficients) is staged in LDS once per workgroup.
constexpr int kAlphasMaxKnots = 256;

// alpha_s(Q^2) at n points, the table and its search hints staged in LDS;
// four independent evaluations in flight per lane.
constexpr int kAlphasMaxHints = 2048;

__global__ __launch_bounds__(256) void k_alphas(AlphasDev A, const double* __restrict__ Q2, int64_t n,
                                                double* __restrict__ out, unsigned long long* __restrict__ nerr) {
  __shared__ double sk[kAlphasMaxKnots];
  __shared__ double sv[kAlphasMaxKnots];
  __shared__ CellCoef sc[kAlphasMaxKnots];
  __shared__ short sh[kAlphasMaxHints];
  for (int i = threadIdx.x; i < A.n; i += 256) {
    sk[i] = A.knots[i];
    sv[i] = A.vals[i];
    sc[i] = A.cells[i];
  }
  for (int i = threadIdx.x; i < A.nhints; i += 256) sh[i] = A.hints[i];
  __syncthreads();
  // each wave takes 256 consecutive points per step, lane l the points l + 64 j
  // (j = 0..3): every load and store instruction covers 512 contiguous bytes.
  // The next step's Q^2 are loaded before the current step is evaluated.
  const int lane = threadIdx.x & 63;
  const int64_t nchunks = (n + 255) / 256;
  const int64_t wstride = (int64_t)gridDim.x * (256 / 64);
  int64_t c = (int64_t)blockIdx.x * (256 / 64) + (threadIdx.x >> 6);
  double q[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int64_t i = c * 256 + j * 64 + lane;
    q[j] = i < n ? Q2[i] : 1.0;
  }
  unsigned long long cnt = 0;
  for (; c < nchunks; c += wstride) {
    double qn[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = (c + wstride) * 256 + j * 64 + lane;
      qn[j] = i < n ? Q2[i] : 1.0;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t i = c * 256 + j * 64 + lane;
      const double r = alphas_point(A, sk, sv, sc, sh, q[j]);
      if (i < n) out[i] = r;
      cnt += __popcll(__ballot(i < n && !(q[j] > 0.0 && q[j] < INFINITY)));
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = qn[j];
  }
  if (cnt && lane == 0) atomicAdd(nerr, cnt);
}

// ---------------------------------------------------------------------------------------
// Launchers (host side, called by pdfmi.cpp)

// Location tables up to this size are staged in LDS (typical sets need
// 10-40 KB: a few hundred knots of 8 bytes plus 48 bytes of coefficients per
// cell); larger ones are read from global memory.
constexpr size_t kMaxLdsTables = 56 * 1024;
static bool tables_fit(const MemberDev& m) { return (size_t)m.tbl_bytes <= kMaxLdsTables; }

// LDS bytes of the alpha_s table staged for a fused alpha_s output.
size_t alphas_lds_bytes(const AlphasDev* A) {
  if (!A) return 0;
  const size_t an2 = (size_t)((A->n + 1) & ~1);
  return an2 * (8 + 8 + sizeof(CellCoef)) + (size_t)A->nhints * 2;
}

// LDS bytes of k_xfxq2 other than the staged grid, for a block of bs threads.
static size_t shared_bytes(const MemberDev& m, bool f32, int bs, bool tables) {
  return (tables ? (size_t)m.tbl_bytes : 0) + kMaxReq * 4 +
         (bs / kWave) * (f32 ? wave_record_bytes<float>() : wave_record_bytes<double>());
}
constexpr int kBlockGlobal = 256;   // tables and grid read from global memory
// Below this many points each workgroup sees only a few tiles, and staging the
// whole location table (tens of KB) costs more than reading the few entries
// each point needs from global memory: the tables are then read in place
// (measured: 1e3 and 1e4 points 15-20 % faster; at 1e5 points staging wins).
constexpr int64_t kStageTablesMinPoints = 32768;
constexpr int kBlockTables = 512;   // tables staged in LDS, grid read from global memory
constexpr int kBlockLds = 1024;     // tables and grid staged once per workgroup in LDS
size_t xfxq2_shared_bytes(const MemberDev& m, bool f32) {
  return shared_bytes(m, f32, kBlockLds, true) + alphas_lds_bytes(nullptr);
}

// Launch context: the alpha_s table and output of a fused evaluation (A and
// aout null when alpha_s is not requested).
struct AsOut {
  const AlphasDev* A;
  double* aout;
};

template <typename T, int G, int BS, bool kLdsGrid, bool kLdsTables, bool kAlphas>
static hipError_t launch_one(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2, int64_t n,
                             T* out, unsigned long long* nerr, int lds_grid_elems, double invL01, int64_t nb,
                             size_t shm, const AsOut& ao, hipStream_t s) {
  const void* fn = reinterpret_cast<const void*>(&k_xfxq2<T, kLdsGrid, G, BS, kLdsTables, kAlphas>);
  hipError_t e = allow_dynamic_lds(fn, shm);
  if (e != hipSuccess) return e;
  const AlphasDev A = ao.A ? *ao.A : AlphasDev{};
  hipLaunchKernelGGL((k_xfxq2<T, kLdsGrid, G, BS, kLdsTables, kAlphas>), dim3((unsigned)nb), dim3(BS), shm, s, m, rc, x, q2,
                     n, out, nerr, lds_grid_elems, invL01, A, ao.aout);
  return hipGetLastError();
}

template <typename T, int G, bool kAlphas>
static hipError_t launch_xfxq2_g(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2,
                                 int64_t n, T* out, unsigned long long* nerr, int lds_grid_elems,
                                 double invL01, const LaunchCfg& cfg, const AsOut& ao, hipStream_t s) {
  const int n_cu = cfg.n_cu;
  const bool f32 = sizeof(T) == 4;
  const size_t as_bytes = alphas_lds_bytes(ao.A);
  if (lds_grid_elems > 0) {
    const size_t shm = shared_bytes(m, f32, kBlockLds, true) + (size_t)lds_grid_elems * sizeof(T) + as_bytes;
    const int per_cu = (int)(160 * 1024 / shm) > 0 ? (int)(160 * 1024 / shm) : 1;
    const int64_t ntiles = (n + kBlockLds - 1) / kBlockLds;
    const int64_t nb = min(ntiles, (int64_t)n_cu * per_cu);
    return launch_one<T, G, kBlockLds, true, true, kAlphas>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, nb, shm, ao,
                                                   s);
  }
  if (tables_fit(m) && n >= kStageTablesMinPoints) {
    const size_t shm = shared_bytes(m, f32, kBlockTables, true) + as_bytes;
    const int64_t ntiles = (n + kBlockTables - 1) / kBlockTables;
    const int64_t nb = min(ntiles, (int64_t)n_cu * cfg.blocks_per_cu);
    return launch_one<T, G, kBlockTables, false, true, kAlphas>(m, rc, x, q2, n, out, nerr, 0, invL01, nb, shm, ao, s);
  }
  const size_t shm = shared_bytes(m, f32, kBlockGlobal, false) + as_bytes;
  const int64_t ntiles = (n + kBlockGlobal - 1) / kBlockGlobal;
  const int64_t nb = min(ntiles, (int64_t)n_cu * cfg.blocks_per_cu);
  return launch_one<T, G, kBlockGlobal, false, false, kAlphas>(m, rc, x, q2, n, out, nerr, 0, invL01, nb, shm, ao, s);
}

// The vectorised kernel serves requests for every stored column in load order.
// Its groups of G columns need at least G of them.
static bool all_columns(const MemberDev& m, const ReqCols& rc, int G) {
  if (rc.n != m.P || rc.n < G) return false;
  for (int j = 0; j < rc.n; ++j)
    if (rc.col[j] != j) return false;
  return true;
}

// A, aout: the alpha_s table and output of a fused evaluation, or null.
hipError_t launch_xfxq2_f64(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2, int64_t n,
                            double* out, unsigned long long* nerr, int lds_grid_elems, double invL01,
                            const LaunchCfg& cfg, const AlphasDev* A, double* aout, hipStream_t s) {
  const AsOut ao{aout ? A : nullptr, aout};
  const bool vec = cfg.vector_cols && all_columns(m, rc, 2);
  if (aout)
    return vec ? launch_xfxq2_g<double, 2, true>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s)
               : launch_xfxq2_g<double, 1, true>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s);
  return vec ? launch_xfxq2_g<double, 2, false>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s)
             : launch_xfxq2_g<double, 1, false>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s);
}

hipError_t launch_xfxq2_f32(const MemberDev& m, const ReqCols& rc, const double* x, const double* q2, int64_t n,
                            float* out, unsigned long long* nerr, int lds_grid_elems, double invL01,
                            const LaunchCfg& cfg, const AlphasDev* A, double* aout, hipStream_t s) {
  const AsOut ao{aout ? A : nullptr, aout};
  const bool vec = cfg.vector_cols && all_columns(m, rc, 4);
  if (aout)
    return vec ? launch_xfxq2_g<float, 4, true>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s)
               : launch_xfxq2_g<float, 1, true>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s);
  return vec ? launch_xfxq2_g<float, 4, false>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s)
             : launch_xfxq2_g<float, 1, false>(m, rc, x, q2, n, out, nerr, lds_grid_elems, invL01, cfg, ao, s);
}

hipError_t launch_locate(const MemberDev& m, const double* x, const double* q2, int64_t n, int32_t* k, int32_t* ix,
                         int32_t* iq, int8_t* reg, int n_cu, hipStream_t s) {
  const int64_t nb = min((n + 255) / 256, (int64_t)n_cu * 16);
  hipLaunchKernelGGL(k_locate, dim3((unsigned)nb), dim3(256), 0, s, m, x, q2, n, k, ix, iq, reg);
  return hipGetLastError();
}

hipError_t launch_alphas(const AlphasDev& A, const double* q2, int64_t n, double* out, unsigned long long* nerr,
                         int n_cu, hipStream_t s) {
  const int64_t nb = min((n + 1023) / 1024, (int64_t)n_cu * 8);
  hipLaunchKernelGGL(k_alphas, dim3((unsigned)nb), dim3(256), 0, s, A, q2, n, out, nerr);
  return hipGetLastError();
}

}  // namespace pdfmi

namespace pdfmi {

// ---------------------------------------------------------------------------------------
// Monte-Carlo luminosity chunk sum (the integrand-shaped load of the paper's
// section 4.1): S = sum_i alpha_s(Q^2_i) * sum_j xf1[i][j] * xf2[i][j], FP64,
// in a fixed order that depends only on n: stage 1 gives one partial per
// block of kMcBlock points (each thread sums its strided points in index
// order, then a fixed binary tree in LDS); stage 2 sums the partials with the
// same tree in one workgroup.  Bit-identical across runs.
constexpr int kMcThreads = 256;
constexpr int kMcBlock = 1024;  // 4 points per thread: a 1e6-point chunk spans ~1000 blocks

__device__ __forceinline__ double block_tree_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = kMcThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// Stage 1 when the rows do not fit LDS (many flavours): the same order read
// straight from global memory.
template <typename T>
__global__ __launch_bounds__(kMcThreads) void k_mc_partial_direct(const T* __restrict__ xf1,
                                                                  const T* __restrict__ xf2, int P,
                                                                  const double* __restrict__ as, int64_t n,
                                                                  double* __restrict__ partial) {
  __shared__ double sh[kMcThreads];
  const int64_t beg = (int64_t)blockIdx.x * kMcBlock;
  const int64_t end = min(beg + kMcBlock, n);
  double acc = 0.0;
  for (int k = 0; k < kMcBlock / kMcThreads; ++k) {
    const int64_t i = beg + threadIdx.x + (int64_t)kMcThreads * k;
    if (i < end) {
      double lum = 0.0;
      for (int j = 0; j < P; ++j) lum = fma((double)xf1[i * P + j], (double)xf2[i * P + j], lum);
      acc = fma(as[i], lum, acc);
    }
  }
  const double s = block_tree_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// Stage 1.  The block's points are taken 256 at a time: their xf1 and xf2
// rows (contiguous in memory) are copied to LDS with coalesced loads, then
// thread t forms sum_j xf1 xf2 of its point in flavour order and accumulates
// alpha_s times it -- thread t sees points beg + t + 256 k in increasing k.
template <typename T>
__global__ __launch_bounds__(kMcThreads) void k_mc_partial(const T* __restrict__ xf1, const T* __restrict__ xf2,
                                                           int P, const double* __restrict__ as, int64_t n,
                                                           double* __restrict__ partial) {
  __shared__ double sh[kMcThreads];
  extern __shared__ __align__(16) unsigned char mc_smem[];
  T* s1 = reinterpret_cast<T*>(mc_smem);  // [256][P]
  T* s2 = s1 + kMcThreads * P;            // [256][P]
  const int64_t beg = (int64_t)blockIdx.x * kMcBlock;
  const int64_t end = min(beg + kMcBlock, n);
  double acc = 0.0;
  for (int k = 0; k < kMcBlock / kMcThreads; ++k) {
    const int64_t p0 = beg + (int64_t)kMcThreads * k;
    if (p0 >= end) break;  // uniform across the block
    const int np = (int)min((int64_t)kMcThreads, end - p0);
    __syncthreads();       // previous step's rows consumed
    for (int e = threadIdx.x; e < np * P; e += kMcThreads) {
      s1[e] = xf1[p0 * P + e];
      s2[e] = xf2[p0 * P + e];
    }
    __syncthreads();
    if ((int)threadIdx.x < np) {
      double lum = 0.0;
      for (int j = 0; j < P; ++j) lum = fma((double)s1[threadIdx.x * P + j], (double)s2[threadIdx.x * P + j], lum);
      acc = fma(as[p0 + threadIdx.x], lum, acc);
    }
  }
  const double s = block_tree_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(kMcThreads) void k_mc_final(const double* __restrict__ partial, int64_t np,
                                                         double* __restrict__ sum_out) {
  __shared__ double sh[kMcThreads];
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < np; i += kMcThreads) acc += partial[i];
  const double s = block_tree_sum(acc, sh);
  if (threadIdx.x == 0) *sum_out = s;
}

int64_t mc_partials(int64_t n) { return (n + kMcBlock - 1) / kMcBlock; }

template <typename T>
hipError_t launch_mc_sum(const T* xf1, const T* xf2, int P, const double* as, int64_t n, double* partial,
                         double* sum_out, hipStream_t s) {
  const int64_t np = mc_partials(n);
  if (np > 0) {
    const size_t shm = (size_t)2 * kMcThreads * P * sizeof(T);
    if (shm <= 96 * 1024) {
      hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_mc_partial<T>), shm);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_mc_partial<T>, dim3((unsigned)np), dim3(kMcThreads), shm, s, xf1, xf2, P, as, n, partial);
    } else {
      hipLaunchKernelGGL(k_mc_partial_direct<T>, dim3((unsigned)np), dim3(kMcThreads), 0, s, xf1, xf2, P, as, n,
                         partial);
    }
  }
  hipLaunchKernelGGL(k_mc_final, dim3(1), dim3(kMcThreads), 0, s, partial, np, sum_out);
  return hipGetLastError();
}
// Fused Monte-Carlo chunk sum: the same S as xfxq2(x1) + xfxq2(x2) +
// alpha_s + the chunk sum above, without writing the PDF values out (24 bytes
// of input per point instead of 24 + 2 R sizeof(T) out and back in).  Each
// 256-thread quarter of a workgroup takes one kMcBlock-point block of the
// chunk, each thread its points beg + t + 256 k in increasing k: one lane per
// point locates x1 and x2, evaluates every requested flavour of both with the
// same device functions as k_xfxq2, forms sum_j xf1_j xf2_j in flavour order
// and accumulates alpha_s times it -- the summation order of k_mc_partial, so
// both paths give bit-identical sums.  The grid is staged in LDS when it
// fits (kLdsGrid), else read from global memory.  In FP32 the LDS rows are
// padded with zeros to a multiple of kGW = 4 columns when that fits too, and
// the stencils are then read four columns at a time: one 16-byte LDS read
// brings four columns of a stencil row (a random-row gather of 16-byte reads
// delivers 2.3x the values per clock of 4-byte reads).  The flavour loop then
// walks a list of column-group steps built once per workgroup from the
// request: a step reads one group and applies the terms of the next 1..kGW
// requested flavours whose columns fall in it, in request order, so the sum
// is still formed flavour by flavour in that order; a flavour absent from the
// grid is a step of its own with no read.  Otherwise the rows keep stride P
// and each requested column is read on its own (kGW = 1), as in FP64: pairs
// of FP64 columns measured no faster than single 8-byte reads (with rows of
// 12 columns every stencil row starts on a 32-byte boundary and the reads of
// one instruction use half of the banks; padding the x stride by 16 bytes
// against that brought the pairs level with single reads, not below).
constexpr int kMcFusedBS = 4 * kMcThreads;
constexpr int kStepAbsent = -1;   // a step whose flavour is absent from the grid
constexpr int kStepOrdered = 1 << 19;  // the step's terms are the group's columns 0, 1, ... in order

// Column-group steps of a request (see above) into st[1..], their count into st[0].
// Step: group's first column (bits 0-15), term count (16-18), kStepOrdered,
// and the column within the group of term t in bits 20 + 2t, 21 + 2t.
template <int kGW>
__device__ __forceinline__ void mc_build_steps(const ReqCols& rc, int* st) {
  int ns = 0;
  for (int j = 0; j < rc.n;) {
    const int c = rc.col[j];
    if (c < 0) {
      st[1 + ns++] = kStepAbsent;
      ++j;
      continue;
    }
    const int g0 = c & ~(kGW - 1);
    int nt = 1, sel = c - g0;
    bool ordered = c == g0;
    while (nt < kGW && j + nt < rc.n && rc.col[j + nt] >= 0 && (rc.col[j + nt] & ~(kGW - 1)) == g0) {
      sel |= (rc.col[j + nt] - g0) << (2 * nt);
      ordered = ordered && rc.col[j + nt] - g0 == nt;
      ++nt;
    }
    st[1 + ns++] = g0 | (nt << 16) | (ordered ? kStepOrdered : 0) | (sel << 20);
    j += nt;
  }
  st[0] = ns;
}

// Element e (uniform) of a kGW-array of values held in registers.
template <typename T, int kGW>
__device__ __forceinline__ T mc_pick(const T (&f)[kGW], int e) {
  if constexpr (kGW == 1) {
    return f[0];
  } else if constexpr (kGW == 2) {
    return e ? f[1] : f[0];
  } else {
    static_assert(kGW == 4, "column groups of 2 or 4");
    return e == 0 ? f[0] : (e == 1 ? f[1] : (e == 2 ? f[2] : f[3]));
  }
}

// One flavour of one located point, the value k_xfxq2 writes for it: NaN for
// an invalid point, 0 for a flavour absent from the grid, the stencil sum
// inside the grid, the extrapolation formula outside.  g points at the
// stencil origin's entry of the flavour's column; sa, P are the x and Q^2
// strides of the values read.
template <typename T, bool kMaySlow>
__device__ __forceinline__ T mc_value(const T* g, const PointLoc& L, const T w[4], const T v[4], int sa, int P,
                                      int col, double invL01) {
  if (L.mode & kInvalid) return (T)NAN;
  if (col < 0) return (T)0;
  if (!kMaySlow || !(L.mode & (kLowX | kLowQ | kHighQ))) {
    T F[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) F[a][b] = g[a * sa + b * P];
    return interp_stencil<T>(F, w, v);
  }
  const Wts wt{(double)w[0], (double)w[1], (double)w[2], (double)w[3],
               (double)v[0], (double)v[1], (double)v[2], (double)v[3]};
  return (T)extrap_entry<T>(g, sa, P, L.mode, wt, L.p0, L.p1, invL01);
}

// Location of a point in the values read by k_mc_fused: element offset of
// the stencil origin and stride between x knots (Q^2 stride P).
__device__ __forceinline__ void mc_origin(const Tables& tb, const int* soff, const PointLoc& L, int P, int& base,
                                          int& sa) {
  const int k = max(L.k, 0);
  const int nqp = tb.subs[k].nqp;
  sa = nqp * P;
  base = soff[k] + (L.sx * nqp + L.sq) * P;
}

template <typename T, bool kLdsGrid, int kGW>
__global__ __launch_bounds__(kMcFusedBS) void k_mc_fused(MemberDev m, ReqCols rc, AlphasDev A,
                                                         const double* __restrict__ X1,
                                                         const double* __restrict__ X2,
                                                         const double* __restrict__ Q2, int64_t n,
                                                         double* __restrict__ partial,
                                                         unsigned long long* __restrict__ nerr, double invL01) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int an2 = (A.n + 1) & ~1;
  unsigned char* stbl = smem;
  double* ask = reinterpret_cast<double*>(smem + m.tbl_bytes);
  double* asv = ask + an2;
  CellCoef* asc = reinterpret_cast<CellCoef*>(asv + an2);
  short* ash = reinterpret_cast<short*>(asc + an2);          // [A.nhints, padded to 8]
  double* tree = reinterpret_cast<double*>(ash + ((A.nhints + 7) & ~7));  // [4][256]
  int* scol = reinterpret_cast<int*>(tree + kMcFusedBS);  // [kMaxReq]
  int* soff = scol + kMaxReq;                             // [kMaxSub] staged sub-grid offsets
  int* sstep = soff + kMaxSub;                            // [kMaxReq + 4] column-group steps (kGW > 1)
  T* sgrid = reinterpret_cast<T*>(sstep + kMaxReq + 4);   // 16-byte aligned: 2 kMaxReq + kMaxSub + 4 ints

  stage_copy<kMcFusedBS>(stbl, m.tables, m.tbl_bytes);
  for (int i = threadIdx.x; i < A.n; i += kMcFusedBS) {
    ask[i] = A.knots[i];
    asv[i] = A.vals[i];
    asc[i] = A.cells[i];
  }
  for (int i = threadIdx.x; i < A.nhints; i += kMcFusedBS) ash[i] = A.hints[i];
  for (int i = threadIdx.x; i < rc.n; i += kMcFusedBS) scol[i] = rc.col[i];
  const int Pp = sizeof(T) == 8 ? m.P64 : m.P32;
  const T* __restrict__ gvals = member_values<T>(m);
  // row stride of the values read below: in LDS P, or P rounded up to whole
  // column groups (<= Pp, whose padding columns are zero in global memory)
  const int P = kLdsGrid ? (m.P + kGW - 1) & ~(kGW - 1) : Pp;
  if (threadIdx.x == 0) {
    int off = 0;
    for (int k = 0; k < m.K; ++k) {
      soff[k] = kLdsGrid ? off : (int)(sizeof(T) == 8 ? m.sub[k].val_off64 : m.sub[k].val_off32);
      off += m.sub[k].nxp * m.sub[k].nqp * P;
    }
    if constexpr (kGW > 1) mc_build_steps<kGW>(rc, sstep);
  }
  if constexpr (kLdsGrid) {
    int off = 0;
    for (int k = 0; k < m.K; ++k) {
      const SubDesc& S = m.sub[k];
      const int rows = S.nxp * S.nqp;
      stage_rows<kMcFusedBS>(sgrid + off, gvals + (sizeof(T) == 8 ? S.val_off64 : S.val_off32), rows, P, Pp);
      off += rows * P;
    }
  }
  __syncthreads();
  const Tables tb = tables_at(stbl, m);
  const T* grid = kLdsGrid ? sgrid : gvals;

  const int q = threadIdx.x / kMcThreads, t = threadIdx.x % kMcThreads;
  const int R = rc.n;
  const int64_t nmb = (n + kMcBlock - 1) / kMcBlock;
  for (int64_t mb0 = (int64_t)blockIdx.x * 4; mb0 < nmb; mb0 += (int64_t)gridDim.x * 4) {
    const int64_t mb = mb0 + q;
    const int64_t beg = mb * kMcBlock, end = min(beg + (int64_t)kMcBlock, n);
    double acc = 0.0;
    for (int k = 0; k < kMcBlock / kMcThreads; ++k) {
      const int64_t i = beg + t + (int64_t)kMcThreads * k;
      const bool live = mb < nmb && i < end;
      double x1 = 0.5, x2 = 0.5, q2 = 10.0;
      if (live) {
        x1 = X1[i];
        x2 = X2[i];
        q2 = Q2[i];
      }
      // Q^2 weights: the shared location's.  locate_x copies them for a valid
      // point (and zeros them for an invalid one, whose value is NaN before
      // any weight is read), so both lookups read them from Qs.
      T w1[4], w2[4], vx[4];
      const QLoc<T> Qs = locate_q<T>(m, tb, q2);  // shared Q^2: located once for both lookups
      const PointLoc L1 = locate_x<T>(m, tb, Qs, x1, w1, vx);
      const PointLoc L2 = locate_x<T>(m, tb, Qs, x2, w2, vx);
      const T* v = Qs.v;
      const double as = alphas_point(A, ask, asv, asc, ash, q2);
      const bool bad1 = live && (L1.mode & kInvalid), bad2 = live && (L2.mode & kInvalid);
      const bool bada = live && !(q2 > 0.0 && q2 < INFINITY);
      const unsigned long long nb = __popcll(__ballot(bad1)) + __popcll(__ballot(bad2)) + __popcll(__ballot(bada));
      if (nb && (threadIdx.x & 63) == 0) atomicAdd(nerr, nb);
      int b1, sa1, b2, sa2;
      mc_origin(tb, soff, L1, P, b1, sa1);
      mc_origin(tb, soff, L2, P, b2, sa2);
      double lum = 0.0;
      if (kLdsGrid && kGW > 1 && !((L1.mode | L2.mode) & (kLowX | kLowQ | kHighQ))) {
        // both lookups inside the LDS-staged grid, read a column group at a
        // time: per step, the kGW values of each lookup that mc_value gives
        // for the group's columns, then the step's terms in request order
        using V = typename VecOf<T, kGW>::type;
        const bool inv1 = L1.mode & kInvalid, inv2 = L2.mode & kInvalid;
        const int ns = __builtin_amdgcn_readfirstlane(sstep[0]);
        for (int s = 0; s < ns; ++s) {
          const int st = __builtin_amdgcn_readfirstlane(sstep[1 + s]);
          if (st == kStepAbsent) {
            const T f1 = inv1 ? (T)NAN : (T)0, f2 = inv2 ? (T)NAN : (T)0;
            lum = fma((double)f1, (double)f2, lum);
            continue;
          }
          const T* g1 = grid + b1 + (st & 0xFFFF);
          const T* g2 = grid + b2 + (st & 0xFFFF);
          // the stencils Q^2 row by Q^2 row (interp_stencil's steps): one
          // row's reads of both lookups in flight at a time
          T f1[kGW], f2[kGW];
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            T u1[4][kGW], u2[4][kGW];
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              const V q1 = *reinterpret_cast<const V*>(g1 + a * sa1 + b * P);
              const V q2v = *reinterpret_cast<const V*>(g2 + a * sa2 + b * P);
              __builtin_memcpy(u1[a], &q1, sizeof(V));
              __builtin_memcpy(u2[a], &q2v, sizeof(V));
            }
#pragma unroll
            for (int i = 0; i < kGW; ++i) {
              f1[i] = stencil_step<T>(b, f1[i], u1[0][i], u1[1][i], u1[2][i], u1[3][i], w1, v);
              f2[i] = stencil_step<T>(b, f2[i], u2[0][i], u2[1][i], u2[2][i], u2[3][i], w2, v);
            }
          }
#pragma unroll
          for (int i = 0; i < kGW; ++i) {
            f1[i] = inv1 ? (T)NAN : f1[i];
            f2[i] = inv2 ? (T)NAN : f2[i];
          }
          const int nt = (st >> 16) & 7;
          if (st & kStepOrdered) {
#pragma unroll
            for (int t = 0; t < kGW; ++t)
              if (t < nt) lum = fma((double)f1[t], (double)f2[t], lum);
          } else {
#pragma unroll
            for (int t = 0; t < kGW; ++t)
              if (t < nt) {
                const int e = (st >> (20 + 2 * t)) & 3;
                lum = fma((double)mc_pick<T, kGW>(f1, e), (double)mc_pick<T, kGW>(f2, e), lum);
              }
          }
        }
      } else if (kLdsGrid && kGW == 1 && !((L1.mode | L2.mode) & (kLowX | kLowQ | kHighQ))) {
        // both lookups inside the LDS-staged grid: the values mc_value gives,
        // with both stencils' reads issued together and no branch per point
        // (an invalid point reads the in-bounds stencil at offset 0 and takes
        // NaN); from global memory the 32 loads in flight would spill
        const bool inv1 = L1.mode & kInvalid, inv2 = L2.mode & kInvalid;
        for (int j = 0; j < R; ++j) {
          const int col = __builtin_amdgcn_readfirstlane(scol[j]);
          T f1 = (T)0, f2 = (T)0;
          if (col >= 0) {
            T F1[4][4], F2[4][4];
            const T* g1 = grid + b1 + col;
            const T* g2 = grid + b2 + col;
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) {
                F1[a][b] = g1[a * sa1 + b * P];
                F2[a][b] = g2[a * sa2 + b * P];
              }
            f1 = interp_stencil<T>(F1, w1, v);
            f2 = interp_stencil<T>(F2, w2, v);
          }
          f1 = inv1 ? (T)NAN : f1;
          f2 = inv2 ? (T)NAN : f2;
          lum = fma((double)f1, (double)f2, lum);
        }
      } else if (!((L1.mode | L2.mode) & (kLowX | kLowQ | kHighQ))) {
        for (int j = 0; j < R; ++j) {
          const int col = scol[j];
          const T f1 = mc_value<T, false>(grid + b1 + col, L1, w1, v, sa1, P, col, invL01);
          const T f2 = mc_value<T, false>(grid + b2 + col, L2, w2, v, sa2, P, col, invL01);
          lum = fma((double)f1, (double)f2, lum);
        }
      } else {
        // at least one side extrapolated (rare): the same loop with the
        // extrapolation formulas
        for (int j = 0; j < R; ++j) {
          const int col = scol[j];
          const T f1 = mc_value<T, true>(grid + b1 + col, L1, w1, v, sa1, P, col, invL01);
          const T f2 = mc_value<T, true>(grid + b2 + col, L2, w2, v, sa2, P, col, invL01);
          lum = fma((double)f1, (double)f2, lum);
        }
      }
      if (live) acc = fma(as, lum, acc);
    }
    // the tree of block_tree_sum, per quarter
    double* sh = tree + q * kMcThreads;
    sh[t] = acc;
    __syncthreads();
    for (int st = kMcThreads / 2; st > 0; st >>= 1) {
      if (t < st) sh[t] += sh[t + st];
      __syncthreads();
    }
    if (t == 0 && mb < nmb) partial[mb] = sh[0];
    __syncthreads();
  }
}

// LDS bytes of k_mc_fused (grid_elems > 0: the grid staged with row stride P).
size_t mc_fused_shared_bytes(const MemberDev& m, const AlphasDev& A, int64_t grid_elems, bool f32) {
  const size_t an2 = (size_t)((A.n + 1) & ~1);
  return (size_t)m.tbl_bytes + an2 * (8 + 8 + sizeof(CellCoef)) + (size_t)((A.nhints + 7) & ~7) * 2 +
         kMcFusedBS * 8 + (2 * kMaxReq + kMaxSub + 4) * 4 +
         (size_t)grid_elems * (f32 ? 4 : 8);
}

template <typename T>
hipError_t launch_mc_fused(const MemberDev& m, const ReqCols& rc, const AlphasDev& A, const double* x1,
                           const double* x2, const double* q2, int64_t n, double* partial, double* sum_out,
                           unsigned long long* nerr, double invL01, int n_cu, hipStream_t s) {
  const int64_t np = mc_partials(n);
  if (np > 0) {
    constexpr int kGW = sizeof(T) == 4 ? 4 : 1;  // column groups in FP32 only
    const int Pg = (m.P + kGW - 1) & ~(kGW - 1);
    int64_t rows = 0;
    for (int k = 0; k < m.K; ++k) rows += (int64_t)m.sub[k].nxp * m.sub[k].nqp;
    const bool f32 = sizeof(T) == 4;
    // grid in LDS in column groups, else in LDS with stride P, else in global memory
    const size_t lds_g = mc_fused_shared_bytes(m, A, rows * Pg, f32);
    const size_t lds_1 = mc_fused_shared_bytes(m, A, rows * m.P, f32);
    const int mode = kGW > 1 && lds_g <= 160 * 1024 ? 2 : (lds_1 <= 160 * 1024 ? 1 : 0);
    const size_t shm = mode == 2 ? lds_g : (mode == 1 ? lds_1 : mc_fused_shared_bytes(m, A, 0, f32));
    const void* fn = mode == 2   ? reinterpret_cast<const void*>(&k_mc_fused<T, true, kGW>)
                     : mode == 1 ? reinterpret_cast<const void*>(&k_mc_fused<T, true, 1>)
                                 : reinterpret_cast<const void*>(&k_mc_fused<T, false, 1>);
    hipError_t e = allow_dynamic_lds(fn, shm);
    if (e != hipSuccess) return e;
    const int per_cu = max(1, (int)(160 * 1024 / shm));
    const int64_t nb = min((np + 3) / 4, (int64_t)n_cu * per_cu);
    if (mode == 2)
      hipLaunchKernelGGL((k_mc_fused<T, true, kGW>), dim3((unsigned)nb), dim3(kMcFusedBS), shm, s, m, rc, A, x1, x2,
                         q2, n, partial, nerr, invL01);
    else if (mode == 1)
      hipLaunchKernelGGL((k_mc_fused<T, true, 1>), dim3((unsigned)nb), dim3(kMcFusedBS), shm, s, m, rc, A, x1, x2,
                         q2, n, partial, nerr, invL01);
    else
      hipLaunchKernelGGL((k_mc_fused<T, false, 1>), dim3((unsigned)nb), dim3(kMcFusedBS), shm, s, m, rc, A, x1, x2,
                         q2, n, partial, nerr, invL01);
  }
  hipLaunchKernelGGL(k_mc_final, dim3(1), dim3(kMcThreads), 0, s, partial, np, sum_out);
  return hipGetLastError();
}
template hipError_t launch_mc_fused<double>(const MemberDev&, const ReqCols&, const AlphasDev&, const double*,
                                            const double*, const double*, int64_t, double*, double*,
                                            unsigned long long*, double, int, hipStream_t);
template hipError_t launch_mc_fused<float>(const MemberDev&, const ReqCols&, const AlphasDev&, const double*,
                                           const double*, const double*, int64_t, double*, double*,
                                           unsigned long long*, double, int, hipStream_t);

template hipError_t launch_mc_sum<double>(const double*, const double*, int, const double*, int64_t, double*, double*,
                                          hipStream_t);
template hipError_t launch_mc_sum<float>(const float*, const float*, int, const double*, int64_t, double*, double*,
                                         hipStream_t);

}  // namespace pdfmi

namespace pdfmi {

// ---------------------------------------------------------------------------------------
// Batched evaluation of many requests over many members (the paper's
// multi-member evaluation of section 4.3): one persistent launch in which
// each workgroup repeatedly takes the next tile from a global counter,
// stages that tile's member grid (and knots) in LDS when it differs from the
// one already staged, and runs the same per-wave tile pipeline as k_xfxq2.
// Every wave reaches the exit once the counter passes the tile count.
constexpr int kBatchBS = 1024;

__global__ void k_batch_reset(unsigned* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0u;
}

template <typename T, bool kLdsGrid, bool kLdsTables>
__global__ __launch_bounds__(kBatchBS) void k_batched(const BatchReq* __restrict__ reqs, const int* __restrict__ cols,
                                                      const BatchTile* __restrict__ tiles, int ntiles,
                                                      const MemberDev* __restrict__ members,
                                                      const double* __restrict__ invL01s, unsigned* counter,
                                                      unsigned long long* __restrict__ nerr, int max_tbl,
                                                      int vector_cols) {
  static_assert(kLdsTables || !kLdsGrid, "a staged grid needs staged tables");
  constexpr int kWaves = kBatchBS / kWave;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int s_tile, s_member;
  unsigned char* stbl = smem;                                              // [max_tbl] if staged
  int* scol = reinterpret_cast<int*>(smem + (kLdsTables ? max_tbl : 0));  // [kMaxReq]
  unsigned char* srec = reinterpret_cast<unsigned char*>(scol + kMaxReq);  // per-wave records
  T* sgrid = reinterpret_cast<T*>(srec + kWaves * wave_record_bytes<T>());
  const int lane = threadIdx.x & (kWave - 1);
  const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  unsigned char* rec = srec + wv * wave_record_bytes<T>();
  if (threadIdx.x == 0) s_member = -1;
  for (;;) {
    __syncthreads();  // previous tile finished by every wave before the LDS is reused
    if (threadIdx.x == 0) s_tile = (int)atomicAdd(counter, 1u);
    __syncthreads();
    const int t = __builtin_amdgcn_readfirstlane(s_tile);
    if (t >= ntiles) break;
    const BatchTile tl = tiles[t];
    const BatchReq rq = reqs[tl.req];
    const MemberDev& m = members[rq.member];
    const T* __restrict__ gvals = member_values<T>(m);
    const uint32_t gbytes = (uint32_t)((sizeof(T) == 8 ? m.elems64 : m.elems32) * (int64_t)sizeof(T));
    if (rq.member != s_member) {
      if constexpr (kLdsTables) stage_copy<kBatchBS>(stbl, m.tables, m.tbl_bytes);
      if constexpr (kLdsGrid) stage_copy<kBatchBS>(sgrid, gvals, (int64_t)gbytes);
    }
    for (int i = threadIdx.x; i < rq.R; i += kBatchBS) scol[i] = cols[rq.col_off + i];
    __syncthreads();
    if (threadIdx.x == 0) s_member = rq.member;
    const Tables tb = kLdsTables ? tables_at(stbl, m) : Tables{m.knots, m.cells, m.hints, m.subs};
    const double invL01 = invL01s[rq.member];
    T* out = reinterpret_cast<T*>(rq.out);
    for (int w0 = wv * kWave; w0 < tl.count; w0 += kWaves * kWave) {
      const int64_t pbeg = tl.start + w0;
      const int tp = min(kWave, tl.count - w0);
      constexpr int G = 16 / sizeof(T);
      const double xv = lane < tp ? rq.x[pbeg + lane] : 0.0;
      const double qv = lane < tp ? rq.q2[pbeg + lane] : 0.0;
      if (vector_cols && rq.all_cols && rq.R >= G)
        wave_tile<T, kLdsGrid, G>(m, tb, scol, rq.R, sgrid, gvals, gbytes, xv, qv, tp, out + pbeg * rq.R, nerr,
                                  invL01, rec, lane, kNoAlphas, AsView{});
      else if (kLdsGrid && sizeof(T) == 4 && m.P32 == 12)  // 9-12 stored flavours in FP32: 48-byte rows
        wave_tile<T, kLdsGrid, 1, false, !kLdsGrid, 48>(m, tb, scol, rq.R, sgrid, gvals, gbytes, xv, qv, tp,
                                                        out + pbeg * rq.R, nerr, invL01, rec, lane, kNoAlphas,
                                                        AsView{});
      else
        wave_tile<T, kLdsGrid, 1>(m, tb, scol, rq.R, sgrid, gvals, gbytes, xv, qv, tp, out + pbeg * rq.R, nerr,
                                  invL01, rec, lane, kNoAlphas, AsView{});
    }
  }
}

// Location tables are staged when the largest member's fit (always when the
// grid is staged too).
static bool batch_tables(bool lds, int max_tbl) { return lds || (size_t)max_tbl <= kMaxLdsTables; }

size_t batch_shared_bytes(int max_tbl, bool f32, bool lds) {
  return (batch_tables(lds, max_tbl) ? (size_t)max_tbl : 0) + kMaxReq * 4 +
         (kBatchBS / kWave) * (f32 ? wave_record_bytes<float>() : wave_record_bytes<double>());
}

// Kernel node parameters of one batched run: the counter reset and the
// persistent kernel (used for direct launches and for building a hipGraph).

template <typename T>
static const void* batch_fn(bool lds, bool tables) {
  if (lds) return reinterpret_cast<const void*>(&k_batched<T, true, true>);
  return tables ? reinterpret_cast<const void*>(&k_batched<T, false, true>)
                : reinterpret_cast<const void*>(&k_batched<T, false, false>);
}

BatchLaunch batch_launch_params(bool f32, bool lds, int max_tbl, int64_t max_elems, int n_cu, int blocks_per_cu,
                                int ntiles) {
  BatchLaunch L{};
  L.reset_fn = reinterpret_cast<const void*>(&k_batch_reset);
  L.shm = batch_shared_bytes(max_tbl, f32, lds) + (lds ? (size_t)max_elems * (f32 ? 4 : 8) : 0);
  const bool tables = batch_tables(lds, max_tbl);
  L.main_fn = f32 ? batch_fn<float>(lds, tables) : batch_fn<double>(lds, tables);
  const int64_t g = min((int64_t)ntiles, (int64_t)n_cu * blocks_per_cu);
  L.grid = (unsigned)max((int64_t)1, g);
  return L;
}

hipError_t batch_prepare(const BatchLaunch& L) {
  return allow_dynamic_lds(L.main_fn, L.shm);
}

hipError_t batch_launch(const BatchLaunch& L, void** args, unsigned* counter, hipStream_t s) {
  void* rargs[] = {&counter};
  hipError_t e = hipLaunchKernel(L.reset_fn, dim3(1), dim3(64), rargs, 0, s);
  if (e != hipSuccess) return e;
  return hipLaunchKernel(L.main_fn, dim3(L.grid), dim3(kBatchBS), args, L.shm, s);
}

}  // namespace pdfmi
