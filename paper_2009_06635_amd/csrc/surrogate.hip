// MLP surrogate of one member's PDFs (growth path of the interpolation
// library): (ln x, ln Q^2) -> all stored flavours, 2 -> 64 -> 64 -> 64 -> 16
// (outputs beyond the stored columns are padding), tanh hidden activations,
// BF16 weights and activations with FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x32_bf16), FP32 master weights, Adam.
//
// The network predicts y_c = xf_c / E_c(x), where E_c is a positive envelope
// of the grid (largest |xf_c| over Q^2 at each x knot, linear in ln x between
// knots), so every target is O(1).  Inference falls back to the FP32
// interpolator outside the grid and in the first/last x or Q^2 cell of a
// sub-grid (which includes the cells next to flavour thresholds).
//
// Training is deterministic: every reduction has a fixed order (one wave per
// 16x16 output tile loops over the whole batch; bias sums are sequential per
// column), so a checkpointed and resumed run reproduces a straight run bit for
// bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "interp_dev.h"
#include "pdfmi_dev.h"

namespace pdfmi {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kH = 64;   // hidden width
constexpr int kO = 16;   // output width (stored columns padded)
// flat FP32 parameter layout
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kH * 2, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kH, kOffW4 = kOffB3 + kH, kOffB4 = kOffW4 + kO * kH,
              kNParams = kOffB4 + kO;

__device__ __forceinline__ unsigned short bf16_bits(float f) {
  const __bf16 h = (__bf16)f;  // round to nearest even
  return __builtin_bit_cast(unsigned short, h);
}
__device__ __forceinline__ float bf16_float(unsigned short b) {
  return __uint_as_float(((unsigned)b) << 16);
}

// tanh(z) = 1 - 2 / (exp(2z) + 1) from the hardware exp2 and reciprocal:
// exp2 overflows to +inf (result 1) and underflows to 0 (result -1); near 0
// the absolute error is a few 1e-8, far below the BF16 rounding of the
// activations.
constexpr float kTwoLog2e = 2.8853900817779268f;  // 2 log2(e)
// tanh(z) from zs = 2 log2(e) z (inference folds the factor into its weights and biases)
__device__ __forceinline__ float tanh_scaled(float zs) {
  return fmaf(-2.0f, __builtin_amdgcn_rcpf(__builtin_amdgcn_exp2f(zs) + 1.0f), 1.0f);
}
__device__ __forceinline__ float tanh_f(float z) { return tanh_scaled(kTwoLog2e * z); }

// ---------------------------------------------------------------------------------------
// Generic BF16 GEMM tile: C[m][n] = sum_k A(m,k) B(k,n) (+ bias[n]) (then tanh)
// A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn] (BF16 bit patterns);
// M, N multiples of 16; K any (zero padded to 32).  One wave per 16x16 tile,
// K walked in order (fixed summation order).  Writes FP32 C (ldc) and, if
// Cb != null, its BF16 copy.
// With gridDim.y > 1 workgroup y covers k in [y kchunk, (y + 1) kchunk) and
// writes its partial tile to C + y M ldc (the slices are added in order by
// k_sum_slices); bias and activation then belong to the unsplit form only.
__global__ __launch_bounds__(64) void k_gemm_bf16(const unsigned short* __restrict__ A, int sam, int sak,
                                                  const unsigned short* __restrict__ B, int sbk, int sbn,
                                                  float* __restrict__ C, int ldc, unsigned short* __restrict__ Cb,
                                                  int M, int N, int K, const float* __restrict__ bias, int act,
                                                  int kchunk) {
  const int tn = N / 16;
  const int m0 = (blockIdx.x / tn) * 16, n0 = (blockIdx.x % tn) * 16;
  const int l = threadIdx.x, r = l & 15, g = l >> 4;
  const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  C += (int64_t)blockIdx.y * M * ldc;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    bf16x8 a, b;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + 8 * g + i;
      const unsigned short av = k < ke ? A[(int64_t)(m0 + r) * sam + (int64_t)k * sak] : (unsigned short)0;
      const unsigned short bv = k < ke ? B[(int64_t)k * sbk + (int64_t)(n0 + r) * sbn] : (unsigned short)0;
      a[i] = __builtin_bit_cast(__bf16, av);
      b[i] = __builtin_bit_cast(__bf16, bv);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * g + i, n = n0 + r;
    float v = acc[i];
    if (bias) v += bias[n];
    if (act) v = tanh_f(v);
    C[(int64_t)m * ldc + n] = v;
    if (Cb) Cb[(int64_t)m * ldc + n] = bf16_bits(v);
  }
}

// Layer 1 (K = 2, on the vector ALUs): h1 = tanh(W1 in + b1), FP32 and BF16.
__global__ void k_layer1(const float* __restrict__ in, const float* __restrict__ P, int B, float* __restrict__ h,
                         unsigned short* __restrict__ hb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * kH) return;
  const int b = (int)(i / kH), j = (int)(i % kH);
  // the inputs and W1 are BF16-rounded like every other matrix operand
  const float u = bf16_float(bf16_bits(in[2 * b])), v = bf16_float(bf16_bits(in[2 * b + 1]));
  const float w0 = bf16_float(bf16_bits(P[kOffW1 + 2 * j])), w1 = bf16_float(bf16_bits(P[kOffW1 + 2 * j + 1]));
  const float z = fmaf(w0, u, fmaf(w1, v, P[kOffB1 + j]));
  const float t = tanh_f(z);
  h[i] = t;
  hb[i] = bf16_bits(t);
}

// Loss (mean squared error over B x kO) and its gradient dY = 2 (Y - T) / (B kO).
__global__ void k_loss_grad(const float* __restrict__ Y, const float* __restrict__ T, int B, float* __restrict__ dY,
                            unsigned short* __restrict__ dYb, float* __restrict__ sq) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * kO) return;
  const float d = Y[i] - T[i];
  const float gr = 2.0f * d / (float)((int64_t)B * kO);
  dY[i] = gr;
  dYb[i] = bf16_bits(gr);
  sq[i] = d * d;
}

// dZ = dH * (1 - H^2) (tanh derivative), FP32 and BF16.
__global__ void k_tanh_back(const float* __restrict__ dH, const float* __restrict__ H, int64_t n,
                            float* __restrict__ dZ, unsigned short* __restrict__ dZb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float h = H[i];
  const float v = dH[i] * (1.0f - h * h);
  dZ[i] = v;
  dZb[i] = bf16_bits(v);
}

// out[y][c] = sum over b in slice y of X[b][c] (sequential in b), for c < ncols;
// slices of kchunk rows, one per blockIdx.y (added in order afterwards).
__global__ void k_col_sum(const float* __restrict__ X, int B, int ncols, int kchunk, float* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const int b0 = blockIdx.y * kchunk, b1 = min(B, b0 + kchunk);
  float s = 0.0f;
#pragma unroll 16
  for (int b = b0; b < b1; ++b) s += X[(int64_t)b * ncols + c];
  out[(int64_t)blockIdx.y * ncols + c] = s;
}

// dW1[j][t] = sum_b dZ1[b][j] in[b][t] (BF16-rounded operands, FP32 sum in b
// order within a slice of kchunk rows per blockIdx.y; slices added in order).
__global__ void k_dw1(const unsigned short* __restrict__ dZb, const float* __restrict__ in, int B, int kchunk,
                      float* __restrict__ dW1) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= kH * 2) return;
  const int j = o / 2, t = o % 2;
  const int b0 = blockIdx.y * kchunk, b1 = min(B, b0 + kchunk);
  float s = 0.0f;
#pragma unroll 16
  for (int b = b0; b < b1; ++b) s = fmaf(bf16_float(dZb[(int64_t)b * kH + j]), bf16_float(bf16_bits(in[2 * b + t])), s);
  dW1[(int64_t)blockIdx.y * kH * 2 + o] = s;
}

// Adam step on the FP32 masters, then their BF16 copies.
__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mm,
                       float* __restrict__ Vm, unsigned short* __restrict__ Pb, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float g = G[i];
  const float m = b1 * Mm[i] + (1.0f - b1) * g;
  const float v = b2 * Vm[i] + (1.0f - b2) * g * g;
  Mm[i] = m;
  Vm[i] = v;
  const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[i] = p;
  Pb[i] = bf16_bits(p);
}

__global__ void k_to_bf16(const float* __restrict__ P, unsigned short* __restrict__ Pb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) Pb[i] = bf16_bits(P[i]);
}

// ---------------------------------------------------------------------------------------
// Sample preparation: normalised inputs and envelope-scaled targets.


__device__ __forceinline__ void envelope(const SurDev& S, float lx, float e[kO]) {
  int lo = 0, hi = S.nx - 2;
  while (lo < hi) {  // largest i <= nx-2 with lxk[i] <= lx
    const int mid = (lo + hi + 1) >> 1;
    if (S.lxk[mid] <= lx) lo = mid; else hi = mid - 1;
  }
  const float t = fminf(fmaxf((lx - S.lxk[lo]) / (S.lxk[lo + 1] - S.lxk[lo]), 0.0f), 1.0f);
#pragma unroll
  for (int c = 0; c < kO; ++c) e[c] = S.env[lo * kO + c] + t * (S.env[(lo + 1) * kO + c] - S.env[lo * kO + c]);
}

__global__ void k_prep_samples(SurDev S, const double* __restrict__ X, const double* __restrict__ Q2,
                               const double* __restrict__ XF, int64_t n, float* __restrict__ in,
                               float* __restrict__ T) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double lx = log(X[i]), lq = log(Q2[i]);
  in[2 * i] = (float)(2.0 * (lx - S.lx0) * S.ilx - 1.0);
  in[2 * i + 1] = (float)(2.0 * (lq - S.lq0) * S.ilq - 1.0);
  float e[kO];
  envelope(S, (float)lx, e);
  for (int c = 0; c < kO; ++c) {
    float t = 0.0f;
    if (c < S.P && e[c] > 0.0f) {
      const double xf = XF[i * S.P + c];
      t = isfinite(xf) ? (float)(xf / (double)e[c]) : 0.0f;
    }
    T[i * kO + c] = t;
  }
}

// ---------------------------------------------------------------------------------------
// Fused inference.  Each wave takes 64 consecutive points: their inputs,
// fallback flags and envelope cells are prepared one lane per point, then the
// network runs on four 16-point sub-tiles (layer 1 on the VALUs directly into
// the A-operand layout of layer 2; layers 2-4 on the matrix cores with the
// weight fragments held in registers; hidden activations re-laid out from the
// accumulator layout to the A-operand layout through 2 KB of LDS per wave).
// (Keeping the activations in registers by computing the transposed products,
// weights as the A operand, needs ~250 registers and ran 40 % slower.)
// Points in the fallback domain are then evaluated by the FP32 interpolator:
// each is located once (one lane per point: sub-grid, cells, weights), after
// which one lane per (point, flavour) gathers its 4x4 stencil.
constexpr int kSurWaves = 4;

__device__ __forceinline__ bool trusted(const SurDev& S, const MemberDev& m, double x, double q2) {
  if (!(x >= m.xmin && x <= m.xmax && q2 >= m.qmin && q2 <= m.qmax)) return false;
  int k = 0;
  for (int j = 1; j < m.K; ++j)
    if (m.sub[j].qfirst <= q2) k = j;
  return S.trust[k] && x >= S.txlo[k] && x < S.txhi[k] && q2 >= S.tqlo[k] && q2 < S.tqhi[k];
}

// Location of one fallback point (what interp_point derives before its gathers).
struct FbRec {
  float w[4], v[4];
  int base, sa, mode, pt;  // grid offset and x stride (elements), region bits, point within the 64
  double p0, p1;           // extrapolation parameters
};

// LDS of k_sur_infer: [nx] ln x knots, [nx][16] envelope, W1 (BF16-rounded; W1 and
// b1-b3 times 2 log2(e)),
// b1, b2, b3, b4, then per wave the fallback records, the activation tile and
// the point records.
size_t sur_infer_shared_bytes(int nx) {
  const size_t head = (size_t)4 * (nx + nx * kO + 2 * kH + 3 * kH + kO);
  return ((head + 15) & ~(size_t)15) + (size_t)kSurWaves * (64 * sizeof(FbRec) + 16 * kH * 2 + 64 * 16);
}


__global__ __launch_bounds__(64 * kSurWaves) void k_sur_infer(SurDev S, MemberDev m, const unsigned short* __restrict__ Pb,
                                                             const float* __restrict__ Pf,
                                                             const double* __restrict__ X,
                                                             const double* __restrict__ Q2, int64_t n,
                                                             float* __restrict__ out, double invL01,
                                                             unsigned long long* __restrict__ nerr) {
  extern __shared__ __align__(16) float sdyn[];
  float* slxk = sdyn;                         // [nx]
  float* senv = slxk + S.nx;                  // [nx][kO]
  float* sw1 = senv + S.nx * kO;              // [kH][2], BF16-rounded
  float* sb1 = sw1 + 2 * kH;
  float* sb2 = sb1 + kH;
  float* sb3 = sb2 + kH;
  float* sb4 = sb3 + kH;                      // [kO]
  const size_t head = (size_t)4 * (S.nx + S.nx * kO + 2 * kH + 3 * kH + kO);
  FbRec* sfb = reinterpret_cast<FbRec*>(reinterpret_cast<unsigned char*>(sdyn) + ((head + 15) & ~(size_t)15));
  unsigned short* shs = reinterpret_cast<unsigned short*>(sfb + kSurWaves * 64);  // [waves][16 * kH]
  float* spt = reinterpret_cast<float*>(shs + kSurWaves * 16 * kH);                // [waves][64][4]
  for (int i = threadIdx.x; i < S.nx; i += 64 * kSurWaves) slxk[i] = S.lxk[i];
  for (int i = threadIdx.x; i < S.nx * kO; i += 64 * kSurWaves) senv[i] = S.env[i];
  // hidden-layer weights and biases staged times 2 log2(e), the argument scale of tanh_scaled
  for (int i = threadIdx.x; i < 2 * kH; i += 64 * kSurWaves)
    sw1[i] = kTwoLog2e * bf16_float(bf16_bits(Pf[kOffW1 + i]));
  for (int i = threadIdx.x; i < kH; i += 64 * kSurWaves) {
    sb1[i] = kTwoLog2e * Pf[kOffB1 + i];
    sb2[i] = kTwoLog2e * Pf[kOffB2 + i];
    sb3[i] = kTwoLog2e * Pf[kOffB3 + i];
  }
  for (int i = threadIdx.x; i < kO; i += 64 * kSurWaves) sb4[i] = Pf[kOffB4 + i];
  __syncthreads();

  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, r = l & 15, g = l >> 4;
  unsigned short* hs = shs + wv * 16 * kH;
  float* pt4 = spt + wv * 64 * 4;   // per point: u, v, envelope t, envelope cell (as int bits)
  FbRec* fbr = sfb + wv * 64;
  // weight fragments: B operand of layer L, N-tile t, K-step s: lane holds W[n = 16t + r][k = 32s + 8g + i]
  bf16x8 w2[4][2], w3[4][2], w4[2];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int nn = 16 * t + r, kk = 32 * s + 8 * g + i;
        w2[t][s][i] = __builtin_bit_cast(__bf16, Pb[kOffW2 + nn * kH + kk]);
        w3[t][s][i] = __builtin_bit_cast(__bf16, Pb[kOffW3 + nn * kH + kk]);
      }
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 8; ++i) w4[s][i] = __builtin_bit_cast(__bf16, Pb[kOffW4 + r * kH + 32 * s + 8 * g + i]);
  const Tables gtb{m.knots, m.cells, m.hints, m.subs};
  const float* __restrict__ gvals = member_values<float>(m);

  const int64_t ntiles = (n + 63) / 64;
  for (int64_t tile = (int64_t)blockIdx.x * kSurWaves + wv; tile < ntiles; tile += (int64_t)gridDim.x * kSurWaves) {
    const int64_t p0 = tile * 64;
    const int np = (int)min((int64_t)64, n - p0);
    // one lane per point: inputs, fallback flag, envelope interval
    double xr = 0.5, qr = 1.0;
    bool fb = false;
    if (l < np) {
      xr = X[p0 + l];
      qr = Q2[p0 + l];
      fb = !trusted(S, m, xr, qr);
      const double lx = log(xr), lq = log(qr);
      pt4[4 * l] = (float)(2.0 * (lx - S.lx0) * S.ilx - 1.0);
      pt4[4 * l + 1] = (float)(2.0 * (lq - S.lq0) * S.ilq - 1.0);
      const float lxf = (float)lx;
      int lo = 0, hi = S.nx - 2;
      while (lo < hi) {  // largest i <= nx-2 with lxk[i] <= ln x
        const int mid = (lo + hi + 1) >> 1;
        if (slxk[mid] <= lxf) lo = mid; else hi = mid - 1;
      }
      pt4[4 * l + 2] = fminf(fmaxf((lxf - slxk[lo]) / (slxk[lo + 1] - slxk[lo]), 0.0f), 1.0f);
      pt4[4 * l + 3] = __int_as_float(lo);
    } else {
      pt4[4 * l] = pt4[4 * l + 1] = pt4[4 * l + 2] = 0.0f;
      pt4[4 * l + 3] = __int_as_float(0);
    }
    const unsigned long long fbmask = __ballot(fb);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q0 = 0; q0 < np; q0 += 16) {
      // layer 1 straight into the A layout: lane (r, g) holds h1[point q0 + r][32 s + 8 g + i]
      const float u = bf16_float(bf16_bits(pt4[4 * (q0 + r)])), v = bf16_float(bf16_bits(pt4[4 * (q0 + r) + 1]));
      bf16x8 a[2];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int j = 32 * s + 8 * g + i;
          const float zs = fmaf(sw1[2 * j], u, fmaf(sw1[2 * j + 1], v, sb1[j]));
          a[s][i] = __builtin_bit_cast(__bf16, bf16_bits(tanh_scaled(zs)));
        }
      // layers 2 and 3
#pragma unroll
      for (int layer = 0; layer < 2; ++layer) {
        const float* bl = layer == 0 ? sb2 : sb3;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], layer == 0 ? w2[t][0] : w3[t][0], acc, 0, 0, 0);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], layer == 0 ? w2[t][1] : w3[t][1], acc, 0, 0, 0);
          const float bn = bl[16 * t + r];
#pragma unroll
          for (int i = 0; i < 4; ++i) hs[(4 * g + i) * kH + 16 * t + r] = bf16_bits(tanh_scaled(fmaf(acc[i], kTwoLog2e, bn)));
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int i = 0; i < 8; ++i) a[s][i] = __builtin_bit_cast(__bf16, hs[r * kH + 32 * s + 8 * g + i]);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // layer 4: lane (r, g) gets y[point q0 + 4 g + i][output r]; times the envelope
      f32x4 y = {0.f, 0.f, 0.f, 0.f};
      y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[0], w4[0], y, 0, 0, 0);
      y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[1], w4[1], y, 0, 0, 0);
      const float b4 = sb4[r];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int pt = q0 + 4 * g + i;
        if (pt < np && r < S.P && !((fbmask >> pt) & 1ull)) {
          const int lo = __float_as_int(pt4[4 * pt + 3]);
          const float t = pt4[4 * pt + 2];
          const float e0 = senv[lo * kO + r], e1 = senv[(lo + 1) * kO + r];
          out[(p0 + pt) * S.P + r] = (y[i] + b4) * (e0 + t * (e1 - e0));
        }
      }
    }
    // fallback points: located once each, then one lane per (point, stored column)
    if (fbmask) {
      const int nfb = __popcll(fbmask);
      bool bad = false;
      if (fb) {
        FbRec& rc = fbr[__popcll(fbmask & ((1ull << l) - 1))];
        const PointLoc L = locate_point<float>(m, gtb, xr, qr, rc.w, rc.v);
        rc.base = L.base;
        rc.sa = L.sa;
        rc.mode = L.mode;
        rc.pt = l;
        rc.p0 = L.p0;
        rc.p1 = L.p1;
        bad = L.mode & kInvalid;
      }
      const unsigned long long badm = __ballot(bad);
      if (badm && l == 0) atomicAdd(nerr, (unsigned long long)__popcll(badm));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int e = l; e < nfb * S.P; e += 64) {
        const int k = e / S.P, c = e - k * S.P;
        const FbRec& rc = fbr[k];
        float val;
        if (rc.mode & kInvalid) {
          val = NAN;
        } else {
          const float* f = gvals + rc.base + c;
          if (!(rc.mode & (kLowX | kLowQ | kHighQ))) {
            float F[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) F[a][b] = f[a * rc.sa + b * m.P32];
            val = interp_stencil<float>(F, rc.w, rc.v);
          } else {
            const Wts wt{(double)rc.w[0], (double)rc.w[1], (double)rc.w[2], (double)rc.w[3],
                         (double)rc.v[0], (double)rc.v[1], (double)rc.v[2], (double)rc.v[3]};
            val = (float)extrap_entry<float>(f, rc.sa, m.P32, rc.mode, wt, rc.p0, rc.p1, invL01);
          }
        }
        out[(p0 + rc.pt) * S.P + c] = val;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
}

}  // namespace pdfmi

namespace pdfmi {

// ---------------------------------------------------------------------------------------
// Host-side launchers.


int sur_nparams() { return kNParams; }
int sur_out_width() { return kO; }
int sur_hidden() { return kH; }
size_t sur_batch_floats(int B) { return (size_t)B * (3 * kH + 3 * kO + 2 * kH) ; }

static unsigned nb(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// out[i] = sum over slices s = 0..S-1 (in order) of P[s n + i].
__global__ void k_sum_slices(const float* __restrict__ P, int S, int n, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = P[i];
  for (int q = 1; q < S; ++q) acc += P[(int64_t)q * n + i];
  out[i] = acc;
}

// Long reductions (the weight gradients, K = batch) are split into slices of
// kSplitK rows so that the few 16x16 output tiles keep many waves busy.
constexpr int kSplitK = 256;
constexpr int kMaxSlices = 64;

static void gemm(const unsigned short* A, int sam, int sak, const unsigned short* B, int sbk, int sbn, float* C, int ldc,
                 unsigned short* Cb, int M, int N, int K, const float* bias, int act, float* ws, hipStream_t s) {
  const unsigned tiles = (unsigned)((M / 16) * (N / 16));
  int S = (K + kSplitK - 1) / kSplitK;
  if (S > kMaxSlices) S = kMaxSlices;
  if (S > 1 && !bias && !act && !Cb && ws && ldc == N) {
    const int kchunk = ((K + S - 1) / S + 31) / 32 * 32;
    S = (K + kchunk - 1) / kchunk;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(tiles, (unsigned)S), dim3(64), 0, s, A, sam, sak, B, sbk, sbn, ws, ldc,
                       nullptr, M, N, K, nullptr, 0, kchunk);
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s, ws, S, M * N, C);
    return;
  }
  hipLaunchKernelGGL(k_gemm_bf16, dim3(tiles), dim3(64), 0, s, A, sam, sak, B, sbk, sbn, C, ldc, Cb, M, N, K, bias,
                     act, K);
}

// Sum of 256 per-thread values of a 256-thread block by a fixed pairwise tree
// (the same order on every call); the result is valid in thread 0.
__device__ float block_tree_sum(float v, float* red) {
  red[threadIdx.x] = v;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  return red[0];
}

// 256 blocks of 256 threads: block j sums its contiguous share of x, its
// threads striding through it (coalesced), into partial[j].
__global__ void k_sum_partial(const float* __restrict__ x, int64_t n, float* __restrict__ partial) {
  __shared__ float red[256];
  const int64_t per = (n + 255) / 256;
  const int64_t b = blockIdx.x * per, e = min(b + per, n);
  float s = 0.0f;
  for (int64_t i = b + threadIdx.x; i < e; i += 256) s += x[i];
  s = block_tree_sum(s, red);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
__global__ void k_sum_final(const float* __restrict__ partial, float scale, float* __restrict__ out) {
  __shared__ float red[256];
  const float s = block_tree_sum(partial[threadIdx.x], red);
  if (threadIdx.x == 0) *out = s * scale;
}

// Column sums and the first-layer weight gradient over the batch, in row
// slices of at least kColRows rows added in order (a thread per column and
// slice: short slices give the few columns enough waves to hide latency).
constexpr int kColRows = 64;
static void col_sum(const float* X, int B, int ncols, float* out, float* ws, hipStream_t s) {
  const int S = min(kMaxSlices, (B + kColRows - 1) / kColRows);
  const int kchunk = (B + S - 1) / S;
  hipLaunchKernelGGL(k_col_sum, dim3((unsigned)((ncols + 63) / 64), (unsigned)S), dim3(64), 0, s, X, B, ncols, kchunk,
                     ws);
  hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((ncols + 255) / 256)), dim3(256), 0, s, ws, S, ncols, out);
}

static void dw1(const unsigned short* dZb, const float* in, int B, float* out, float* ws, hipStream_t s) {
  const int S = min(kMaxSlices, (B + kColRows - 1) / kColRows);
  const int kchunk = (B + S - 1) / S;
  hipLaunchKernelGGL(k_dw1, dim3(1, (unsigned)S), dim3(128), 0, s, dZb, in, B, kchunk, ws);
  hipLaunchKernelGGL(k_sum_slices, dim3(1), dim3(256), 0, s, ws, S, kH * 2, out);
}

// One forward + backward pass on a batch (inputs in[B][2], targets T[B][kO]):
// gradients into buf.G, loss (mean squared error) into buf.loss.
hipError_t sur_forward_backward(const SurBufs& b, const float* in, const float* T, int B, hipStream_t s) {
  const unsigned short* W2 = b.Pb + kOffW2;
  const unsigned short* W3 = b.Pb + kOffW3;
  const unsigned short* W4 = b.Pb + kOffW4;
  hipLaunchKernelGGL(k_layer1, dim3(nb((int64_t)B * kH, 256)), dim3(256), 0, s, in, b.P, B, b.h1, b.h1b);
  // z = h W^T + b: A(m=b,k) = h[b][k]; B(k,n) = W[n][k]
  gemm(b.h1b, kH, 1, W2, 1, kH, b.h2, kH, b.h2b, B, kH, kH, b.P + kOffB2, 1, b.wpart, s);
  gemm(b.h2b, kH, 1, W3, 1, kH, b.h3, kH, b.h3b, B, kH, kH, b.P + kOffB3, 1, b.wpart, s);
  gemm(b.h3b, kH, 1, W4, 1, kH, b.y, kO, nullptr, B, kO, kH, b.P + kOffB4, 0, b.wpart, s);
  hipLaunchKernelGGL(k_loss_grad, dim3(nb((int64_t)B * kO, 256)), dim3(256), 0, s, b.y, T, B, b.dy, b.dyb, b.sq);
  hipLaunchKernelGGL(k_sum_partial, dim3(256), dim3(256), 0, s, b.sq, (int64_t)B * kO, b.partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, b.partial, 1.0f / (float)((int64_t)B * kO), b.loss);
  // layer 4: dW4[o][i] = sum_b dy[b][o] h3[b][i]; db4; dh3 = dy W4
  gemm(b.dyb, 1, kO, b.h3b, kH, 1, b.G + kOffW4, kH, nullptr, kO, kH, B, nullptr, 0, b.wpart, s);
  col_sum(b.dy, B, kO, b.G + kOffB4, b.wpart, s);
  gemm(b.dyb, kO, 1, W4, kH, 1, b.dh, kH, nullptr, B, kH, kO, nullptr, 0, b.wpart, s);
  // layers 3 and 2
  const float* Hs[3] = {b.h1, b.h2, b.h3};
  const unsigned short* Hbs[3] = {b.h1b, b.h2b, b.h3b};
  const unsigned short* Ws[2] = {W2, W3};
  const int offW[2] = {kOffW2, kOffW3}, offB[2] = {kOffB2, kOffB3};
  for (int L = 1; L >= 0; --L) {  // L = 1: layer 3 (input h2, output h3); L = 0: layer 2 (h1 -> h2)
    hipLaunchKernelGGL(k_tanh_back, dim3(nb((int64_t)B * kH, 256)), dim3(256), 0, s, b.dh, Hs[L + 1],
                       (int64_t)B * kH, b.dz, b.dzb);
    gemm(b.dzb, 1, kH, Hbs[L], kH, 1, b.G + offW[L], kH, nullptr, kH, kH, B, nullptr, 0, b.wpart, s);
    col_sum(b.dz, B, kH, b.G + offB[L], b.wpart, s);
    // dh_in = dz W: A(m=b, k=j) = dz[b][j]; B(k=j, n=i) = W[j][i]
    gemm(b.dzb, kH, 1, Ws[L], kH, 1, b.dh, kH, nullptr, B, kH, kH, nullptr, 0, b.wpart, s);
  }
  // layer 1
  hipLaunchKernelGGL(k_tanh_back, dim3(nb((int64_t)B * kH, 256)), dim3(256), 0, s, b.dh, b.h1, (int64_t)B * kH, b.dz,
                     b.dzb);
  dw1(b.dzb, in, B, b.G + kOffW1, b.wpart, s);
  col_sum(b.dz, B, kH, b.G + kOffB1, b.wpart, s);
  return hipGetLastError();
}

hipError_t sur_adam(const SurBufs& b, float lr, int step, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(k_adam, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.P, b.G, b.M, b.V, b.Pb, kNParams, lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t sur_refresh_bf16(const SurBufs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.P, b.Pb, kNParams);
  return hipGetLastError();
}

hipError_t sur_prep(const SurDev& S, const double* x, const double* q2, const double* xf, int64_t n, float* in,
                    float* T, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_prep_samples, dim3(nb(n, 256)), dim3(256), 0, s, S, x, q2, xf, n, in, T);
  return hipGetLastError();
}

hipError_t sur_infer(const SurDev& S, const MemberDev& m, const SurBufs& b, const double* x, const double* q2,
                     int64_t n, float* out, double invL01, unsigned long long* nerr, int n_cu, hipStream_t s) {
  const int64_t tiles = (n + 63) / 64;
  const int64_t blocks = min((tiles + kSurWaves - 1) / kSurWaves, (int64_t)n_cu * 8);
  if (blocks > 0) {
    const size_t shm = sur_infer_shared_bytes(S.nx);
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_sur_infer), shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sur_infer, dim3((unsigned)blocks), dim3(64 * kSurWaves), shm, s, S, m, b.Pb, b.P, x, q2, n,
                       out, invL01, nerr);
  }
  return hipGetLastError();
}

}  // namespace pdfmi
