// MLP surrogate of one member's PDFs (growth path of the interpolation
// library): (ln x, ln Q^2) -> all stored flavours, 2 -> 64 -> 64 -> 64 -> 16
// (outputs beyond the stored columns are padding), tanh hidden activations,
// FP32 master weights trained with Adam.
//
// Arithmetic: the first layer (two inputs) in FP32 on the vector ALUs;
// layers 2-4 on the matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation) with every operand carried as a BF16 pair (value = hi + lo,
// lo = bf16(value - hi)) and each product formed as hi*hi + lo*hi + hi*lo:
// about 16 significant bits per operand, where single BF16 operands (8 bits)
// left the network's relative error near 1e-3.  The backward pass multiplies
// BF16 signals with the hi halves.
//
// The network predicts y_c = xf_c / E_c(x), where E_c is a signed cubic
// Hermite envelope in ln x through the grid value of largest magnitude at
// each x knot (it follows the x dependence, sign changes included, so the
// targets are smooth and O(1)).  Training uses only samples inside the
// network's domain; inference falls back to the FP32 interpolator outside
// the grid and in the first/last x or Q^2 cell of a sub-grid (which includes
// the cells next to flavour thresholds).
//
// Training is deterministic: every reduction has a fixed order (one wave per
// 16x16 output tile loops over the whole batch; bias sums are sequential per
// column), so a checkpointed and resumed run reproduces a straight run bit for
// bit.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>

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
// BF16 pair of v: hi = bf16(v), lo = bf16(v - hi) (the difference is exact in FP32)
__device__ __forceinline__ void split_bits(float v, unsigned short& hi, unsigned short& lo) {
  hi = bf16_bits(v);
  lo = bf16_bits(v - bf16_float(hi));
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
// with A2 / B2 (the lo halves of split operands, same strides) the products
// are A B + A2 B + A B2.  M, N multiples of 16; K any (zero padded to 32).
// One wave per 16x16 tile, K walked in order (fixed summation order).
// Writes FP32 C (ldc) and, if Cb != null, its BF16 hi half (and the lo half
// to Cl if not null).
// With gridDim.y > 1 workgroup y covers k in [y kchunk, (y + 1) kchunk) and
// writes its partial tile to C + y M ldc (the slices are added in order by
// k_sum_slices); bias and activation then belong to the unsplit form only.
__global__ __launch_bounds__(64) void k_gemm_bf16(const unsigned short* __restrict__ A,
                                                  const unsigned short* __restrict__ A2, int sam, int sak,
                                                  const unsigned short* __restrict__ B,
                                                  const unsigned short* __restrict__ B2, int sbk, int sbn,
                                                  float* __restrict__ C, int ldc, unsigned short* __restrict__ Cb,
                                                  unsigned short* __restrict__ Cl, int M, int N, int K,
                                                  const float* __restrict__ bias, int act, int kchunk) {
  const int tn = N / 16;
  const int m0 = (blockIdx.x / tn) * 16, n0 = (blockIdx.x % tn) * 16;
  const int l = threadIdx.x, r = l & 15, g = l >> 4;
  const int kb = blockIdx.y * kchunk, ke = min(K, kb + kchunk);
  C += (int64_t)blockIdx.y * M * ldc;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kb; k0 < ke; k0 += 32) {
    bf16x8 a, b, a2, b2;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int k = k0 + 8 * g + i;
      const int64_t ia = (int64_t)(m0 + r) * sam + (int64_t)k * sak, ib = (int64_t)k * sbk + (int64_t)(n0 + r) * sbn;
      a[i] = __builtin_bit_cast(__bf16, k < ke ? A[ia] : (unsigned short)0);
      b[i] = __builtin_bit_cast(__bf16, k < ke ? B[ib] : (unsigned short)0);
      a2[i] = __builtin_bit_cast(__bf16, (A2 && k < ke) ? A2[ia] : (unsigned short)0);
      b2[i] = __builtin_bit_cast(__bf16, (B2 && k < ke) ? B2[ib] : (unsigned short)0);
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    if (A2) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2, b, acc, 0, 0, 0);
    if (B2) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b2, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * g + i, n = n0 + r;
    float v = acc[i];
    if (bias) v += bias[n];
    if (act) v = tanh_f(v);
    C[(int64_t)m * ldc + n] = v;
    if (Cb) {
      unsigned short hi, lo;
      split_bits(v, hi, lo);
      Cb[(int64_t)m * ldc + n] = hi;
      if (Cl) Cl[(int64_t)m * ldc + n] = lo;
    }
  }
}

// Layer 1 (K = 2, FP32 on the vector ALUs): h1 = tanh(W1 in + b1), FP32 and
// its BF16 pair.
// Batch slice of a training step: rows (step % nb) * B of the training set
// when st is given (in and T are then the set's first rows), else as passed.
__device__ __forceinline__ int64_t batch_row(const SurStep* st, int B) {
  return st ? (st->step % st->nb) * (int64_t)B : 0;
}

__global__ void k_layer1(const float* __restrict__ in, const SurStep* __restrict__ st, const float* __restrict__ P,
                         int B, float* __restrict__ h, unsigned short* __restrict__ hb,
                         unsigned short* __restrict__ hl) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * kH) return;
  in += 2 * batch_row(st, B);
  const int b = (int)(i / kH), j = (int)(i % kH);
  const float z = fmaf(P[kOffW1 + 2 * j], in[2 * b], fmaf(P[kOffW1 + 2 * j + 1], in[2 * b + 1], P[kOffB1 + j]));
  const float t = tanh_f(z);
  h[i] = t;
  split_bits(t, hb[i], hl[i]);
}

// Loss (mean squared error over B x kO) and its gradient dY = 2 (Y - T) / (B kO).
__global__ void k_loss_grad(const float* __restrict__ Y, const float* __restrict__ T, const SurStep* __restrict__ st,
                            int B, float* __restrict__ dY, unsigned short* __restrict__ dYb, float* __restrict__ sq) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)B * kO) return;
  T += kO * batch_row(st, B);
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

// dW1[j][t] = sum_b dZ1[b][j] in[b][t] (FP32, in b order within a slice of
// kchunk rows per blockIdx.y; slices added in order).
__global__ void k_dw1(const float* __restrict__ dZ, const float* __restrict__ in, const SurStep* __restrict__ st,
                      int B, int kchunk, float* __restrict__ dW1) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= kH * 2) return;
  in += 2 * batch_row(st, B);
  const int j = o / 2, t = o % 2;
  const int b0 = blockIdx.y * kchunk, b1 = min(B, b0 + kchunk);
  float s = 0.0f;
#pragma unroll 16
  for (int b = b0; b < b1; ++b) s = fmaf(dZ[(int64_t)b * kH + j], in[2 * b + t], s);
  dW1[(int64_t)blockIdx.y * kH * 2 + o] = s;
}

// Adam step on the FP32 masters (Kingma & Ba, bias-corrected moments; c1 =
// 1 - b1^t, c2 = 1 - b2^t for update number t), then their BF16 pairs.  With
// st the update number is st->step + 1 and the learning rate follows the
// cosine schedule lrf + (lr0 - lrf)(1 + cos(pi min(1, step / total))) / 2.
__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mm,
                       float* __restrict__ Vm, unsigned short* __restrict__ Pb, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2, const SurStep* __restrict__ st) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (st) {
    const double t = (double)st->step;
    const double frac = fmin(1.0, t / (double)st->total);
    lr = (float)(st->lrf + 0.5 * ((double)st->lr0 - st->lrf) * (1.0 + cos(3.141592653589793 * frac)));
    c1 = (float)(1.0 - pow(0.9, t + 1.0));  // the betas in FP64, as the host computes them
    c2 = (float)(1.0 - pow(0.999, t + 1.0));
  }
  const float g = G[i];
  const float m = b1 * Mm[i] + (1.0f - b1) * g;
  const float v = b2 * Vm[i] + (1.0f - b2) * g * g;
  Mm[i] = m;
  Vm[i] = v;
  const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[i] = p;
  split_bits(p, Pb[i], Pb[n + i]);
}

// Start of a training call: the global step, the call's step index, the schedule and the loss output.
__global__ void k_train_begin(SurStep* st, int64_t step, int64_t nb, int total, float lr0, float lrf,
                              float* loss_out) {
  st->step = step;
  st->call = 0;
  st->nb = nb;
  st->total = total;
  st->lr0 = lr0;
  st->lrf = lrf;
  st->loss_out = loss_out;
}

// End of a training step.
__global__ void k_train_advance(SurStep* st) {
  st->step += 1;
  st->call += 1;
}

__global__ void k_to_bf16(const float* __restrict__ P, unsigned short* __restrict__ Pb, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) split_bits(P[i], Pb[i], Pb[n + i]);
}

// ---------------------------------------------------------------------------------------
// Envelope and sample preparation.

// Hermite weights of the envelope at ln x: cell i (largest i <= nx-2 with
// lxk[i] <= ln x, clamped) and the basis h00, h10 D, h01, h11 D of its
// parameter t (clamped to [0, 1]), D = lxk[i+1] - lxk[i].
struct EnvW {
  int i;
  float h00, h10, h01, h11;
};

__device__ __forceinline__ EnvW env_weights(const double* lxk, int nx, double lx) {
  int lo = 0, hi = nx - 2;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (lxk[mid] <= lx) lo = mid; else hi = mid - 1;
  }
  const double D = lxk[lo + 1] - lxk[lo];
  const double t = fmin(fmax((lx - lxk[lo]) / D, 0.0), 1.0);
  const double s = 1.0 - t, t2 = t * t, s2 = s * s;  // factored basis: no cancellation near t = 0, 1
  EnvW w;
  w.i = lo;
  w.h00 = (float)(s2 * (1.0 + 2.0 * t));
  w.h10 = (float)(t * s2 * D);
  w.h01 = (float)(t2 * (3.0 - 2.0 * t));
  w.h11 = (float)(-(s * t2) * D);
  return w;
}

// E_c at the point whose weights are w (tables [nx][kO] of values and slopes)
__device__ __forceinline__ float env_at(const float* e, const float* d, int i, float h00, float h10, float h01,
                                        float h11, int c) {
  const int a = i * kO + c, b = a + kO;
  return fmaf(h00, e[a], fmaf(h10, d[a], fmaf(h01, e[b], h11 * d[b])));
}

__device__ __forceinline__ bool trusted(const SurDev& S, const MemberDev& m, double x, double q2) {
  if (!(x >= m.xmin && x <= m.xmax && q2 >= m.qmin && q2 <= m.qmax)) return false;
  int k = 0;
  for (int j = 1; j < m.K; ++j)
    if (m.sub[j].qfirst <= q2) k = j;
  return S.trust[k] && x >= S.txlo[k] && x < S.txhi[k] && q2 >= S.tqlo[k] && q2 < S.tqhi[k];
}

// Normalised inputs, targets xf_c / E_c (0 where E_c = 0 or xf is not
// finite) and whether the sample lies in the network's domain.
__global__ void k_prep_samples(SurDev S, MemberDev m, const double* __restrict__ X, const double* __restrict__ Q2,
                               const double* __restrict__ XF, int64_t n, float* __restrict__ in,
                               float* __restrict__ T, unsigned char* __restrict__ keep) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double x = X[i], q2 = Q2[i];
  keep[i] = trusted(S, m, x, q2) ? 1 : 0;
  const double lx = log(x), lq = log(q2);
  in[2 * i] = (float)(2.0 * (lx - S.lx0) * S.ilx - 1.0);
  in[2 * i + 1] = (float)(2.0 * (lq - S.lq0) * S.ilq - 1.0);
  const EnvW w = env_weights(S.lxk, S.nx, lx);
  for (int c = 0; c < kO; ++c) {
    float t = 0.0f;
    if (c < S.P) {
      const float e = env_at(S.env, S.envd, w.i, w.h00, w.h10, w.h01, w.h11, c);
      const double xf = XF[i * S.P + c];
      if (e != 0.0f && isfinite(xf)) t = (float)(xf / (double)e);
    }
    T[i * kO + c] = t;
  }
}

// in[j], T[j] = in_all[idx[j]], T_all[idx[j]] for j < n (the kept samples, in order).
__global__ void k_gather_samples(const float* __restrict__ in_all, const float* __restrict__ T_all,
                                 const int64_t* __restrict__ idx, int64_t n, float* __restrict__ in,
                                 float* __restrict__ T) {
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t i = idx[j];
  in[2 * j] = in_all[2 * i];
  in[2 * j + 1] = in_all[2 * i + 1];
#pragma unroll
  for (int c = 0; c < kO; ++c) T[j * kO + c] = T_all[i * kO + c];
}

// ---------------------------------------------------------------------------------------
// Fused inference.  Each wave takes 64 consecutive points: their inputs,
// fallback flags and envelope weights are prepared one lane per point, then
// the network runs on four 16-point sub-tiles: layer 1 on the VALUs straight
// into the A-operand layout of layer 2 (as BF16 pairs); layers 2-4 on the
// matrix cores, three products per operand pair, with the hi halves of the
// weight fragments held in registers and the lo halves read from LDS; hidden
// activations re-laid out from the accumulator layout to the A-operand layout
// through LDS.  The outputs times the envelope go to a 16 x 16 LDS tile from
// which the requested columns are stored point-major, consecutive lanes on
// consecutive values.  Points in the fallback domain are then evaluated by
// the FP32 interpolator: each is located once (one lane per point: sub-grid,
// cells, weights), after which one lane per (point, requested column)
// gathers its 4x4 stencil.
//
// LDS rows of 64 BF16 values (the activation tiles, the lo weight halves)
// hold their eight 16-byte chunks in the order chunk ^ (row & 7), so the 16
// rows an operand read touches spread over the banks.
// Launch shapes: with the hi weight fragments in registers (kWeightsInLds =
// false) a wave needs ~200 VGPRs (2 waves per SIMD, blocks of 4 waves); with
// both halves of the weights in LDS it fits 128 VGPRs and blocks of 16 waves
// fill the CU's LDS (4 waves per SIMD).
constexpr bool kWeightsInLds = true;
constexpr int kSurWaves = kWeightsInLds ? 16 : 4;
constexpr int kSurRec = 8;   // floats per point record: u, v, h00, h10 D, h01, h11 D, cell, fallback

__device__ __forceinline__ int swz(int row, int col) {  // element offset of (row, col) in a swizzled [.][64] tile
  return row * kH + ((((col >> 3) ^ row) & 7) << 3) + (col & 7);
}

// Location of one fallback point (what interp_point derives before its gathers).
struct FbRec {
  float w[4], v[4];
  int base, sa, mode, pt;  // grid offset and x stride (elements), region bits, point within the 64
  double p0, p1;           // extrapolation parameters
};

// LDS of k_sur_infer: the lo halves of W2, W3 (64 x 64) and W4 (16 x 64),
// [nx] ln x knots (double), [nx][16] envelope values and slopes, W1 and b1-b3
// times 2 log2(e) (the argument scale of tanh_scaled), b4; then per wave a
// 4 KB area (activation pair tile, then the output tile, then the fallback
// records) and the point records.
constexpr size_t kSurWaveArea = 2 * 16 * kH * 2;  // 4096 bytes
constexpr size_t kSurWTile = (size_t)2 * (2 * kH * kH + kO * kH);  // one half of W2, W3, W4 (BF16)
__host__ __device__ static inline size_t sur_head_bytes(int nx) {
  const size_t b = (kWeightsInLds ? 2 : 1) * kSurWTile + (size_t)8 * nx + (size_t)4 * (2 * nx * kO + 2 * kH + 3 * kH + kO);
  return (b + 15) & ~(size_t)15;
}
constexpr size_t kSurWaveBytes = kSurWaveArea + 64 * kSurRec * 4;
// Waves per block: kSurWaves, fewer when the per-block tables (which grow
// with the number of x knots) leave less LDS.
int sur_infer_waves(int nx) {
  const size_t head = sur_head_bytes(nx);
  const size_t lds = 160 * 1024;
  const int w = head >= lds ? 0 : (int)((lds - head) / kSurWaveBytes);
  return w < kSurWaves ? w : kSurWaves;
}
size_t sur_infer_shared_bytes(int nx, int waves) { return sur_head_bytes(nx) + (size_t)waves * kSurWaveBytes; }

__global__ __launch_bounds__(64 * kSurWaves) __attribute__((amdgpu_waves_per_eu(kWeightsInLds ? 4 : 1)))
void k_sur_infer(SurDev S, MemberDev m, ReqCols rc,
                                                             const unsigned short* __restrict__ Pb,
                                                             const float* __restrict__ Pf,
                                                             const double* __restrict__ X,
                                                             const double* __restrict__ Q2, int64_t n,
                                                             float* __restrict__ out, double invL01,
                                                             unsigned long long* __restrict__ nerr) {
  extern __shared__ __align__(16) unsigned char sraw[];
  const int BS = blockDim.x, nwav = BS >> 6;
  unsigned short* sw2l = reinterpret_cast<unsigned short*>(sraw);  // [kH][kH] swizzled (16-byte chunks)
  unsigned short* sw3l = sw2l + kH * kH;
  unsigned short* sw4l = sw3l + kH * kH;                   // [kO][kH] swizzled
  unsigned short* sw2h = sw4l + kO * kH;                   // hi halves, same layout (kWeightsInLds)
  unsigned short* sw3h = sw2h + kH * kH;
  unsigned short* sw4h = sw3h + kH * kH;
  double* slxk = reinterpret_cast<double*>(kWeightsInLds ? sw4h + kO * kH : sw2h);  // [nx]
  float* senv = reinterpret_cast<float*>(slxk + S.nx);     // [nx][kO]
  float* senvd = senv + S.nx * kO;                         // [nx][kO]
  float* sw1 = senvd + S.nx * kO;                          // [kH][2]
  float* sb1 = sw1 + 2 * kH;
  float* sb2 = sb1 + kH;
  float* sb3 = sb2 + kH;
  float* sb4 = sb3 + kH;                                   // [kO]
  unsigned char* waves = sraw + sur_head_bytes(S.nx);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, r = l & 15, g = l >> 4;
  unsigned char* area = waves + (size_t)wv * kSurWaveArea;
  unsigned short* hs_hi = reinterpret_cast<unsigned short*>(area);   // [16][kH] swizzled
  unsigned short* hs_lo = hs_hi + 16 * kH;
  float* so = reinterpret_cast<float*>(area);                         // [16][kO] output tile
  FbRec* fbr = reinterpret_cast<FbRec*>(area);                        // [64] fallback records
  float* rec = reinterpret_cast<float*>(waves + (size_t)nwav * kSurWaveArea) + wv * 64 * kSurRec;

  for (int i = threadIdx.x; i < S.nx; i += BS) slxk[i] = S.lxk[i];
  for (int i = threadIdx.x; i < S.nx * kO; i += BS) {
    senv[i] = S.env[i];
    senvd[i] = S.envd[i];
  }
  for (int i = threadIdx.x; i < 2 * kH; i += BS) sw1[i] = kTwoLog2e * Pf[kOffW1 + i];
  for (int i = threadIdx.x; i < kH; i += BS) {
    sb1[i] = kTwoLog2e * Pf[kOffB1 + i];
    sb2[i] = kTwoLog2e * Pf[kOffB2 + i];
    sb3[i] = kTwoLog2e * Pf[kOffB3 + i];
  }
  for (int i = threadIdx.x; i < kO; i += BS) sb4[i] = Pf[kOffB4 + i];
  const unsigned short* Pl = Pb + kNParams;  // lo halves
  for (int i = threadIdx.x; i < kH * kH; i += BS) {
    const int row = i / kH, col = i % kH;
    sw2l[swz(row, col)] = Pl[kOffW2 + i];
    sw3l[swz(row, col)] = Pl[kOffW3 + i];
    if (kWeightsInLds) {
      sw2h[swz(row, col)] = Pb[kOffW2 + i];
      sw3h[swz(row, col)] = Pb[kOffW3 + i];
    }
  }
  for (int i = threadIdx.x; i < kO * kH; i += BS) {
    sw4l[swz(i / kH, i % kH)] = Pl[kOffW4 + i];
    if (kWeightsInLds) sw4h[swz(i / kH, i % kH)] = Pb[kOffW4 + i];
  }
  __syncthreads();

  // hi weight fragments: B operand of layer L, N-tile t, K-step s: lane holds W[n = 16t + r][k = 32s + 8g + i]
  bf16x8 w2[4][2], w3[4][2], w4[2];
  if (!kWeightsInLds) {
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
  }
  // an 8-value chunk (16 bytes) of a swizzled LDS row, as an operand fragment
  auto frag = [&](const unsigned short* tile, int row, int col0) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(tile + swz(row, col0));
  };
  const Tables gtb{m.knots, m.cells, m.hints, m.subs};
  const float* __restrict__ gvals = member_values<float>(m);
  const int R = rc.n;

  const int64_t ntiles = (n + 63) / 64;
  for (int64_t tile = (int64_t)blockIdx.x * nwav + wv; tile < ntiles; tile += (int64_t)gridDim.x * nwav) {
    const int64_t p0 = tile * 64;
    const int np = (int)min((int64_t)64, n - p0);
    // one lane per point: inputs, fallback flag, envelope weights
    double xr = 0.5, qr = 1.0;
    bool fb = false;
    float* pr = rec + l * kSurRec;
    if (l < np) {
      xr = X[p0 + l];
      qr = Q2[p0 + l];
      fb = !trusted(S, m, xr, qr);
      const double lx = log(xr), lq = log(qr);
      pr[0] = (float)(2.0 * (lx - S.lx0) * S.ilx - 1.0);
      pr[1] = (float)(2.0 * (lq - S.lq0) * S.ilq - 1.0);
      const EnvW ew = env_weights(slxk, S.nx, fb ? S.lx0 : lx);
      pr[2] = ew.h00;
      pr[3] = ew.h10;
      pr[4] = ew.h01;
      pr[5] = ew.h11;
      pr[6] = __int_as_float(ew.i);
    } else {
      pr[0] = pr[1] = pr[2] = pr[3] = pr[4] = pr[5] = 0.0f;
      pr[6] = __int_as_float(0);
    }
    pr[7] = fb ? 1.0f : 0.0f;
    const unsigned long long fbmask = __ballot(fb);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    for (int q0 = 0; q0 < np; q0 += 16) {
      // layer 1 straight into the A layout: lane (r, g) holds h1[point q0 + r][32 s + 8 g + i]
      const float u = rec[(q0 + r) * kSurRec], v = rec[(q0 + r) * kSurRec + 1];
      bf16x8 ah[2], al[2];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int j = 32 * s + 8 * g + i;
          unsigned short hb, lb;
          split_bits(tanh_scaled(fmaf(sw1[2 * j], u, fmaf(sw1[2 * j + 1], v, sb1[j]))), hb, lb);
          ah[s][i] = __builtin_bit_cast(__bf16, hb);
          al[s][i] = __builtin_bit_cast(__bf16, lb);
        }
      // layers 2 and 3
#pragma unroll
      for (int layer = 0; layer < 2; ++layer) {
        const float* bl = layer == 0 ? sb2 : sb3;
        const unsigned short* wl = layer == 0 ? sw2l : sw3l;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const bf16x8 wh = kWeightsInLds ? frag(layer == 0 ? sw2h : sw3h, 16 * t + r, 32 * s + 8 * g)
                                            : (layer == 0 ? w2[t][s] : w3[t][s]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], wh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s], wh, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], frag(wl, 16 * t + r, 32 * s + 8 * g), acc, 0, 0, 0);
          }
          const float bn = bl[16 * t + r];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int o = swz(4 * g + i, 16 * t + r);
            split_bits(tanh_scaled(fmaf(acc[i], kTwoLog2e, bn)), hs_hi[o], hs_lo[o]);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          ah[s] = frag(hs_hi, r, 32 * s + 8 * g);
          al[s] = frag(hs_lo, r, 32 * s + 8 * g);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      }
      // layer 4: lane (r, g) gets y[point q0 + 4 g + i][output r]; times the envelope into the output tile
      f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 wh = kWeightsInLds ? frag(sw4h, r, 32 * s + 8 * g) : w4[s];
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], wh, y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[s], wh, y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[s], frag(sw4l, r, 32 * s + 8 * g), y, 0, 0, 0);
      }
      const float b4 = sb4[r];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float* pq = rec + (q0 + 4 * g + i) * kSurRec;
        const float e = env_at(senv, senvd, __float_as_int(pq[6]), pq[2], pq[3], pq[4], pq[5], r);
        so[(4 * g + i) * kO + r] = (y[i] + b4) * e;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // requested columns of the network's points, point-major
      const int nq = min(16, np - q0);
      for (int e = l; e < nq * R; e += 64) {
        const int pt = e / R, j = e - pt * R;
        if (rec[(q0 + pt) * kSurRec + 7] == 0.0f) {
          const int c = rc.col[j];
          out[(p0 + q0 + pt) * R + j] = c >= 0 ? so[pt * kO + c] : 0.0f;
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // fallback points: located once each, then one lane per (point, requested column)
    if (fbmask) {
      const int nfb = __popcll(fbmask);
      bool bad = false;
      if (fb) {
        FbRec& fr = fbr[__popcll(fbmask & ((1ull << l) - 1))];
        const PointLoc L = locate_point<float>(m, gtb, xr, qr, fr.w, fr.v);
        fr.base = L.base;
        fr.sa = L.sa;
        fr.mode = L.mode;
        fr.pt = l;
        fr.p0 = L.p0;
        fr.p1 = L.p1;
        bad = L.mode & kInvalid;
      }
      const unsigned long long badm = __ballot(bad);
      if (badm && l == 0) atomicAdd(nerr, (unsigned long long)__popcll(badm));
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      for (int e = l; e < nfb * R; e += 64) {
        const int k = e / R, j = e - k * R;
        const FbRec& fr = fbr[k];
        const int c = rc.col[j];
        float val;
        if (fr.mode & kInvalid) {
          val = NAN;
        } else if (c < 0) {
          val = 0.0f;
        } else {
          const float* f = gvals + fr.base + c;
          if (!(fr.mode & (kLowX | kLowQ | kHighQ))) {
            float F[4][4];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
              for (int b = 0; b < 4; ++b) F[a][b] = f[a * fr.sa + b * m.P32];
            val = interp_stencil<float>(F, fr.w, fr.v);
          } else {
            const Wts wt{(double)fr.w[0], (double)fr.w[1], (double)fr.w[2], (double)fr.w[3],
                         (double)fr.v[0], (double)fr.v[1], (double)fr.v[2], (double)fr.v[3]};
            val = (float)extrap_entry<float>(f, fr.sa, m.P32, fr.mode, wt, fr.p0, fr.p1, invL01);
          }
        }
        out[(p0 + fr.pt) * R + j] = val;
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

// C = A B (A2, B2: lo halves of split operands, or null), see k_gemm_bf16.
static void gemm(const unsigned short* A, const unsigned short* A2, int sam, int sak, const unsigned short* B,
                 const unsigned short* B2, int sbk, int sbn, float* C, int ldc, unsigned short* Cb,
                 unsigned short* Cl, int M, int N, int K, const float* bias, int act, float* ws, hipStream_t s) {
  const unsigned tiles = (unsigned)((M / 16) * (N / 16));
  int S = (K + kSplitK - 1) / kSplitK;
  if (S > kMaxSlices) S = kMaxSlices;
  if (S > 1 && !bias && !act && !Cb && ws && ldc == N) {
    const int kchunk = ((K + S - 1) / S + 31) / 32 * 32;
    S = (K + kchunk - 1) / kchunk;
    hipLaunchKernelGGL(k_gemm_bf16, dim3(tiles, (unsigned)S), dim3(64), 0, s, A, A2, sam, sak, B, B2, sbk, sbn, ws,
                       ldc, nullptr, nullptr, M, N, K, nullptr, 0, kchunk);
    hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((M * N + 255) / 256)), dim3(256), 0, s, ws, S, M * N, C);
    return;
  }
  hipLaunchKernelGGL(k_gemm_bf16, dim3(tiles), dim3(64), 0, s, A, A2, sam, sak, B, B2, sbk, sbn, C, ldc, Cb, Cl, M, N,
                     K, bias, act, K);
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
__global__ void k_sum_final(const float* __restrict__ partial, float scale, float* __restrict__ out,
                            float* __restrict__ out2, const SurStep* __restrict__ st) {
  __shared__ float red[256];
  const float s = block_tree_sum(partial[threadIdx.x], red);
  if (threadIdx.x == 0) {
    *out = s * scale;
    if (out2) *out2 = s * scale;
    if (st && st->loss_out) st->loss_out[st->call] = s * scale;
  }
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

static void dw1(const float* dZ, const float* in, const SurStep* st, int B, float* out, float* ws, hipStream_t s) {
  const int S = min(kMaxSlices, (B + kColRows - 1) / kColRows);
  const int kchunk = (B + S - 1) / S;
  hipLaunchKernelGGL(k_dw1, dim3(1, (unsigned)S), dim3(128), 0, s, dZ, in, st, B, kchunk, ws);
  hipLaunchKernelGGL(k_sum_slices, dim3(1), dim3(256), 0, s, ws, S, kH * 2, out);
}

// One forward + backward pass on a batch (inputs in[B][2], targets T[B][kO];
// with st, the step's slice of the training set starting at in, T): gradients
// into buf.G, loss (mean squared error) into buf.loss and, if not null,
// *loss_out (and the call's loss_out entry of st).
hipError_t sur_forward_backward(const SurBufs& b, const float* in, const float* T, int B, float* loss_out,
                                const SurStep* st, hipStream_t s) {
  const unsigned short* Wh = b.Pb;              // hi halves
  const unsigned short* Wl = b.Pb + kNParams;   // lo halves
  hipLaunchKernelGGL(k_layer1, dim3(nb((int64_t)B * kH, 256)), dim3(256), 0, s, in, st, b.P, B, b.h1, b.h1b, b.h1l);
  // z = h W^T + b: A(m=b,k) = h[b][k]; B(k,n) = W[n][k]; split operands
  gemm(b.h1b, b.h1l, kH, 1, Wh + kOffW2, Wl + kOffW2, 1, kH, b.h2, kH, b.h2b, b.h2l, B, kH, kH, b.P + kOffB2, 1,
       b.wpart, s);
  gemm(b.h2b, b.h2l, kH, 1, Wh + kOffW3, Wl + kOffW3, 1, kH, b.h3, kH, b.h3b, b.h3l, B, kH, kH, b.P + kOffB3, 1,
       b.wpart, s);
  gemm(b.h3b, b.h3l, kH, 1, Wh + kOffW4, Wl + kOffW4, 1, kH, b.y, kO, nullptr, nullptr, B, kO, kH, b.P + kOffB4, 0,
       b.wpart, s);
  hipLaunchKernelGGL(k_loss_grad, dim3(nb((int64_t)B * kO, 256)), dim3(256), 0, s, b.y, T, st, B, b.dy, b.dyb,
                     b.sq);
  hipLaunchKernelGGL(k_sum_partial, dim3(256), dim3(256), 0, s, b.sq, (int64_t)B * kO, b.partial);
  hipLaunchKernelGGL(k_sum_final, dim3(1), dim3(256), 0, s, b.partial, 1.0f / (float)((int64_t)B * kO), b.loss,
                     loss_out, st);
  // backward on the hi halves: layer 4: dW4[o][i] = sum_b dy[b][o] h3[b][i]; db4; dh3 = dy W4
  gemm(b.dyb, nullptr, 1, kO, b.h3b, nullptr, kH, 1, b.G + kOffW4, kH, nullptr, nullptr, kO, kH, B, nullptr, 0,
       b.wpart, s);
  col_sum(b.dy, B, kO, b.G + kOffB4, b.wpart, s);
  gemm(b.dyb, nullptr, kO, 1, Wh + kOffW4, nullptr, kH, 1, b.dh, kH, nullptr, nullptr, B, kH, kO, nullptr, 0, b.wpart,
       s);
  // layers 3 and 2
  const float* Hs[3] = {b.h1, b.h2, b.h3};
  const unsigned short* Hbs[3] = {b.h1b, b.h2b, b.h3b};
  const int offW[2] = {kOffW2, kOffW3}, offB[2] = {kOffB2, kOffB3};
  for (int L = 1; L >= 0; --L) {  // L = 1: layer 3 (input h2, output h3); L = 0: layer 2 (h1 -> h2)
    hipLaunchKernelGGL(k_tanh_back, dim3(nb((int64_t)B * kH, 256)), dim3(256), 0, s, b.dh, Hs[L + 1],
                       (int64_t)B * kH, b.dz, b.dzb);
    gemm(b.dzb, nullptr, 1, kH, Hbs[L], nullptr, kH, 1, b.G + offW[L], kH, nullptr, nullptr, kH, kH, B, nullptr, 0,
         b.wpart, s);
    col_sum(b.dz, B, kH, b.G + offB[L], b.wpart, s);
    // dh_in = dz W: A(m=b, k=j) = dz[b][j]; B(k=j, n=i) = W[j][i]
    gemm(b.dzb, nullptr, kH, 1, Wh + offW[L], nullptr, kH, 1, b.dh, kH, nullptr, nullptr, B, kH, kH, nullptr, 0,
         b.wpart, s);
  }
  // layer 1 (FP32)
  hipLaunchKernelGGL(k_tanh_back, dim3(nb((int64_t)B * kH, 256)), dim3(256), 0, s, b.dh, b.h1, (int64_t)B * kH, b.dz,
                     b.dzb);
  dw1(b.dz, in, st, B, b.G + kOffW1, b.wpart, s);
  col_sum(b.dz, B, kH, b.G + kOffB1, b.wpart, s);
  return hipGetLastError();
}

hipError_t sur_adam(const SurBufs& b, float lr, int step, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(k_adam, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.P, b.G, b.M, b.V, b.Pb, kNParams, lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2, (const SurStep*)nullptr);
  return hipGetLastError();
}

// Start of a training call (the state the step kernels read).
hipError_t sur_train_begin(const SurBufs& b, int64_t step, int64_t nbatches, int total, float lr0, float lrf,
                           float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_train_begin, dim3(1), dim3(1), 0, s, b.st, step, nbatches, total, lr0, lrf, loss_out);
  return hipGetLastError();
}

// One training step on the slice of the training set (in, T) that b.st
// selects: forward + backward, Adam at the scheduled learning rate, advance.
// The same launches at every step (recorded once as a graph by the caller).
hipError_t sur_train_step(const SurBufs& b, const float* in, const float* T, int B, hipStream_t s) {
  hipError_t e = sur_forward_backward(b, in, T, B, nullptr, b.st, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_adam, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.P, b.G, b.M, b.V, b.Pb, kNParams, 0.0f,
                     0.9f, 0.999f, 1e-8f, 1.0f, 1.0f, (const SurStep*)b.st);
  hipLaunchKernelGGL(k_train_advance, dim3(1), dim3(1), 0, s, b.st);
  return hipGetLastError();
}

hipError_t sur_refresh_bf16(const SurBufs& b, hipStream_t s) {
  hipLaunchKernelGGL(k_to_bf16, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.P, b.Pb, kNParams);
  return hipGetLastError();
}

hipError_t sur_prep(const SurDev& S, const MemberDev& m, const double* x, const double* q2, const double* xf,
                    int64_t n, float* in, float* T, unsigned char* keep, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_prep_samples, dim3(nb(n, 256)), dim3(256), 0, s, S, m, x, q2, xf, n, in, T, keep);
  return hipGetLastError();
}

hipError_t sur_gather(const float* in_all, const float* T_all, const int64_t* idx, int64_t n, float* in, float* T,
                      hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_gather_samples, dim3(nb(n, 256)), dim3(256), 0, s, in_all, T_all, idx, n, in, T);
  return hipGetLastError();
}

hipError_t sur_infer(const SurDev& S, const MemberDev& m, const ReqCols& rc, const SurBufs& b, const double* x,
                     const double* q2, int64_t n, float* out, double invL01, unsigned long long* nerr, int n_cu,
                     hipStream_t s) {
  const int64_t tiles = (n + 63) / 64;
  const int waves = sur_infer_waves(S.nx);
  if (waves < 1) return hipErrorInvalidValue;  // envelope tables beyond LDS (the create call bounds nx)
  const size_t shm = sur_infer_shared_bytes(S.nx, waves);
  const int64_t per_cu = std::max<int64_t>(1, (int64_t)(160 * 1024) / (int64_t)shm);
  const int64_t blocks = min((tiles + waves - 1) / waves, (int64_t)n_cu * per_cu);
  if (blocks > 0) {
    hipError_t e = allow_dynamic_lds(reinterpret_cast<const void*>(&k_sur_infer), shm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sur_infer, dim3((unsigned)blocks), dim3(64 * waves), shm, s, S, m, rc, b.Pb, b.P, x, q2, n,
                       out, invL01, nerr);
  }
  return hipGetLastError();
}

}  // namespace pdfmi
