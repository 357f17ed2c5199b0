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
// Training is deterministic: every reduction has a fixed order (within a
// 64-row slice of the batch, then the slices in order), so a checkpointed and
// resumed run reproduces a straight run bit for bit.
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
// Training step, fused into two launches.  k_train_fb: one workgroup of four
// waves per 64-row slice of the batch runs the forward and backward passes
// of its rows (wave w owns rows 16 w .. 16 w + 15; hidden activations stay in
// registers and LDS) and writes the slice's gradient and its sum of squared
// errors to the workspace.  k_train_update (k_grad_reduce without the
// update) adds the slices in slice order and applies Adam.
//
// Matrix products on v_mfma_f32_16x16x32_bf16: lane l = 16 g + r holds
// A(row r, k = 8 g .. 8 g + 7) and B(k = 8 g .. 8 g + 7, column r) of a
// 32-deep step and receives C(rows 4 g .. 4 g + 3, column r).  The forward
// products take the three split terms per k step (hi*hi, lo*hi, hi*lo) and
// walk k in order; the backward products multiply BF16 (hi) signals with the
// hi halves.  Weight gradients sum over the slice's 64 rows in two k steps,
// bias gradients (and the FP32 first-layer weight gradient) over each lane's
// four rows, then lanes g = 0..3 of waves 0..3 in that order.
//
// LDS tiles of BF16 with 64 columns are rows of 128 bytes whose 16-byte
// chunks are rotated by (row & 7), so that the 16-byte operand reads of eight
// lanes on consecutive rows hit eight different chunk positions; tiles of 16
// columns (32-byte rows) swap their two chunks on rows 4..7 of every eight.
constexpr int kTRows = 64, kTWaves = 4, kTThreads = 64 * kTWaves;
constexpr int kNPad = (kNParams + 1 + 63) / 64 * 64;  // workspace stride per slice: gradient, then the loss sum

__device__ __forceinline__ int swz64(int row, int col) {
  return row * 128 + ((((col >> 3) ^ row) & 7) << 4) + ((col & 7) << 1);
}
__device__ __forceinline__ int swz16(int row, int col) {
  return row * 32 + ((((col >> 3) ^ (row >> 2)) & 1) << 4) + ((col & 7) << 1);
}
__device__ __forceinline__ bf16x8 ld8(const unsigned char* base, int off) {
  return *reinterpret_cast<const bf16x8*>(base + off);
}
__device__ __forceinline__ void st_bf16(unsigned char* base, int off, unsigned short v) {
  *reinterpret_cast<unsigned short*>(base + off) = v;
}
// four consecutive columns c .. c + 3 (c a multiple of 4) of one row
__device__ __forceinline__ void st4_bf16(unsigned char* base, int off, const unsigned short v[4]) {
  *reinterpret_cast<uint2*>(base + off) =
      make_uint2((unsigned)v[0] | ((unsigned)v[1] << 16), (unsigned)v[2] | ((unsigned)v[3] << 16));
}

// Byte offsets of the LDS regions of k_train_fb.
constexpr int kT64 = 64 * 64 * 2, kT16 = 64 * 16 * 2;
constexpr int kLW2h = 0, kLW2l = kLW2h + kT64, kLW3h = kLW2l + kT64, kLW3l = kLW3h + kT64;  // W[n][k]
constexpr int kLW2t = kLW3l + kT64, kLW3t = kLW2t + kT64;                                   // W^T[k][n], hi
constexpr int kLW4h = kLW3t + kT64, kLW4l = kLW4h + kT16, kLW4t = kLW4l + kT16;           // W4[o][k]; W4^T[k][o]
constexpr int kLAh0 = kLW4t + kT16, kLAl0 = kLAh0 + kT64, kLAh1 = kLAl0 + kT64, kLAl1 = kLAh1 + kT64;  // layer inputs
constexpr int kLH1t = kLAl1 + kT64, kLH2t = kLH1t + kT64, kLH3t = kLH2t + kT64;  // activations^T [unit][row], hi
constexpr int kLDz = kLH3t + kT64, kLDzt = kLDz + kT64;                          // dz [row][unit], dz^T, hi
constexpr int kLDy = kLDzt + kT64, kLDyt = kLDy + kT16;                          // dy [row][o], dy^T [o][row]
constexpr int kLIn = kLDyt + kT16;                                               // in [row][2], FP32
constexpr int kLRed = kLIn + kTRows * 2 * 4;                                     // [3][waves][4][64] FP32
constexpr int kLLoss = kLRed + 3 * kTWaves * 4 * 64 * 4;                         // [threads] FP32
constexpr int kTrainLds = kLLoss + kTThreads * 4;

// The three split products of one 32-deep k step, in the order hi*hi, lo*hi, hi*lo.
__device__ __forceinline__ f32x4 mfma3(bf16x8 a, bf16x8 al, bf16x8 b, bf16x8 bl, f32x4 c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bl, c, 0, 0, 0);
}

// Stores a hidden layer's outputs h (this lane's rows 4 g + i, columns 16 t + r)
// as the next layer's split A operand and as hi^T for the weight gradient.
__device__ __forceinline__ void store_hidden(unsigned char* L, int ah, int al, int ht, int R0, int g, int r,
                                             const float h[4][4]) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    unsigned short hi[4], lo[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      split_bits(h[t][i], hi[i], lo[i]);
      st_bf16(L + ah, swz64(R0 + 4 * g + i, 16 * t + r), hi[i]);
      st_bf16(L + al, swz64(R0 + 4 * g + i, 16 * t + r), lo[i]);
    }
    st4_bf16(L + ht, swz64(16 * t + r, R0 + 4 * g), hi);
  }
}

// Hidden layer 2 or 3 forward: h = tanh(A W^T + b) for this wave's rows.
__device__ __forceinline__ void hidden_fwd(const unsigned char* L, int ah, int al, int wh, int wl,
                                           const float* __restrict__ bias, int R0, int g, int r, float h[4][4]) {
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < kH; k0 += 32) {
    const bf16x8 a = ld8(L + ah, swz64(R0 + r, k0 + 8 * g)), a2 = ld8(L + al, swz64(R0 + r, k0 + 8 * g));
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = mfma3(a, a2, ld8(L + wh, swz64(16 * t + r, k0 + 8 * g)), ld8(L + wl, swz64(16 * t + r, k0 + 8 * g)),
                     acc[t]);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const float bv = bias[16 * t + r];
#pragma unroll
    for (int i = 0; i < 4; ++i) h[t][i] = tanh_f(acc[t][i] + bv);
  }
}

// Weight gradient of a 64-unit layer for output units 16 w .. 16 w + 15:
// dW[j][i] = sum over the slice's rows of dz[b][j] h[b][i] (hi operands).
__device__ __forceinline__ void weight_grad(const unsigned char* L, int dzt, int ht, int w, int g, int r,
                                            float* __restrict__ out) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < kTRows; k0 += 32)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(L + dzt, swz64(16 * w + r, k0 + 8 * g)),
                                                    ld8(L + ht, swz64(16 * t + r, k0 + 8 * g)), acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(16 * w + 4 * g + i) * kH + 16 * t + r] = acc[i];
  }
}

// dh = dz W for this wave's rows (K = the 64 output units, W^T staged).
__device__ __forceinline__ void input_grad(const unsigned char* L, int dz, int wt, int R0, int g, int r,
                                           float dh[4][4]) {
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k0 = 0; k0 < kH; k0 += 32) {
    const bf16x8 a = ld8(L + dz, swz64(R0 + r, k0 + 8 * g));
#pragma unroll
    for (int t = 0; t < 4; ++t)
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, ld8(L + wt, swz64(16 * t + r, k0 + 8 * g)), acc[t], 0, 0,
                                                       0);
  }
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) dh[t][i] = acc[t][i];
}

// dz = dh (1 - h^2) (tanh derivative) into dh; its hi halves to the dz and
// dz^T tiles; this lane's sum over its four rows of each column to red[w][g].
__device__ __forceinline__ void tanh_back(unsigned char* L, float* red, const float h[4][4], float dh[4][4],
                                          int R0, int w, int g, int r) {
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    unsigned short hi[4];
    float s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      dh[t][i] = dh[t][i] * (1.0f - h[t][i] * h[t][i]);
      hi[i] = bf16_bits(dh[t][i]);
      st_bf16(L + kLDz, swz64(R0 + 4 * g + i, 16 * t + r), hi[i]);
      s += dh[t][i];
    }
    st4_bf16(L + kLDzt, swz64(16 * t + r, R0 + 4 * g), hi);
    red[(w * 4 + g) * 64 + 16 * t + r] = s;
  }
}

// Column c's sum of red[w][g][c] over w = 0..3, g = 0..3 in that order.
__device__ __forceinline__ float red_sum(const float* red, int c) {
  float s = red[c];
#pragma unroll
  for (int q = 1; q < kTWaves * 4; ++q) s += red[q * 64 + c];
  return s;
}

// Batch slice of a training step: rows (step % nb) * B of the training set
// when st is given (in and T are then the set's first rows), else as passed.
__device__ __forceinline__ int64_t batch_row(const SurStep* st, int B) {
  return st ? (st->step % st->nb) * (int64_t)B : 0;
}

__global__ __launch_bounds__(kTThreads) void k_train_fb(const float* __restrict__ in, const float* __restrict__ T,
                                                        const SurStep* __restrict__ st, const float* __restrict__ P,
                                                        const unsigned short* __restrict__ Pb, int B,
                                                        float* __restrict__ ws) {
  extern __shared__ __align__(16) unsigned char L[];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, r = lane & 15, g = lane >> 4;
  const int R0 = 16 * w;
  const int64_t row0 = batch_row(st, B) + (int64_t)blockIdx.x * kTRows;
  const int nrow = min(kTRows, B - (int)blockIdx.x * kTRows);  // valid rows of this slice
  float* out = ws + (int64_t)blockIdx.x * kNPad;
  float* red = reinterpret_cast<float*>(L + kLRed);

  // stage the weights: split W2, W3, W4 row-major; hi of W2^T, W3^T, W4^T
  {
    const unsigned short* Wh = Pb;
    const unsigned short* Wl = Pb + kNParams;
    for (int c = tid; c < 64 * 8; c += kTThreads) {  // 16-byte chunks of the 64 x 64 matrices
      const int n = c >> 3, k = (c & 7) * 8;
      const uint4 w2h = *reinterpret_cast<const uint4*>(Wh + kOffW2 + n * kH + k);
      const uint4 w3h = *reinterpret_cast<const uint4*>(Wh + kOffW3 + n * kH + k);
      *reinterpret_cast<uint4*>(L + kLW2h + swz64(n, k)) = w2h;
      *reinterpret_cast<uint4*>(L + kLW2l + swz64(n, k)) = *reinterpret_cast<const uint4*>(Wl + kOffW2 + n * kH + k);
      *reinterpret_cast<uint4*>(L + kLW3h + swz64(n, k)) = w3h;
      *reinterpret_cast<uint4*>(L + kLW3l + swz64(n, k)) = *reinterpret_cast<const uint4*>(Wl + kOffW3 + n * kH + k);
      const unsigned short* e2 = reinterpret_cast<const unsigned short*>(&w2h);
      const unsigned short* e3 = reinterpret_cast<const unsigned short*>(&w3h);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        st_bf16(L + kLW2t, swz64(k + q, n), e2[q]);
        st_bf16(L + kLW3t, swz64(k + q, n), e3[q]);
      }
    }
    for (int c = tid; c < kO * 8; c += kTThreads) {  // W4: 16 rows of 8 chunks
      const int o = c >> 3, k = (c & 7) * 8;
      const uint4 w4h = *reinterpret_cast<const uint4*>(Wh + kOffW4 + o * kH + k);
      *reinterpret_cast<uint4*>(L + kLW4h + swz64(o, k)) = w4h;
      *reinterpret_cast<uint4*>(L + kLW4l + swz64(o, k)) = *reinterpret_cast<const uint4*>(Wl + kOffW4 + o * kH + k);
      const unsigned short* e4 = reinterpret_cast<const unsigned short*>(&w4h);
#pragma unroll
      for (int q = 0; q < 8; ++q) st_bf16(L + kLW4t, swz16(k + q, o), e4[q]);
    }
    float* sin = reinterpret_cast<float*>(L + kLIn);
    if (tid < 2 * kTRows) sin[tid] = tid < 2 * nrow ? in[2 * row0 + tid] : 0.0f;
  }
  __syncthreads();
  const float* sin = reinterpret_cast<const float*>(L + kLIn);

  // layer 1 (FP32): h1[b][j] = tanh(W1[j][0] in[b][0] + W1[j][1] in[b][1] + b1[j])
  float h1[4][4], h2[4][4], h3[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int j = 16 * t + r;
    const float w0 = P[kOffW1 + 2 * j], w1 = P[kOffW1 + 2 * j + 1], bj = P[kOffB1 + j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = R0 + 4 * g + i;
      h1[t][i] = tanh_f(fmaf(w0, sin[2 * b], fmaf(w1, sin[2 * b + 1], bj)));
    }
  }
  store_hidden(L, kLAh0, kLAl0, kLH1t, R0, g, r, h1);
  __syncthreads();
  hidden_fwd(L, kLAh0, kLAl0, kLW2h, kLW2l, P + kOffB2, R0, g, r, h2);
  store_hidden(L, kLAh1, kLAl1, kLH2t, R0, g, r, h2);
  __syncthreads();
  hidden_fwd(L, kLAh1, kLAl1, kLW3h, kLW3l, P + kOffB3, R0, g, r, h3);
  store_hidden(L, kLAh0, kLAl0, kLH3t, R0, g, r, h3);
  __syncthreads();

  // layer 4 and the loss: y = h3 W4^T + b4; d = y - T; dy = 2 d / (B kO)
  {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < kH; k0 += 32)
      acc = mfma3(ld8(L + kLAh0, swz64(R0 + r, k0 + 8 * g)), ld8(L + kLAl0, swz64(R0 + r, k0 + 8 * g)),
                  ld8(L + kLW4h, swz64(r, k0 + 8 * g)), ld8(L + kLW4l, swz64(r, k0 + 8 * g)), acc);
    const float bo = P[kOffB4 + r];
    const float scale = (float)((int64_t)B * kO);
    unsigned short hi[4];
    float sq = 0.0f, s = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = R0 + 4 * g + i;
      const float d = b < nrow ? (acc[i] + bo) - T[(row0 + b) * kO + r] : 0.0f;
      const float gr = 2.0f * d / scale;
      hi[i] = bf16_bits(gr);
      st_bf16(L + kLDy, swz16(b, r), hi[i]);
      sq += d * d;
      s += gr;
    }
    st4_bf16(L + kLDyt, swz64(r, R0 + 4 * g), hi);
    red[(w * 4 + g) * 64 + r] = s;
    reinterpret_cast<float*>(L + kLLoss)[tid] = sq;
  }
  __syncthreads();

  // layer 4 backward: dW4 (wave w: input units 16 w ..), db4, dh3 = dy W4
  {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k0 = 0; k0 < kTRows; k0 += 32)
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(L + kLDyt, swz64(r, k0 + 8 * g)),
                                                    ld8(L + kLH3t, swz64(R0 + r, k0 + 8 * g)), acc, 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i) out[kOffW4 + (4 * g + i) * kH + R0 + r] = acc[i];
  }
  if (tid < kO) out[kOffB4 + tid] = red_sum(red, tid);
  if (tid == 0) {
    const float* ls = reinterpret_cast<const float*>(L + kLLoss);
    float s = ls[0];
    for (int q = 1; q < kTThreads; ++q) s += ls[q];
    out[kNParams] = s;
  }
  float dh[4][4];
  {
    const bf16x8 zero = {};
    const bf16x8 a = g < 2 ? ld8(L + kLDy, swz16(R0 + r, 8 * g)) : zero;  // K = 16 of 32
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf16x8 bw = g < 2 ? ld8(L + kLW4t, swz16(16 * t + r, 8 * g)) : zero;
      const f32x4 acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bw, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
#pragma unroll
      for (int i = 0; i < 4; ++i) dh[t][i] = acc[i];
    }
  }
  __syncthreads();  // red and the loss sums consumed

  // layer 3 backward
  tanh_back(L, red, h3, dh, R0, w, g, r);
  __syncthreads();
  weight_grad(L, kLDzt, kLH2t, w, g, r, out + kOffW3);
  if (tid < kH) out[kOffB3 + tid] = red_sum(red, tid);
  input_grad(L, kLDz, kLW3t, R0, g, r, dh);
  __syncthreads();
  // layer 2 backward
  tanh_back(L, red, h2, dh, R0, w, g, r);
  __syncthreads();
  weight_grad(L, kLDzt, kLH1t, w, g, r, out + kOffW2);
  if (tid < kH) out[kOffB2 + tid] = red_sum(red, tid);
  input_grad(L, kLDz, kLW2t, R0, g, r, dh);
  __syncthreads();
  // layer 1 backward (FP32): dW1[j][t] = sum_b dz[b][j] in[b][t], db1
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    float s0 = 0.0f, s1 = 0.0f, sb = 0.0f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int b = R0 + 4 * g + i;
      const float dz = dh[t][i] * (1.0f - h1[t][i] * h1[t][i]);
      s0 = fmaf(dz, sin[2 * b], s0);
      s1 = fmaf(dz, sin[2 * b + 1], s1);
      sb += dz;
    }
    const int q = (w * 4 + g) * 64 + 16 * t + r;
    red[q] = s0;
    red[kTWaves * 4 * 64 + q] = s1;
    red[2 * kTWaves * 4 * 64 + q] = sb;
  }
  __syncthreads();
  if (tid < kH) {
    out[kOffW1 + 2 * tid] = red_sum(red, tid);
    out[kOffW1 + 2 * tid + 1] = red_sum(red + kTWaves * 4 * 64, tid);
    out[kOffB1 + tid] = red_sum(red + 2 * kTWaves * 4 * 64, tid);
  }
}

// Adam step of parameter i (Kingma & Ba, bias-corrected moments; c1 = 1 -
// b1^t, c2 = 1 - b2^t for update number t), then its BF16 pair.
__device__ __forceinline__ void adam_update(int i, int n, float g, float lr, float b1, float b2, float eps, float c1,
                                            float c2, float* __restrict__ P, float* __restrict__ Mm,
                                            float* __restrict__ Vm, unsigned short* __restrict__ Pb) {
  const float m = b1 * Mm[i] + (1.0f - b1) * g;
  const float v = b2 * Vm[i] + (1.0f - b2) * g * g;
  Mm[i] = m;
  Vm[i] = v;
  const float p = P[i] - lr * (m / c1) / (sqrtf(v / c2) + eps);
  P[i] = p;
  split_bits(p, Pb[i], Pb[n + i]);
}

// Learning rate and bias corrections of update number st->step + 1: cosine
// schedule lrf + (lr0 - lrf)(1 + cos(pi min(1, step / total))) / 2; the
// betas' powers in FP64, as the host computes them.
__device__ __forceinline__ void schedule(const SurStep* st, float& lr, float& c1, float& c2) {
  const double t = (double)st->step;
  const double frac = fmin(1.0, t / (double)st->total);
  lr = (float)(st->lrf + 0.5 * ((double)st->lr0 - st->lrf) * (1.0 + cos(3.141592653589793 * frac)));
  c1 = (float)(1.0 - pow(0.9, t + 1.0));
  c2 = (float)(1.0 - pow(0.999, t + 1.0));
}

// Adam with a given gradient G (pdf_surrogate_adam).
__global__ void k_adam(float* __restrict__ P, const float* __restrict__ G, float* __restrict__ Mm,
                       float* __restrict__ Vm, unsigned short* __restrict__ Pb, int n, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) adam_update(i, n, G[i], lr, b1, b2, eps, c1, c2, P, Mm, Vm, Pb);
}

// Gradient i = sum over the S slices of the workspace, in slice order.
__device__ __forceinline__ float slice_sum(const float* __restrict__ ws, int S, int i) {
  float g = ws[i];
  for (int q = 1; q < S; ++q) g += ws[(int64_t)q * kNPad + i];
  return g;
}

// The gradient and loss of k_train_fb's slices (no update).
__global__ __launch_bounds__(256) void k_grad_reduce(const float* __restrict__ ws, int S, float* __restrict__ G,
                                                     float inv_n, float* __restrict__ loss,
                                                     float* __restrict__ loss_out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNParams) G[i] = slice_sum(ws, S, i);
  if (i == 0) {
    const float l = slice_sum(ws, S, kNParams) * inv_n;
    *loss = l;
    if (loss_out) *loss_out = l;
  }
}

// Gradient of the slices, Adam at the scheduled rate, and -- in the last
// workgroup to finish -- the step's loss and the advance of the step state.
__global__ __launch_bounds__(256) void k_train_update(const float* __restrict__ ws, int S, float* __restrict__ P,
                                                      float* __restrict__ G, float* __restrict__ Mm,
                                                      float* __restrict__ Vm, unsigned short* __restrict__ Pb,
                                                      float inv_n, float* __restrict__ loss, SurStep* st) {
  __shared__ int last;
  float lr, c1, c2;
  schedule(st, lr, c1, c2);
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < kNParams) {
    const float g = slice_sum(ws, S, i);
    G[i] = g;
    adam_update(i, kNParams, g, lr, 0.9f, 0.999f, 1e-8f, c1, c2, P, Mm, Vm, Pb);
  }
  __syncthreads();  // every thread of this workgroup has read the step state
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&st->done, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    const float l = slice_sum(ws, S, kNParams) * inv_n;
    *loss = l;
    if (st->loss_out) st->loss_out[st->call] = l;
    st->step += 1;
    st->call += 1;
    st->done = 0;
  }
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
  st->done = 0;
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
// the network runs on four 16-point sub-tiles with the activations kept in
// registers from layer to layer.  Each layer is formed transposed on the
// matrix cores, h' = tanh(W h + b) with the weights as the A operand and the
// 16 points' activations as the B operand, three products per operand pair:
// lane (r, g) then receives units 16 t + 4 g + i (t, i = 0..3) of point r,
// which are the 16 values it supplies to the next layer's B operand when
// that layer's 64-deep k index k' = 32 s + 8 g + i stands for unit
// kunit(k') = 16 (2 s + i / 4) + 4 g + i % 4.  The weight columns are staged
// in LDS in that order (once per workgroup), so no activation passes through
// LDS.  Layer 1 (two inputs) runs on the VALUs straight into that layout.
// The outputs times the envelope go to a 16 x 16 LDS tile from which the
// requested columns are stored point-major, consecutive lanes on consecutive
// values.  Points in the fallback domain are queued per wave and evaluated
// 64 at a time by the FP32 interpolator: each is located once (one lane per
// point: sub-grid, cells, weights), after which one lane per (point,
// requested column) gathers its 4x4 stencil.
//
// LDS rows of 64 BF16 values (the weight halves) hold their eight 16-byte
// chunks in the order chunk ^ (row & 7), so the 16 rows an operand read
// touches spread over the banks.  Blocks of 16 waves fill the CU's LDS
// (4 waves per SIMD, at most 128 VGPRs).
constexpr int kSurWaves = 16;
constexpr int kSurRec = 8;   // floats per point record: u, v, h00, h10 D, h01, h11 D, cell, fallback

__device__ __forceinline__ int swz(int row, int col) {  // element offset of (row, col) in a swizzled [.][64] tile
  return row * kH + ((((col >> 3) ^ row) & 7) << 3) + (col & 7);
}
// Hidden unit that the k index k' of a layer's B operand stands for (see above).
__device__ __forceinline__ int kunit(int kp) {
  return ((kp >> 5) << 5) + (((kp >> 2) & 1) << 4) + (((kp >> 3) & 3) << 2) + (kp & 3);
}

// Location of one fallback point (what interp_point derives before its gathers).
struct FbRec {
  float w[4], v[4];
  int base, sa, mode, pt;  // grid offset and x stride (elements), region bits, slot in the wave's queue
  double p0, p1;           // extrapolation parameters
};

// LDS of k_sur_infer: the lo and hi halves of W2, W3 (64 x 64) and W4
// (16 x 64) with their columns in kunit order, [nx] ln x knots (double),
// [nx][16] envelope values and slopes, W1 and b1-b3 times 2 log2(e) (the
// argument scale of tanh_scaled), b4; then per wave a 5 KB area (4 KB for
// the output tile, later the fallback records; 1 KB for the fallback queue)
// and the point records.
constexpr size_t kSurWaveArea = 4096 + 128 * 8;  // output tile or fallback records, then the fallback queue
constexpr size_t kSurWTile = (size_t)2 * (2 * kH * kH + kO * kH);  // one half of W2, W3, W4 (BF16)
__host__ __device__ static inline size_t sur_head_bytes(int nx) {
  const size_t b = 2 * kSurWTile + (size_t)8 * nx +
                   (size_t)4 * (2 * nx * kO + 2 * kH + 3 * kH + kO + kMaxReq);
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

__global__ __launch_bounds__(64 * kSurWaves) __attribute__((amdgpu_waves_per_eu(4)))
void k_sur_infer(SurDev S, MemberDev m, ReqCols rc, const unsigned short* __restrict__ Pb,
                 const float* __restrict__ Pf, const double* __restrict__ X, const double* __restrict__ Q2,
                 int64_t n, float* __restrict__ out, double invL01, unsigned long long* __restrict__ nerr) {
  extern __shared__ __align__(16) unsigned char sraw[];
  const int BS = blockDim.x, nwav = BS >> 6;
  unsigned short* sw2l = reinterpret_cast<unsigned short*>(sraw);  // [kH][kH] swizzled (16-byte chunks)
  unsigned short* sw3l = sw2l + kH * kH;
  unsigned short* sw4l = sw3l + kH * kH;                   // [kO][kH] swizzled
  unsigned short* sw2h = sw4l + kO * kH;                   // hi halves, same layout
  unsigned short* sw3h = sw2h + kH * kH;
  unsigned short* sw4h = sw3h + kH * kH;
  double* slxk = reinterpret_cast<double*>(sw4h + kO * kH);  // [nx]
  float* senv = reinterpret_cast<float*>(slxk + S.nx);     // [nx][kO]
  float* senvd = senv + S.nx * kO;                         // [nx][kO]
  float* sw1 = senvd + S.nx * kO;                          // [kH][2]
  float* sb1 = sw1 + 2 * kH;
  float* sb2 = sb1 + kH;
  float* sb3 = sb2 + kH;
  float* sb4 = sb3 + kH;                                   // [kO]
  int* scol = reinterpret_cast<int*>(sb4 + kO);            // [kMaxReq] stored column of each requested flavour
  unsigned char* waves = sraw + sur_head_bytes(S.nx);
  const int l = threadIdx.x & 63, wv = threadIdx.x >> 6, r = l & 15, g = l >> 4;
  unsigned char* area = waves + (size_t)wv * kSurWaveArea;
  float* so = reinterpret_cast<float*>(area);                         // [16][kO] output tile
  FbRec* fbr = reinterpret_cast<FbRec*>(area);                        // [64] fallback records
  int64_t* fq = reinterpret_cast<int64_t*>(area + 4096);              // [128] queued fallback points
  static_assert(64 * sizeof(FbRec) <= 4096, "fallback records fit the wave area");
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
  for (int i = threadIdx.x; i < rc.n; i += BS) scol[i] = rc.col[i];
  const unsigned short* Pl = Pb + kNParams;  // lo halves
  for (int i = threadIdx.x; i < kH * kH; i += BS) {  // stored column kp of row n holds W[n][kunit(kp)]
    const int row = i / kH, kp = i % kH, src = row * kH + kunit(kp);
    sw2l[swz(row, kp)] = Pl[kOffW2 + src];
    sw3l[swz(row, kp)] = Pl[kOffW3 + src];
    sw2h[swz(row, kp)] = Pb[kOffW2 + src];
    sw3h[swz(row, kp)] = Pb[kOffW3 + src];
  }
  for (int i = threadIdx.x; i < kO * kH; i += BS) {
    const int row = i / kH, kp = i % kH, src = row * kH + kunit(kp);
    sw4l[swz(row, kp)] = Pl[kOffW4 + src];
    sw4h[swz(row, kp)] = Pb[kOffW4 + src];
  }
  __syncthreads();

  // an 8-value chunk (16 bytes) of a swizzled LDS row, as an operand fragment
  auto frag = [&](const unsigned short* tile, int row, int col0) -> bf16x8 {
    return *reinterpret_cast<const bf16x8*>(tile + swz(row, col0));
  };
  const Tables gtb{m.knots, m.cells, m.hints, m.subs};
  const float* __restrict__ gvals = member_values<float>(m);
  const int R = rc.n;

  const int64_t ntiles = (n + 63) / 64;
  int qn = 0;  // queued fallback points of this wave (fewer than 64 between tiles)
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
      // layer 1 straight into the B layout: lane (r, g) holds unit kunit(32 s + 8 g + i) of point q0 + r
      const float u = rec[(q0 + r) * kSurRec], v = rec[(q0 + r) * kSurRec + 1];
      bf16x8 bh[2], bl[2];
#pragma unroll
      for (int s = 0; s < 2; ++s)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          const int j = kunit(32 * s + 8 * g + i);
          unsigned short hb, lb;
          split_bits(tanh_scaled(fmaf(sw1[2 * j], u, fmaf(sw1[2 * j + 1], v, sb1[j]))), hb, lb);
          bh[s][i] = __builtin_bit_cast(__bf16, hb);
          bl[s][i] = __builtin_bit_cast(__bf16, lb);
        }
      // layers 2 and 3: lane (r, g) receives units 16 t + 4 g + i of point q0 + r
#pragma unroll
      for (int layer = 0; layer < 2; ++layer) {
        const float* bias = layer == 0 ? sb2 : sb3;
        const unsigned short* wh = layer == 0 ? sw2h : sw3h;
        const unsigned short* wl = layer == 0 ? sw2l : sw3l;
        float h[4][4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const bf16x8 ah = frag(wh, 16 * t + r, 32 * s + 8 * g);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[s], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[s], acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(wl, 16 * t + r, 32 * s + 8 * g), bh[s], acc, 0, 0, 0);
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) h[t][i] = tanh_scaled(fmaf(acc[i], kTwoLog2e, bias[16 * t + 4 * g + i]));
        }
        // the next layer's B operand: k' = 32 s + 8 g + i is unit 16 (2 s + i / 4) + 4 g + i % 4
#pragma unroll
        for (int s = 0; s < 2; ++s)
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            unsigned short hb, lb;
            split_bits(h[2 * s + (i >> 2)][i & 3], hb, lb);
            bh[s][i] = __builtin_bit_cast(__bf16, hb);
            bl[s][i] = __builtin_bit_cast(__bf16, lb);
          }
      }
      // layer 4: lane (r, g) gets y[output 4 g + i][point q0 + r]; times the envelope into the output tile
      f32x4 y = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 ah = frag(sw4h, r, 32 * s + 8 * g);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh[s], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl[s], y, 0, 0, 0);
        y = __builtin_amdgcn_mfma_f32_16x16x32_bf16(frag(sw4l, r, 32 * s + 8 * g), bh[s], y, 0, 0, 0);
      }
      {
        const float* pq = rec + (q0 + r) * kSurRec;
        const int ei = __float_as_int(pq[6]);
        float yo[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 4 * g + i;
          yo[i] = (y[i] + sb4[c]) * env_at(senv, senvd, ei, pq[2], pq[3], pq[4], pq[5], c);
        }
        *reinterpret_cast<float4*>(so + r * kO + 4 * g) = make_float4(yo[0], yo[1], yo[2], yo[3]);
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      // requested columns of the network's points, point-major
      const int nq = min(16, np - q0);
      // lane (point l / 16 + 4 k, requested flavour j0 + l % 16), flavours in chunks of 16: no division
      for (int j0 = 0; j0 < R; j0 += 16) {
        const int j = j0 + (l & 15);
        const int c = j < R ? scol[j] : -1;
        for (int pt = l >> 4; pt < nq; pt += 4)
          if (j < R && rec[(q0 + pt) * kSurRec + 7] == 0.0f)
            out[(p0 + q0 + pt) * R + j] = c >= 0 ? so[pt * kO + c] : 0.0f;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // fallback points: queued, and evaluated 64 at a time (one lane per point
    // locates it, then one lane per (point, requested column) gathers), so the
    // location runs on full waves rather than on the few fallback lanes of
    // every tile
    if (fb) fq[qn + __popcll(fbmask & ((1ull << l) - 1))] = p0 + l;
    qn += __popcll(fbmask);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const bool last = tile + (int64_t)gridDim.x * nwav >= ntiles;
    while (qn >= 64 || (last && qn > 0)) {
      const int nfb = min(qn, 64);
      bool bad = false;
      if (l < nfb) {
        FbRec& fr = fbr[l];
        const int64_t pi = fq[l];
        const PointLoc L = locate_point<float>(m, gtb, X[pi], Q2[pi], fr.w, fr.v);
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
        const int c = scol[j];
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
        out[fq[fr.pt] * R + j] = val;
      }
      // the rest of the queue (fewer than 64) to its front: the two ranges do not overlap
      const int rest = qn - nfb;
      const int64_t mv = l < rest ? fq[nfb + l] : 0;
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      if (l < rest) fq[l] = mv;
      qn = rest;
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

// Slices of a batch of B rows in the fused training step, and the workspace
// (floats) their partial gradients and losses take.
int sur_slices(int B) { return (B + kTRows - 1) / kTRows; }
size_t sur_workspace_floats(int B) { return (size_t)sur_slices(B) * kNPad; }

// LDS limit of the fused step; called before a step is first launched or recorded.
hipError_t sur_train_prepare() {
  return allow_dynamic_lds(reinterpret_cast<const void*>(&k_train_fb), kTrainLds);
}

// One forward + backward pass on a batch (inputs in[B][2], targets T[B][kO])
// with no update: gradient into buf.G, loss (mean squared error) into
// buf.loss and, if not null, *loss_out.
hipError_t sur_forward_backward(const SurBufs& b, const float* in, const float* T, int B, float* loss_out,
                                hipStream_t s) {
  hipError_t e = sur_train_prepare();
  if (e != hipSuccess) return e;
  const int S = sur_slices(B);
  hipLaunchKernelGGL(k_train_fb, dim3((unsigned)S), dim3(kTThreads), kTrainLds, s, in, T, (const SurStep*)nullptr,
                     b.P, b.Pb, B, b.wpart);
  hipLaunchKernelGGL(k_grad_reduce, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.wpart, S, b.G,
                     1.0f / (float)((int64_t)B * kO), b.loss, loss_out);
  return hipGetLastError();
}

hipError_t sur_adam(const SurBufs& b, float lr, int step, hipStream_t s) {
  const double b1 = 0.9, b2 = 0.999;
  const float c1 = (float)(1.0 - pow(b1, step)), c2 = (float)(1.0 - pow(b2, step));
  hipLaunchKernelGGL(k_adam, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.P, b.G, b.M, b.V, b.Pb, kNParams, lr,
                     (float)b1, (float)b2, 1e-8f, c1, c2);
  return hipGetLastError();
}

// Start of a training call (the state the step kernels read).
hipError_t sur_train_begin(const SurBufs& b, int64_t step, int64_t nbatches, int total, float lr0, float lrf,
                           float* loss_out, hipStream_t s) {
  hipLaunchKernelGGL(k_train_begin, dim3(1), dim3(1), 0, s, b.st, step, nbatches, total, lr0, lrf, loss_out);
  return hipGetLastError();
}

// One training step on the slice of the training set (in, T) that b.st
// selects: the fused forward + backward pass, then the slice sums, Adam at
// the scheduled learning rate and the step advance.  The same two launches
// at every step (recorded once as a graph by the caller); sur_train_prepare
// must have run.
hipError_t sur_train_step(const SurBufs& b, const float* in, const float* T, int B, hipStream_t s) {
  const int S = sur_slices(B);
  hipLaunchKernelGGL(k_train_fb, dim3((unsigned)S), dim3(kTThreads), kTrainLds, s, in, T, (const SurStep*)b.st, b.P,
                     b.Pb, B, b.wpart);
  hipLaunchKernelGGL(k_train_update, dim3(nb(kNParams, 256)), dim3(256), 0, s, b.wpart, S, b.P, b.G, b.M, b.V, b.Pb,
                     1.0f / (float)((int64_t)B * kO), b.loss, b.st);
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
