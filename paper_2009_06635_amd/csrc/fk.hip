// FastKernel-style contraction of PDF members with a kernel table (paper
// section 4.3: theory predictions are convolutions of FK tables with PDFs
// evaluated on an x grid; the multi-member form evaluates many replicas at
// once):
//   T[r][d] = sum_k F[r][k] * FK[d][k],   k = (x point i, flavour a) flattened,
// a dense FP64 contraction of the replica matrix F [nrep][K] with the table
// [ndat][K], on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Tiling: a workgroup of 8 waves computes a 64 x 128 tile of T (64 members x
// 128 table rows); each wave a 32 x 32 part as 2 x 2 MFMA tiles of 16 x 16
// (two workgroups per compute unit: 4 waves per SIMD).
// K is walked in steps of 32 staged in LDS as rows of 33 doubles, with the
// next step's global loads (32 consecutive k per half-wave: 256-byte
// segments) issued before the current step's MFMAs.  An operand read (lane =
// row r + 16 k-column q) is served 16 lanes (128 bytes) at a time; with a row
// stride of 33 doubles the 16 rows of one q land on 16 distinct 8-byte bank
// slots (a stride of 36 put rows r and r + 8 on the same slot and cost ~45 %
// of the kernel's cycles in bank conflicts).  Out-of-range rows and k
// read as zero.  K is split into S slices (chosen from the sizes and the
// number of compute units only) whose partial sums are added in slice order,
// so the summation order is fixed (deterministic results).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace pdfmi {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kFkBM = 64, kFkBN = 128, kFkBK = 32, kFkLd = kFkBK + 1, kFkThreads = 512;
constexpr int kFkRowsA = kFkBM * kFkBK / kFkThreads, kFkRowsB = kFkBN * kFkBK / kFkThreads;  // loads per thread

// One (64 x 128 tile, K slice) per workgroup: the slice [blockIdx.z * kslice,
// min(K, (blockIdx.z + 1) * kslice)) of the sum goes to T + blockIdx.z *
// nrep * ndat (the partial sums of the slices are added in slice order by
// k_fk_reduce).
__global__ __launch_bounds__(kFkThreads) void k_fk_contract(const double* __restrict__ F, const double* __restrict__ FK,
                                                            int nrep, int ndat, int64_t K, int64_t kslice,
                                                            double* __restrict__ T) {
  __shared__ double sa[kFkBM * kFkLd];
  __shared__ double sb[kFkBN * kFkLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 2, wn = wave & 3;  // wave part of the tile: rows 32 wm.., columns 32 wn..
  const int m0 = blockIdx.y * kFkBM, n0 = blockIdx.x * kFkBN;
  // cooperative loads: thread -> k = tid % 32 of rows tid / 32 + 16 i
  const int lk = tid & 31, lr = tid >> 5;
  const int64_t kbeg = (int64_t)blockIdx.z * kslice, kend = min(K, kbeg + kslice);
  T += (int64_t)blockIdx.z * nrep * ndat;
  double ra[kFkRowsA], rb[kFkRowsB];
  auto fetch = [&](int64_t k0) {
    const int64_t k = k0 + lk;
    const bool kok = k < kend;
#pragma unroll
    for (int i = 0; i < kFkRowsA; ++i) {
      const int row = m0 + lr + 16 * i;
      ra[i] = (kok && row < nrep) ? F[(int64_t)row * K + k] : 0.0;
    }
#pragma unroll
    for (int i = 0; i < kFkRowsB; ++i) {
      const int row = n0 + lr + 16 * i;
      rb[i] = (kok && row < ndat) ? FK[(int64_t)row * K + k] : 0.0;
    }
  };
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int r16 = lane & 15, kq = lane >> 4;
  fetch(kbeg);
  for (int64_t k0 = kbeg; k0 < kend; k0 += kFkBK) {
    __syncthreads();  // previous step's operands consumed
#pragma unroll
    for (int i = 0; i < kFkRowsA; ++i) sa[(lr + 16 * i) * kFkLd + lk] = ra[i];
#pragma unroll
    for (int i = 0; i < kFkRowsB; ++i) sb[(lr + 16 * i) * kFkLd + lk] = rb[i];
    __syncthreads();
    if (k0 + kFkBK < kend) fetch(k0 + kFkBK);
#pragma unroll
    for (int kk = 0; kk < kFkBK; kk += 4) {
      double a[2], b[2];
#pragma unroll
      for (int t = 0; t < 2; ++t) a[t] = sa[(wm * 32 + t * 16 + r16) * kFkLd + kk + kq];  // A: row r16, k = kq
#pragma unroll
      for (int t = 0; t < 2; ++t) b[t] = sb[(wn * 32 + t * 16 + r16) * kFkLd + kk + kq];  // B: column r16, k = kq
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
  }
  // accumulator layout of the FP64 16x16x4 form: value v of a lane is row
  // lane / 16 + 4 v, column lane % 16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm * 32 + i * 16 + kq + 4 * v;
        const int n = n0 + wn * 32 + j * 16 + r16;
        if (m < nrep && n < ndat) T[(int64_t)m * ndat + n] = acc[i][j][v];
      }
}

// T[m][n] = sum over slices s = 0..S-1 (in that order) of P[s][m][n].
__global__ void k_fk_reduce(const double* __restrict__ P, int S, int64_t mn, double* __restrict__ T) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < mn; i += (int64_t)gridDim.x * blockDim.x) {
    double acc = P[i];
    for (int s = 1; s < S; ++s) acc += P[(int64_t)s * mn + i];
    T[i] = acc;
  }
}

// K slices for a contraction: enough workgroups to cover the compute units
// about four times, each slice a multiple of the K step and at least 512.
int fk_slices(int nrep, int ndat, int64_t K, int n_cu) {
  const int64_t tiles = (int64_t)((ndat + kFkBN - 1) / kFkBN) * ((nrep + kFkBM - 1) / kFkBM);
  int64_t S = (4 * (int64_t)n_cu + tiles - 1) / std::max<int64_t>(tiles, 1);
  S = min(S, std::max<int64_t>(1, K / 512));
  return (int)std::max<int64_t>(1, std::min<int64_t>(S, 64));
}

// Partial sums of the K slices for callers that cannot allocate
// (pdf_fk_contract_noalloc): a fixed array in device memory, one per GPU the
// library runs on, held until the process ends.  Host code never passes the
// array's name to a kernel: fk_scratch_setup looks up its device address once
// per device and the launches take that pointer.
constexpr size_t kFkScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) double scratch[kFkScratchBytes / sizeof(double)];

constexpr int kFkMaxDevices = 64;
static double* g_scratch_ptr[kFkMaxDevices] = {};

size_t fk_scratch_bytes() { return kFkScratchBytes; }

// Device address of the scratch array on `device`, which must be the current
// device; looked up on the first call for that device.
hipError_t fk_scratch_setup(int device, double** out) {
  *out = nullptr;
  if (device < 0 || device >= kFkMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}

// ws: S * nrep * ndat doubles when S > 1 (unused otherwise).
hipError_t launch_fk_contract(const double* F, const double* FK, int nrep, int ndat, int64_t K, double* T, int S,
                              double* ws, hipStream_t s) {
  int64_t kslice = (K + S - 1) / S;
  kslice = (kslice + kFkBK - 1) / kFkBK * kFkBK;
  const dim3 grid((unsigned)((ndat + kFkBN - 1) / kFkBN), (unsigned)((nrep + kFkBM - 1) / kFkBM), (unsigned)S);
  hipLaunchKernelGGL(k_fk_contract, grid, dim3(kFkThreads), 0, s, F, FK, nrep, ndat, K, std::max<int64_t>(kslice, 1),
                     S > 1 ? ws : T);
  if (S > 1) {
    const int64_t mn = (int64_t)nrep * ndat;
    const int64_t nb = std::min<int64_t>((mn + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fk_reduce, dim3((unsigned)nb), dim3(256), 0, s, ws, S, mn, T);
  }
  return hipGetLastError();
}

}  // namespace pdfmi
