// FastKernel-style contraction of PDF members with a kernel table (paper
// section 4.3: theory predictions are convolutions of FK tables with PDFs
// evaluated on an x grid; the multi-member form evaluates many replicas at
// once):
//   T[r][d] = sum_k F[r][k] * FK[d][k],   k = (x point i, flavour a) flattened,
// a dense FP64 contraction of the replica matrix F [nrep][K] with the table
// [ndat][K], on the FP64 matrix cores (v_mfma_f64_16x16x4_f64).
//
// Tiling: a workgroup of 8 waves computes a BM x 128 tile of T (BM = 64 or
// 80 members, whichever pads the member count less, x 128 table rows); wave w
// owns table rows 16 w .. 16 w + 15 of the tile against all BM members, as
// BM / 16 MFMA tiles of 16 x 16 sharing one B operand per k step.  The kernel
// is held to 128 VGPRs so two workgroups share a compute unit (4 waves per
// SIMD).
// K is walked in steps of 32 staged in LDS as rows of 33 doubles, with the
// next step's global loads (32 consecutive k per half-wave: 256-byte
// segments; one pointer per operand advanced by 32 each step, row i of a
// thread 16 i K further) issued before the current step's MFMAs.  An operand
// read (lane = row r + 16 k-column q) is served 16 lanes (128 bytes) at a
// time; with a row stride of 33 doubles the 16 rows of one q land on 16
// distinct 8-byte bank slots (a stride of 36 put rows r and r + 8 on the
// same slot and cost ~45 % of the kernel's cycles in bank conflicts).
// Out-of-range rows and k read as zero.  K is split into S slices whose
// partial sums are added in slice order, so the summation order is fixed
// (deterministic results); S is chosen from the sizes and the number of
// compute units only, to fill the two workgroup slots of every compute unit
// evenly (a launch of 520 workgroups on 512 slots ran 25 % slower than one of
// 480).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace pdfmi {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kFkBN = 128, kFkBK = 32, kFkLd = kFkBK + 1, kFkThreads = 512;
constexpr int kFkSlotsPerCu = 2;  // resident workgroups per compute unit (LDS and the 128-VGPR bound)

// One (BM x 128 tile, K slice) per workgroup, BM = 16 MT: the slice
// [blockIdx.z * kslice, min(K, (blockIdx.z + 1) * kslice)) of the sum goes to
// T + blockIdx.z * nrep * ndat (the partial sums of the slices are added in
// slice order by k_fk_reduce).
template <int MT>
__global__ __launch_bounds__(kFkThreads) __attribute__((amdgpu_waves_per_eu(4, 4))) void k_fk_contract(
    const double* __restrict__ F, const double* __restrict__ FK, int nrep, int ndat, int64_t K, int64_t kslice,
    double* __restrict__ T) {
  constexpr int BM = 16 * MT;
  constexpr int kRowsA = BM * kFkBK / kFkThreads, kRowsB = kFkBN * kFkBK / kFkThreads;  // loads per thread
  __shared__ double sa[BM * kFkLd];
  __shared__ double sb[kFkBN * kFkLd];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * kFkBN;
  // cooperative loads: thread -> k = tid % 32 of rows tid / 32 + 16 i
  const int lk = tid & 31, lr = tid >> 5;
  const int64_t kbeg = (int64_t)blockIdx.z * kslice, kend = min(K, kbeg + kslice);
  T += (int64_t)blockIdx.z * nrep * ndat;
  const double* pa = F + (int64_t)(m0 + lr) * K + kbeg + lk;
  const double* pb = FK + (int64_t)(n0 + lr) * K + kbeg + lk;
  const int64_t rs = 16 * K;                             // 16 rows further
  const int na = nrep - m0 - lr, nb = ndat - n0 - lr;  // row i of the thread exists when 16 i < na (nb)
  int64_t krem = kend - kbeg - lk;                       // its k exists while krem > 0
  double ra[kRowsA], rb[kRowsB];
  auto fetch = [&]() {
    const bool kok = krem > 0;
#pragma unroll
    for (int i = 0; i < kRowsA; ++i) ra[i] = (kok && 16 * i < na) ? pa[i * rs] : 0.0;
#pragma unroll
    for (int i = 0; i < kRowsB; ++i) rb[i] = (kok && 16 * i < nb) ? pb[i * rs] : 0.0;
    pa += kFkBK;
    pb += kFkBK;
    krem -= kFkBK;
  };
  f64x4 acc[MT];
#pragma unroll
  for (int t = 0; t < MT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  const int r16 = lane & 15, kq = lane >> 4;
  fetch();
  for (int64_t k0 = kbeg; k0 < kend; k0 += kFkBK) {
    __syncthreads();  // previous step's operands consumed
#pragma unroll
    for (int i = 0; i < kRowsA; ++i) sa[(lr + 16 * i) * kFkLd + lk] = ra[i];
#pragma unroll
    for (int i = 0; i < kRowsB; ++i) sb[(lr + 16 * i) * kFkLd + lk] = rb[i];
    __syncthreads();
    if (k0 + kFkBK < kend) fetch();
#pragma unroll
    for (int kk = 0; kk < kFkBK; kk += 4) {
      const double b = sb[(wave * 16 + r16) * kFkLd + kk + kq];  // B: column r16, k = kq
      double a[MT];
#pragma unroll
      for (int t = 0; t < MT; ++t) a[t] = sa[(t * 16 + r16) * kFkLd + kk + kq];  // A: row r16, k = kq
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], b, acc[t], 0, 0, 0);
    }
  }
  // accumulator layout of the FP64 16x16x4 form: value v of a lane is row
  // lane / 16 + 4 v, column lane % 16
#pragma unroll
  for (int t = 0; t < MT; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + t * 16 + kq + 4 * v;
      const int n = n0 + wave * 16 + r16;
      if (m < nrep && n < ndat) T[(int64_t)m * ndat + n] = acc[t][v];
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

// Rows per member tile: 80 when that pads the member count no more than 64
// does (400 members: 5 tiles of 80 against 7 of 64), else 64.
static int fk_tile_rows(int nrep) {
  const int64_t p64 = (int64_t)(nrep + 63) / 64 * 64, p80 = (int64_t)(nrep + 79) / 80 * 80;
  return p80 <= p64 ? 80 : 64;
}

// K slices for a contraction: the smallest S whose tiles x S workgroups fill
// at least 93 % of the rounds of workgroup slots they occupy (two per compute
// unit), with slices of at least 8 K steps and S <= 64; failing that the S
// with the fullest rounds.  Extra slices cost partial sums written and added.
int fk_slices(int nrep, int ndat, int64_t K, int n_cu) {
  const int bm = fk_tile_rows(nrep);
  const int64_t tiles = (int64_t)((ndat + kFkBN - 1) / kFkBN) * ((nrep + bm - 1) / bm);
  const int64_t slots = (int64_t)kFkSlotsPerCu * std::max(n_cu, 1);
  const int64_t smax = std::max<int64_t>(1, std::min<int64_t>(64, K / (8 * kFkBK)));
  int best = 1;
  double best_fill = -1.0;
  for (int64_t S = 1; S <= smax; ++S) {
    const int64_t wg = tiles * S;
    const double fill = (double)wg / (double)(((wg + slots - 1) / slots) * slots);
    if (fill >= 0.93) return (int)S;
    if (fill > best_fill + 1e-12) {
      best_fill = fill;
      best = (int)S;
    }
  }
  return best;
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
  const int bm = fk_tile_rows(nrep);
  const dim3 grid((unsigned)((ndat + kFkBN - 1) / kFkBN), (unsigned)((nrep + bm - 1) / bm), (unsigned)S);
  double* dst = S > 1 ? ws : T;
  kslice = std::max<int64_t>(kslice, 1);
  if (bm == 80)
    hipLaunchKernelGGL(k_fk_contract<5>, grid, dim3(kFkThreads), 0, s, F, FK, nrep, ndat, K, kslice, dst);
  else
    hipLaunchKernelGGL(k_fk_contract<4>, grid, dim3(kFkThreads), 0, s, F, FK, nrep, ndat, K, kslice, dst);
  if (S > 1) {
    const int64_t mn = (int64_t)nrep * ndat;
    const int64_t nb = std::min<int64_t>((mn + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fk_reduce, dim3((unsigned)nb), dim3(256), 0, s, ws, S, mn, T);
  }
  return hipGetLastError();
}

}  // namespace pdfmi
