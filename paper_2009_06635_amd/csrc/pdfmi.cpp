// Host runtime of libpdfmi.so: argument and grid validation, member registry,
// per-cell Hermite coefficients, device packing/upload, flavour->column tables,
// error state and kernel launches.  Implements include/pdfmi.h.
#include "pdfmi.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cerrno>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "pdfmi_dev.h"

namespace pdfmi {
size_t xfxq2_shared_bytes(const MemberDev& m, bool f32);
size_t alphas_lds_bytes(const AlphasDev* A);
hipError_t launch_xfxq2_f64(const MemberDev&, const ReqCols&, const double*, const double*, int64_t, double*,
                            unsigned long long*, int, double, const LaunchCfg&, const AlphasDev*, double*, hipStream_t);
hipError_t launch_xfxq2_f32(const MemberDev&, const ReqCols&, const double*, const double*, int64_t, float*,
                            unsigned long long*, int, double, const LaunchCfg&, const AlphasDev*, double*, hipStream_t);
hipError_t launch_locate(const MemberDev&, const double*, const double*, int64_t, int32_t*, int32_t*, int32_t*,
                         int8_t*, int, hipStream_t);
hipError_t launch_alphas(const AlphasDev&, const double*, int64_t, double*, unsigned long long*, int, hipStream_t);
int64_t mc_partials(int64_t n);
size_t batch_shared_bytes(int max_tbl, bool f32, bool lds);
BatchLaunch batch_launch_params(bool f32, bool lds, int max_tbl, int64_t max_elems, int n_cu, int blocks_per_cu,
                                int ntiles);
hipError_t batch_prepare(const BatchLaunch& L);
hipError_t batch_launch(const BatchLaunch& L, void** args, unsigned* counter, hipStream_t s);
int sur_nparams();
constexpr int kSurMaxEnvKnots = 512;   // the inference kernel stages the envelope in LDS
constexpr int kAlphasMaxHints = 2048;  // alpha_s search hints staged in LDS
int sur_out_width();
int sur_hidden();
int sur_slices(int B);
size_t sur_workspace_floats(int B);
hipError_t sur_train_prepare();
hipError_t sur_forward_backward(const SurBufs& b, const float* in, const float* T, int B, float* loss_out,
                                hipStream_t s);
hipError_t sur_train_begin(const SurBufs& b, int64_t step, int64_t nbatches, int total, float lr0, float lrf,
                           float* loss_out, hipStream_t s);
hipError_t sur_train_step(const SurBufs& b, const float* in, const float* T, int B, hipStream_t s);
hipError_t sur_adam(const SurBufs& b, float lr, int step, hipStream_t s);
hipError_t sur_refresh_bf16(const SurBufs& b, hipStream_t s);
hipError_t sur_prep(const SurDev& S, const MemberDev& m, const double* x, const double* q2, const double* xf,
                    int64_t n, float* in, float* T, unsigned char* keep, hipStream_t s);
hipError_t sur_gather(const float* in_all, const float* T_all, const int64_t* idx, int64_t n, float* in, float* T,
                      hipStream_t s);
hipError_t sur_infer(const SurDev& S, const MemberDev& m, const ReqCols& rc, const SurBufs& b, const double* x,
                     const double* q2, int64_t n, float* out, double invL01, unsigned long long* nerr, int n_cu,
                     hipStream_t s);
template <typename T>
hipError_t launch_mc_sum(const T*, const T*, int, const double*, int64_t, double*, double*, hipStream_t);
template <typename T>
hipError_t launch_mc_fused(const MemberDev&, const ReqCols&, const AlphasDev&, const double*, const double*,
                           const double*, int64_t, double*, double*, unsigned long long*, double, int, hipStream_t);
size_t mc_fused_shared_bytes(const MemberDev& m, const AlphasDev& A, int64_t grid_elems, bool f32);
hipError_t launch_fk_contract(const double* F, const double* FK, int nrep, int ndat, int64_t K, double* T, int S,
                              double* ws, hipStream_t s);
int fk_slices(int nrep, int ndat, int64_t K, int n_cu);
size_t fk_scratch_bytes();
hipError_t fk_scratch_setup(int device, double** out);
}  // namespace pdfmi

using namespace pdfmi;

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int fail_hip(hipError_t e, const char* what) {
  return fail(e == hipErrorOutOfMemory ? PDF_ERR_NOMEM : PDF_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

}  // namespace

namespace pdfmi {
// Error reporting for the library's other host sources (same thread-local message).
int report_error(int code, const char* msg) { return fail(code, "%s", msg); }
}  // namespace pdfmi

namespace {

struct Member {
  bool used = false;
  MemberDev dev{};
  void* dmem = nullptr;
  std::vector<int> pids;   // stored column -> pid (0 normalised to 21)
  std::vector<int> h_shape;       // host copy of the load arguments (surrogate envelopes)
  std::vector<double> h_knots, h_values;
  double invL01 = 0.0;
  uint64_t gen = 0;        // load generation: a slot reused by a later load gets a new one
};

std::mutex g_mu;
std::vector<Member> g_members;
uint64_t g_load_gen = 0;
bool g_init = false;
int g_ncu = 0;
std::string g_arch;  // device architecture name (autotune cache keys)
unsigned long long* g_nerr = nullptr;
bool g_has_alphas = false;
AlphasDev g_alphas{};
void* g_alphas_mem = nullptr;
int g_lds_policy = 0;  // 0 auto, 1 never stage the grid in LDS, 2 whenever it fits
int g_vector_cols = 1; // serve all-column requests with G-wide vector gathers
int g_blocks_per_cu = 32;
void* g_fk_ws = nullptr;      // partial sums of the K slices of pdf_fk_contract (grow-only)
size_t g_fk_ws_bytes = 0;
double* g_fk_scratch = nullptr;  // device address of the fixed scratch of pdf_fk_contract_noalloc
constexpr size_t kLdsBytes = 160 * 1024;

// The part of the set-up that allocates nothing: the device, its compute
// units and the device address of the fixed FK scratch array.
bool g_dev_ready = false;
int ensure_device() {
  if (g_dev_ready) return PDF_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDevice");
  e = hipDeviceGetAttribute(&g_ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return fail_hip(e, "hipDeviceGetAttribute");
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, dev);
  if (e != hipSuccess) return fail_hip(e, "hipGetDeviceProperties");
  g_arch = prop.gcnArchName;
  for (char& c : g_arch)
    if (c == ' ' || c == '\t') c = '_';
  e = fk_scratch_setup(dev, &g_fk_scratch);
  if (e != hipSuccess) return fail_hip(e, "hipGetSymbolAddress(fk scratch)");
  g_dev_ready = true;
  return PDF_OK;
}

int ensure_init() {
  if (g_init) return PDF_OK;
  int rc = ensure_device();
  if (rc != PDF_OK) return rc;
  hipError_t e = hipMalloc(&g_nerr, sizeof(unsigned long long));
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(error counter)");
  e = hipMemset(g_nerr, 0, sizeof(unsigned long long));
  if (e != hipSuccess) return fail_hip(e, "hipMemset(error counter)");
  g_init = true;
  return PDF_OK;
}

bool valid_pid(int p) { return (p >= -6 && p <= 6) || p == 21; }
int norm_pid(int p) { return p == 0 ? 21 : p; }

// Hermite coefficients of every cell of a strictly increasing 1D table
// (see CellCoef); edge flags within [lo, hi].
void cell_coefs(const double* t, int n, CellCoef* out) {
  std::vector<double> D(n - 1);
  for (int i = 0; i + 1 < n; ++i) D[i] = std::log(t[i + 1] / t[i]);
  for (int i = 0; i + 1 < n; ++i) {
    CellCoef c{};
    c.t0 = t[i];
    c.t1 = t[i + 1];
    c.inv_t0 = 1.0 / t[i];
    c.invD = 1.0 / D[i];
    const bool L = i > 0, R = i + 1 < n - 1;
    c.hl = L ? 0.5 * (D[i] / D[i - 1]) : -1.0;
    c.hr = R ? 0.5 * (D[i] / D[i + 1]) : -1.0;
    out[i] = c;
  }
}

bool strictly_increasing(const double* t, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(t[i])) return false;
  for (int i = 0; i + 1 < n; ++i)
    if (!(t[i] < t[i + 1])) return false;
  return true;
}

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bucket hints of a strictly increasing table of positive knots (HintAxis):
// the coarsest buckets (largest shift) with at most two knots strictly
// inside any of them, provided the list stays within kMaxHintsPerAxis;
// otherwise no list (the kernels binary search that table).
constexpr int kMaxHintsPerAxis = 4096;

uint64_t double_bits(double v) {
  uint64_t u;
  std::memcpy(&u, &v, 8);
  return u;
}

HintAxis build_hints(const double* t, int n, std::vector<short>& hints) {
  HintAxis h{-1, 0, 0, 0u};
  if (n < 4) return h;
  const int last = n - 2;
  for (int shift = 52; shift >= 32; --shift) {
    const uint64_t k0 = double_bits(t[0]) >> shift, k1 = double_bits(t[n - 1]) >> shift;
    const uint64_t nb = k1 - k0 + 1;
    if (nb > (uint64_t)kMaxHintsPerAxis) break;  // finer buckets only make the list longer
    std::vector<int> inside(nb, 0);
    const uint64_t low_mask = (1ull << shift) - 1;
    for (int i = 0; i < n; ++i) {
      const uint64_t u = double_bits(t[i]);
      if (u & low_mask) ++inside[(u >> shift) - k0];  // above the bucket's smallest value
    }
    if (*std::max_element(inside.begin(), inside.end()) > 2) continue;
    h.off = (int)hints.size();
    h.n = (int)nb;
    h.shift = shift;
    h.key0 = (unsigned)k0;
    for (uint64_t b = 0; b < nb; ++b) {
      const uint64_t lo_bits = (k0 + b) << shift;
      double lo;
      std::memcpy(&lo, &lo_bits, 8);
      const int i = (int)(std::upper_bound(t, t + n, lo) - t) - 1;  // largest i with t[i] <= lo
      hints.push_back((short)std::min(std::max(i, 0), last));
    }
    return h;
  }
  return h;
}

int check_stream_args(const void* a, const void* b, int64_t n) {
  if (n < 0) return fail(PDF_ERR_ARG, "n < 0");
  if (n > 0 && (!a || !b)) return fail(PDF_ERR_ARG, "null device pointer");
  return PDF_OK;
}

int build_req(const Member& M, const int32_t* pids, int32_t n_pids, ReqCols& rc) {
  if (!pids) {
    if ((int)M.pids.size() > kMaxReq) return fail(PDF_ERR_ARG, "too many stored flavours for one call");
    rc.n = (int)M.pids.size();
    for (int j = 0; j < rc.n; ++j) rc.col[j] = j;
    return PDF_OK;
  }
  if (n_pids < 1 || n_pids > kMaxReq) return fail(PDF_ERR_ARG, "n_pids must be in [1, %d]", kMaxReq);
  rc.n = n_pids;
  for (int j = 0; j < n_pids; ++j) {
    if (!valid_pid(pids[j])) return fail(PDF_ERR_PID, "invalid flavour id %d", pids[j]);
    const int p = norm_pid(pids[j]);
    rc.col[j] = -1;
    for (size_t c = 0; c < M.pids.size(); ++c)
      if (M.pids[c] == p) rc.col[j] = (int)c;
  }
  return PDF_OK;
}

Member* get_member(int32_t id) {
  if (id < 0 || id >= (int32_t)g_members.size() || !g_members[id].used) return nullptr;
  return &g_members[id];
}

// Stage the whole grid in LDS for this call?
// extra: further LDS bytes the launch needs (the alpha_s table of a fused call).
int lds_grid_elems(const Member& M, bool f32, int64_t n, size_t extra = 0) {
  if (g_lds_policy == 1) return 0;
  const int64_t elems = f32 ? M.dev.elems32 : M.dev.elems64;
  const size_t bytes = (size_t)elems * (f32 ? 4 : 8) + xfxq2_shared_bytes(M.dev, f32) + extra;
  if (bytes > kLdsBytes - 1024) return 0;
  if (g_lds_policy == 0) {
    // each workgroup pays one grid copy; require enough tiles to amortise it
    const int64_t tiles = (n + 255) / 256;
    const int per_cu = (int)(kLdsBytes / bytes);
    if (tiles < (int64_t)4 * g_ncu * (per_cu > 0 ? per_cu : 1)) return 0;
  }
  return (int)elems;
}

}  // namespace

// ---------------------------------------------------------------------------------------

extern "C" int pdf_validate_grid(int32_t K, const int32_t* shape, int32_t P, const int32_t* pids,
                                 const double* knots, const double* values) {
  if (!shape || !pids || !knots || !values) return fail(PDF_ERR_ARG, "null pointer");
  if (K < 1 || K > kMaxSub) return fail(PDF_ERR_GRID, "n_subgrids must be in [1, %d]", kMaxSub);
  if (P < 1 || P > 64) return fail(PDF_ERR_GRID, "n_pids must be in [1, 64]");
  for (int c = 0; c < P; ++c) {
    if (!valid_pid(pids[c])) return fail(PDF_ERR_PID, "invalid stored flavour id %d", pids[c]);
    for (int d = 0; d < c; ++d)
      if (norm_pid(pids[d]) == norm_pid(pids[c])) return fail(PDF_ERR_PID, "duplicated flavour id %d", pids[c]);
  }
  int64_t ko = 0, vo = 0;
  double x0 = 0, x1 = 0, qprev = 0;
  for (int k = 0; k < K; ++k) {
    const int nx = shape[2 * k], nq = shape[2 * k + 1];
    if (nx < 2 || nq < 2 || nx > (1 << 20) || nq > (1 << 20))
      return fail(PDF_ERR_GRID, "sub-grid %d: need nx >= 2 and nq >= 2", k);
    const double* xk = knots + ko;
    const double* qk = knots + ko + nx;
    if (!strictly_increasing(xk, nx) || !(xk[0] > 0.0) || !(xk[nx - 1] <= 1.0))
      return fail(PDF_ERR_GRID, "sub-grid %d: x knots must be strictly increasing in (0, 1]", k);
    if (!strictly_increasing(qk, nq) || !(qk[0] > 0.0))
      return fail(PDF_ERR_GRID, "sub-grid %d: Q^2 knots must be strictly increasing and > 0", k);
    if (k == 0) {
      x0 = xk[0];
      x1 = xk[nx - 1];
    } else {
      if (xk[0] != x0 || xk[nx - 1] != x1) return fail(PDF_ERR_GRID, "sub-grid %d: x range differs from sub-grid 0", k);
      if (qk[0] != qprev) return fail(PDF_ERR_GRID, "sub-grid %d: first Q^2 knot must repeat the previous last knot", k);
    }
    qprev = qk[nq - 1];
    const int64_t nv = (int64_t)nx * nq * P;
    for (int64_t i = 0; i < nv; ++i)
      if (!std::isfinite(values[vo + i])) return fail(PDF_ERR_GRID, "sub-grid %d: non-finite value", k);
    ko += nx + nq;
    vo += nv;
  }
  // the kernels address a member's padded FP64 values with 32-bit byte offsets
  int64_t padded_bytes = 0;
  for (int k = 0; k < K; ++k)
    padded_bytes += (int64_t)std::max(shape[2 * k], 4) * std::max(shape[2 * k + 1], 4) * ((P + 15) & ~15) * 8;
  if (padded_bytes > INT32_MAX) return fail(PDF_ERR_GRID, "grid values exceed 2 GiB");
  if (ko > 8192) return fail(PDF_ERR_GRID, "more than 8192 knots in total (they are staged in LDS)");
  return PDF_OK;
}

extern "C" int pdf_load_grid(int32_t K, const int32_t* shape, int32_t P, const int32_t* pids, const double* knots,
                             const double* values, int32_t* member_out) {
  if (!member_out) return fail(PDF_ERR_ARG, "null member_out");
  int rc = pdf_validate_grid(K, shape, P, pids, knots, values);
  if (rc != PDF_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  if ((rc = ensure_init()) != PDF_OK) return rc;

  Member M;
  M.used = true;
  for (int c = 0; c < P; ++c) M.pids.push_back(norm_pid(pids[c]));
  {
    int64_t nk = 0, nv = 0;
    for (int k = 0; k < K; ++k) {
      nk += shape[2 * k] + shape[2 * k + 1];
      nv += (int64_t)shape[2 * k] * shape[2 * k + 1] * P;
    }
    M.h_shape.assign(shape, shape + 2 * K);
    M.h_knots.assign(knots, knots + nk);
    M.h_values.assign(values, values + nv);
  }
  MemberDev& d = M.dev;
  d.K = K;
  d.P = P;
  // FP64 rows are whole 64- or 128-byte lines (fewer cache lines per
  // stencil), FP32 rows a multiple of 16 bytes
  const int P64 = P <= 4 ? 4 : (P <= 8 ? 8 : (P + 15) & ~15), P32 = (P + 3) & ~3;
  d.P64 = P64;
  d.P32 = P32;
  int64_t n64 = 0, n32 = 0;
  for (int k = 0; k < K; ++k) {
    const int nx = shape[2 * k], nq = shape[2 * k + 1];
    SubDesc& S = d.sub[k];
    S.nx = nx;
    S.nq = nq;
    S.nxp = nx < 4 ? 4 : nx;
    S.nqp = nq < 4 ? 4 : nq;
    S.val_off64 = n64;
    S.val_off32 = n32;
    n64 += (int64_t)S.nxp * S.nqp * P64;
    n32 += (int64_t)S.nxp * S.nqp * P32;
  }
  d.elems64 = n64;
  d.elems32 = n32;
  // location tables: knots, cells and hints per axis; sub-grids whose x knots
  // equal sub-grid 0's share its x tables
  std::vector<double> hk;
  std::vector<CellCoef> hc;
  std::vector<short> hh;
  std::vector<double> hv((size_t)n64, 0.0);
  std::vector<float> hf((size_t)n32, 0.0f);
  int64_t ko = 0, vo = 0;
  for (int k = 0; k < K; ++k) {
    SubDesc& S = d.sub[k];
    const double* xk = knots + ko;
    const double* qk = knots + ko + S.nx;
    const SubDesc& S0 = d.sub[0];
    if (k > 0 && S.nx == S0.nx && std::memcmp(xk, knots, sizeof(double) * S.nx) == 0) {
      S.xk_off = S0.xk_off;
      S.xc_off = S0.xc_off;
      S.xh = S0.xh;
    } else {
      S.xk_off = (int)hk.size();
      hk.insert(hk.end(), xk, xk + S.nx);
      S.xc_off = (int)hc.size();
      hc.resize(hc.size() + S.nx - 1);
      cell_coefs(xk, S.nx, &hc[S.xc_off]);
      S.xh = build_hints(xk, S.nx, hh);
    }
    S.qk_off = (int)hk.size();
    hk.insert(hk.end(), qk, qk + S.nq);
    S.qc_off = (int)hc.size();
    hc.resize(hc.size() + S.nq - 1);
    cell_coefs(qk, S.nq, &hc[S.qc_off]);
    S.qh = build_hints(qk, S.nq, hh);
    S.qfirst = qk[0];
    for (int ix = 0; ix < S.nx; ++ix)
      for (int iq = 0; iq < S.nq; ++iq)
        for (int c = 0; c < P; ++c) {
          const double v = values[vo + ((int64_t)ix * S.nq + iq) * P + c];
          hv[S.val_off64 + ((int64_t)ix * S.nqp + iq) * P64 + c] = v;
          hf[S.val_off32 + ((int64_t)ix * S.nqp + iq) * P32 + c] = (float)v;
        }
    ko += S.nx + S.nq;
    vo += (int64_t)S.nx * S.nq * P;
  }
  d.nknots = (int)hk.size();
  d.nknots_pad = (d.nknots + 1) & ~1;
  d.xmin = knots[0];
  d.xmax = knots[shape[0] - 1];
  d.qmin = d.sub[0].qfirst;
  d.qmax = hk[d.sub[K - 1].qk_off + d.sub[K - 1].nq - 1];
  M.invL01 = hc[d.sub[0].qc_off].invD;

  // table block: [knots][cells][hints][sub-grid descriptors], 16-byte aligned parts
  d.cells_off = d.nknots_pad * 8;
  d.hints_off = d.cells_off + (int)(hc.size() * sizeof(CellCoef));
  d.subs_off = d.hints_off + (int)align_up(hh.size() * sizeof(short), 16);
  d.tbl_bytes = d.subs_off + (int)align_up((size_t)K * sizeof(SubDesc), 16);
  const size_t bt = align_up((size_t)d.tbl_bytes, 256);
  const size_t b64 = align_up((size_t)n64 * sizeof(double), 256);
  const size_t b32 = align_up((size_t)n32 * sizeof(float), 256);
  std::vector<unsigned char> blob(bt + b64 + b32, 0);
  std::memcpy(blob.data(), hk.data(), hk.size() * sizeof(double));
  std::memcpy(blob.data() + d.cells_off, hc.data(), hc.size() * sizeof(CellCoef));
  if (!hh.empty()) std::memcpy(blob.data() + d.hints_off, hh.data(), hh.size() * sizeof(short));
  std::memcpy(blob.data() + d.subs_off, d.sub, (size_t)K * sizeof(SubDesc));
  std::memcpy(blob.data() + bt, hv.data(), (size_t)n64 * sizeof(double));
  std::memcpy(blob.data() + bt + b64, hf.data(), (size_t)n32 * sizeof(float));

  hipError_t e = hipMalloc(&M.dmem, blob.size());
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(grid)");
  e = hipMemcpy(M.dmem, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(M.dmem);
    return fail_hip(e, "hipMemcpy(grid)");
  }
  unsigned char* base = static_cast<unsigned char*>(M.dmem);
  d.tables = base;
  d.knots = reinterpret_cast<const double*>(base);
  d.cells = reinterpret_cast<const CellCoef*>(base + d.cells_off);
  d.hints = reinterpret_cast<const short*>(base + d.hints_off);
  d.subs = reinterpret_cast<const SubDesc*>(base + d.subs_off);
  d.v64 = reinterpret_cast<const double*>(base + bt);
  d.v32 = reinterpret_cast<const float*>(base + bt + b64);

  M.gen = ++g_load_gen;
  for (size_t i = 0; i < g_members.size(); ++i) {
    if (!g_members[i].used) {
      g_members[i] = M;
      *member_out = (int32_t)i;
      return PDF_OK;
    }
  }
  g_members.push_back(M);
  *member_out = (int32_t)(g_members.size() - 1);
  return PDF_OK;
}

extern "C" int pdf_unload(int32_t member) {
  std::lock_guard<std::mutex> lock(g_mu);
  Member* M = get_member(member);
  if (!M) return fail(PDF_ERR_MEMBER, "unknown member %d", member);
  hipError_t e = hipFree(M->dmem);
  *M = Member();
  if (e != hipSuccess) return fail_hip(e, "hipFree(grid)");
  return PDF_OK;
}

extern "C" int pdf_validate_alphas(int32_t n, const double* q2k, const double* a) {
  if (!q2k || !a) return fail(PDF_ERR_ARG, "null pointer");
  if (n < 2 || n > 256) return fail(PDF_ERR_GRID, "alpha_s table needs 2..256 knots");
  int seg_len = 1, nseg = 1;
  for (int i = 0; i < n; ++i) {
    if (!std::isfinite(q2k[i]) || !(q2k[i] > 0.0) || !std::isfinite(a[i]))
      return fail(PDF_ERR_GRID, "alpha_s knot %d: need finite Q^2 > 0 and finite value", i);
    if (i == 0) continue;
    if (q2k[i] == q2k[i - 1]) {
      if (seg_len < 2) return fail(PDF_ERR_GRID, "alpha_s segment ending at knot %d has < 2 knots", i);
      if (++nseg > kMaxSeg) return fail(PDF_ERR_GRID, "more than %d alpha_s segments", kMaxSeg);
      seg_len = 1;
    } else if (q2k[i] > q2k[i - 1]) {
      ++seg_len;
    } else {
      return fail(PDF_ERR_GRID, "alpha_s Q^2 knots must be non-decreasing");
    }
  }
  if (seg_len < 2) return fail(PDF_ERR_GRID, "last alpha_s segment has < 2 knots");
  return PDF_OK;
}

extern "C" int pdf_load_alphas(int32_t n, const double* q2k, const double* a) {
  int rc = pdf_validate_alphas(n, q2k, a);
  if (rc != PDF_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  if ((rc = ensure_init()) != PDF_OK) return rc;
  AlphasDev A{};
  A.n = n;
  A.nseg = 0;
  int lo = 0;
  for (int i = 1; i <= n; ++i) {
    if (i == n || q2k[i] == q2k[i - 1]) {
      A.seg_lo[A.nseg] = lo;
      A.seg_hi[A.nseg] = i - 1;
      A.seg_first[A.nseg] = q2k[lo];
      ++A.nseg;
      lo = i;
    }
  }
  std::vector<CellCoef> hc((size_t)n);  // cell j valid when j, j+1 share a segment
  for (int s = 0; s < A.nseg; ++s) cell_coefs(q2k + A.seg_lo[s], A.seg_hi[s] - A.seg_lo[s] + 1, &hc[A.seg_lo[s]]);
  std::vector<short> hh;
  for (int s = 0; s < A.nseg; ++s) {
    A.seg_hint[s] = build_hints(q2k + A.seg_lo[s], A.seg_hi[s] - A.seg_lo[s] + 1, hh);
    if ((int)hh.size() > kAlphasMaxHints) {  // keep the staged list small: binary search this segment
      hh.resize(A.seg_hint[s].off);
      A.seg_hint[s].off = -1;
    }
  }
  A.nhints = (int)hh.size();
  const size_t bk = align_up((size_t)n * 8, 256), bv = align_up((size_t)n * 8, 256);
  const size_t bc = align_up(hc.size() * sizeof(CellCoef), 256);
  std::vector<unsigned char> blob(bk + bv + bc + hh.size() * sizeof(short) + 16, 0);
  std::memcpy(blob.data(), q2k, (size_t)n * 8);
  std::memcpy(blob.data() + bk, a, (size_t)n * 8);
  std::memcpy(blob.data() + bk + bv, hc.data(), hc.size() * sizeof(CellCoef));
  if (!hh.empty()) std::memcpy(blob.data() + bk + bv + bc, hh.data(), hh.size() * sizeof(short));
  void* mem = nullptr;
  hipError_t e = hipMalloc(&mem, blob.size());
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(alpha_s)");
  e = hipMemcpy(mem, blob.data(), blob.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(mem);
    return fail_hip(e, "hipMemcpy(alpha_s)");
  }
  unsigned char* b = static_cast<unsigned char*>(mem);
  A.knots = reinterpret_cast<const double*>(b);
  A.vals = reinterpret_cast<const double*>(b + bk);
  A.cells = reinterpret_cast<const CellCoef*>(b + bk + bv);
  A.hints = reinterpret_cast<const short*>(b + bk + bv + bc);
  if (g_alphas_mem) (void)hipFree(g_alphas_mem);
  g_alphas_mem = mem;
  g_alphas = A;
  g_has_alphas = true;
  return PDF_OK;
}

// aout: alpha_s output of a fused call (nullptr: PDFs only).
template <typename T>
static int xfxq2_impl(int32_t member, const int32_t* pids, int32_t n_pids, const double* x, const double* q2,
                      int64_t n, T* out, double* aout, bool fused, pdf_stream_t stream) {
  int rc = check_stream_args(x, q2, n);
  if (rc != PDF_OK) return rc;
  if (n > 0 && !out) return fail(PDF_ERR_ARG, "null out");
  if (fused && n > 0 && !aout) return fail(PDF_ERR_ARG, "null alphas_out");
  std::lock_guard<std::mutex> lock(g_mu);
  Member* M = get_member(member);
  if (!M) return fail(PDF_ERR_MEMBER, "unknown member %d", member);
  if (fused && !g_has_alphas) return fail(PDF_ERR_STATE, "no alpha_s table loaded");
  ReqCols req{};
  if ((rc = build_req(*M, pids, n_pids, req)) != PDF_OK) return rc;
  if (n == 0) return PDF_OK;
  if (n * (int64_t)req.n > ((int64_t)1 << 40)) return fail(PDF_ERR_ARG, "n too large");
  const bool f32 = sizeof(T) == 4;
  const int lds = lds_grid_elems(*M, f32, n, alphas_lds_bytes(fused ? &g_alphas : nullptr));
  hipError_t e;
  const LaunchCfg cfg{g_ncu, g_blocks_per_cu, g_vector_cols};
  const AlphasDev* A = fused ? &g_alphas : nullptr;
  if constexpr (sizeof(T) == 8)
    e = launch_xfxq2_f64(M->dev, req, x, q2, n, out, g_nerr, lds, M->invL01, cfg, A, aout, (hipStream_t)stream);
  else
    e = launch_xfxq2_f32(M->dev, req, x, q2, n, out, g_nerr, lds, M->invL01, cfg, A, aout, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch xfxq2");
  return PDF_OK;
}

extern "C" int pdf_xfxq2(int32_t member, const int32_t* pids, int32_t n_pids, const double* x, const double* q2,
                         int64_t n, double* out, pdf_stream_t stream) {
  return xfxq2_impl<double>(member, pids, n_pids, x, q2, n, out, nullptr, false, stream);
}

extern "C" int pdf_xfxq2_f32(int32_t member, const int32_t* pids, int32_t n_pids, const double* x,
                             const double* q2, int64_t n, float* out, pdf_stream_t stream) {
  return xfxq2_impl<float>(member, pids, n_pids, x, q2, n, out, nullptr, false, stream);
}

extern "C" int pdf_xfxq2_alphas(int32_t member, const int32_t* pids, int32_t n_pids, const double* x,
                                const double* q2, int64_t n, double* out, double* alphas_out, pdf_stream_t stream) {
  return xfxq2_impl<double>(member, pids, n_pids, x, q2, n, out, alphas_out, true, stream);
}

extern "C" int pdf_xfxq2_alphas_f32(int32_t member, const int32_t* pids, int32_t n_pids, const double* x,
                                    const double* q2, int64_t n, float* out, double* alphas_out,
                                    pdf_stream_t stream) {
  return xfxq2_impl<float>(member, pids, n_pids, x, q2, n, out, alphas_out, true, stream);
}

extern "C" int pdf_alphas_q2(const double* q2, int64_t n, double* out, pdf_stream_t stream) {
  int rc = check_stream_args(q2, out, n);
  if (rc != PDF_OK) return rc;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_has_alphas) return fail(PDF_ERR_STATE, "no alpha_s table loaded");
  if (n == 0) return PDF_OK;
  hipError_t e = launch_alphas(g_alphas, q2, n, out, g_nerr, g_ncu, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch alphas");
  return PDF_OK;
}

extern "C" int pdf_locate(int32_t member, const double* x, const double* q2, int64_t n, int32_t* k, int32_t* ix,
                          int32_t* iq, int8_t* region, pdf_stream_t stream) {
  int rc = check_stream_args(x, q2, n);
  if (rc != PDF_OK) return rc;
  if (n > 0 && (!k || !ix || !iq || !region)) return fail(PDF_ERR_ARG, "null output pointer");
  std::lock_guard<std::mutex> lock(g_mu);
  Member* M = get_member(member);
  if (!M) return fail(PDF_ERR_MEMBER, "unknown member %d", member);
  if (n == 0) return PDF_OK;
  hipError_t e = launch_locate(M->dev, x, q2, n, k, ix, iq, region, g_ncu, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch locate");
  return PDF_OK;
}

extern "C" int pdf_error_count(int64_t* count_out, int32_t reset, pdf_stream_t stream) {
  if (!count_out) return fail(PDF_ERR_ARG, "null count_out");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_init();
  if (rc != PDF_OK) return rc;
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  unsigned long long v = 0;
  e = hipMemcpy(&v, g_nerr, sizeof v, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "hipMemcpy(error counter)");
  *count_out = (int64_t)v;
  if (reset) {
    e = hipMemset(g_nerr, 0, sizeof v);
    if (e != hipSuccess) return fail_hip(e, "hipMemset(error counter)");
  }
  return PDF_OK;
}

extern "C" int pdf_set_tuning(int32_t knob, int32_t value) {
  std::lock_guard<std::mutex> lock(g_mu);
  switch (knob) {
    case PDF_TUNE_LDS_POLICY:
      if (value < 0 || value > 2) return fail(PDF_ERR_ARG, "LDS policy must be 0, 1 or 2");
      g_lds_policy = value;
      return PDF_OK;
    case PDF_TUNE_VECTOR_COLUMNS:
      if (value < 0 || value > 1) return fail(PDF_ERR_ARG, "vector-columns knob must be 0 or 1");
      g_vector_cols = value;
      return PDF_OK;
    case PDF_TUNE_BLOCKS_PER_CU:
      if (value < 1 || value > 4096) return fail(PDF_ERR_ARG, "blocks per CU must be in [1, 4096]");
      g_blocks_per_cu = value;
      return PDF_OK;
    default:
      return fail(PDF_ERR_ARG, "unknown tuning knob %d", knob);
  }
}

extern "C" int pdf_get_tuning(int32_t knob, int32_t* value) {
  if (!value) return fail(PDF_ERR_ARG, "null value");
  std::lock_guard<std::mutex> lock(g_mu);
  switch (knob) {
    case PDF_TUNE_LDS_POLICY: *value = g_lds_policy; return PDF_OK;
    case PDF_TUNE_VECTOR_COLUMNS: *value = g_vector_cols; return PDF_OK;
    case PDF_TUNE_BLOCKS_PER_CU: *value = g_blocks_per_cu; return PDF_OK;
    default: return fail(PDF_ERR_ARG, "unknown tuning knob %d", knob);
  }
}

// ---------------------------------------------------------------------------------------
// Batched plans

namespace {

struct Plan {
  bool used = false;
  int out_f64 = 0;
  int tile_points = 4096;
  int blocks_per_cu = 1;
  int vector_cols = 1;
  int use_graph = 0;
  bool lds = false;
  int max_tbl = 0;   // bytes of the largest member's location tables
  int64_t max_elems = 0;
  std::vector<BatchReq> reqs;
  std::vector<int> cols;
  std::vector<MemberDev> members;
  std::vector<std::pair<int32_t, uint64_t>> member_ids;  // (member id, load generation) behind members
  std::vector<double> invL01;
  int ntiles = 0;
  void* dmem = nullptr;        // reqs, cols, members, invL01, counter
  BatchTile* d_tiles = nullptr;
  int tiles_cap = 0;
  BatchReq* d_reqs = nullptr;
  int* d_cols = nullptr;
  MemberDev* d_members = nullptr;
  double* d_invL01 = nullptr;
  unsigned* d_counter = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // kernel argument storage (addresses handed to hipLaunchKernel / graph nodes)
  int a_ntiles = 0, a_max_tbl = 0, a_vec = 0;
  void* args[10];
};

std::vector<Plan> g_plans;

void plan_free_graph(Plan& P) {
  if (P.exec) (void)hipGraphExecDestroy(P.exec);
  if (P.graph) (void)hipGraphDestroy(P.graph);
  P.exec = nullptr;
  P.graph = nullptr;
}

void plan_release(Plan& P) {
  plan_free_graph(P);
  if (P.dmem) (void)hipFree(P.dmem);
  if (P.d_tiles) (void)hipFree(P.d_tiles);
  P = Plan();
}

// (Re)build the tile list for the plan's tile size and upload it.  The device
// is drained first: a run of this plan still in flight on some stream reads
// the tile list being replaced.
int plan_tiles(Plan& P) {
  if (P.d_tiles) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return fail_hip(e, "hipDeviceSynchronize");
  }
  std::vector<BatchTile> t;
  // tiles grouped by member so that consecutive tiles tend to share a staged grid
  std::vector<int> order(P.reqs.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = (int)i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.reqs[a].member < P.reqs[b].member; });
  for (int r : order)
    for (int64_t s0 = 0; s0 < P.reqs[r].n; s0 += P.tile_points)
      t.push_back(BatchTile{r, (int)std::min<int64_t>(P.tile_points, P.reqs[r].n - s0), s0});
  if ((int64_t)t.size() > (1LL << 30)) return fail(PDF_ERR_ARG, "too many tiles");
  P.ntiles = (int)t.size();
  if (P.ntiles > P.tiles_cap) {
    if (P.d_tiles) (void)hipFree(P.d_tiles);
    P.d_tiles = nullptr;
    hipError_t e = hipMalloc(&P.d_tiles, sizeof(BatchTile) * std::max(1, P.ntiles));
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(tiles)");
    P.tiles_cap = P.ntiles;
  }
  if (P.ntiles) {
    hipError_t e = hipMemcpy(P.d_tiles, t.data(), sizeof(BatchTile) * t.size(), hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail_hip(e, "hipMemcpy(tiles)");
  }
  return PDF_OK;
}

BatchLaunch plan_params(const Plan& P) {
  return batch_launch_params(!P.out_f64, P.lds, P.max_tbl, P.max_elems, g_ncu, P.blocks_per_cu, P.ntiles);
}

void plan_args(Plan& P) {
  P.a_ntiles = P.ntiles;
  P.a_max_tbl = P.max_tbl;
  P.a_vec = P.vector_cols;
  P.args[0] = &P.d_reqs;
  P.args[1] = &P.d_cols;
  P.args[2] = &P.d_tiles;
  P.args[3] = &P.a_ntiles;
  P.args[4] = &P.d_members;
  P.args[5] = &P.d_invL01;
  P.args[6] = &P.d_counter;
  P.args[7] = &g_nerr;
  P.args[8] = &P.a_max_tbl;
  P.args[9] = &P.a_vec;
}

int plan_build_graph(Plan& P) {
  plan_free_graph(P);
  const BatchLaunch L = plan_params(P);
  hipError_t e = batch_prepare(L);
  if (e != hipSuccess) return fail_hip(e, "hipFuncSetAttribute(batched)");
  if ((e = hipGraphCreate(&P.graph, 0)) != hipSuccess) return fail_hip(e, "hipGraphCreate");
  hipKernelNodeParams r{};
  void* rargs[] = {&P.d_counter};
  r.func = const_cast<void*>(L.reset_fn);
  r.gridDim = dim3(1);
  r.blockDim = dim3(64);
  r.sharedMemBytes = 0;
  r.kernelParams = rargs;
  hipGraphNode_t n1, n2;
  if ((e = hipGraphAddKernelNode(&n1, P.graph, nullptr, 0, &r)) != hipSuccess) return fail_hip(e, "graph node");
  hipKernelNodeParams k{};
  k.func = const_cast<void*>(L.main_fn);
  k.gridDim = dim3(L.grid);
  k.blockDim = dim3(1024);
  k.sharedMemBytes = (unsigned)L.shm;
  k.kernelParams = P.args;
  if ((e = hipGraphAddKernelNode(&n2, P.graph, &n1, 1, &k)) != hipSuccess) return fail_hip(e, "graph node");
  if ((e = hipGraphInstantiate(&P.exec, P.graph, nullptr, nullptr, 0)) != hipSuccess)
    return fail_hip(e, "hipGraphInstantiate");
  return PDF_OK;
}

int plan_run(Plan& P, hipStream_t s) {
  if (P.ntiles == 0) return PDF_OK;
  plan_args(P);
  if (P.use_graph) {
    if (!P.exec) {
      int rc = plan_build_graph(P);
      if (rc != PDF_OK) return rc;
    }
    hipError_t e = hipGraphLaunch(P.exec, s);
    if (e != hipSuccess) return fail_hip(e, "hipGraphLaunch");
    return PDF_OK;
  }
  const BatchLaunch L = plan_params(P);
  hipError_t e = batch_prepare(L);
  if (e != hipSuccess) return fail_hip(e, "hipFuncSetAttribute(batched)");
  e = batch_launch(L, P.args, P.d_counter, s);
  if (e != hipSuccess) return fail_hip(e, "launch batched");
  return PDF_OK;
}

Plan* get_plan(int32_t id) {
  if (id < 0 || id >= (int32_t)g_plans.size() || !g_plans[id].used) return nullptr;
  return &g_plans[id];
}

// A plan holds copies of its members' device pointers: every member must still
// be the one loaded when the plan was built (not unloaded, slot not reused).
int plan_members_live(const Plan& P) {
  for (const auto& mg : P.member_ids) {
    const Member* M = get_member(mg.first);
    if (!M || M->gen != mg.second)
      return fail(PDF_ERR_MEMBER, "member %d was unloaded after the plan was built", mg.first);
  }
  return PDF_OK;
}

// Autotune choices (tile points, vector columns) by request signature and
// device, and the file they are also kept in ("" = none).
std::map<std::string, std::pair<int, int>> g_tune_cache;
std::string g_tune_path;

bool valid_tile(int tile) { return tile >= 64 && tile <= (1 << 22) && (tile & 63) == 0; }

// Reads the "key tile vector" lines of a cache file into g_tune_cache; lines
// that do not parse or hold an invalid choice are skipped.  A missing file
// holds no entries.
int tune_cache_load(const char* path) {
  FILE* f = std::fopen(path, "r");
  if (!f) return errno == ENOENT ? PDF_OK : fail(PDF_ERR_ARG, "cannot read autotune cache %s", path);
  char line[512], key[400];
  while (std::fgets(line, sizeof line, f)) {
    int tile = 0, vec = -1;
    if (std::sscanf(line, "%399s %d %d", key, &tile, &vec) == 3 && valid_tile(tile) && (vec == 0 || vec == 1))
      g_tune_cache[key] = {tile, vec};
  }
  std::fclose(f);
  return PDF_OK;
}

}  // namespace

extern "C" int pdf_batch_tune_cache(const char* path) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (!path || !*path) {
    g_tune_path.clear();
    return PDF_OK;
  }
  const int rc = tune_cache_load(path);
  if (rc != PDF_OK) return rc;
  g_tune_path = path;
  return PDF_OK;
}

extern "C" int pdf_batch_create(const pdf_request* reqs, int32_t n_req, int32_t out_f64, int32_t* plan_out) {
  if (!plan_out || (n_req > 0 && !reqs) || n_req < 0) return fail(PDF_ERR_ARG, "bad argument");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_init();
  if (rc != PDF_OK) return rc;
  Plan P;
  P.used = true;
  P.out_f64 = out_f64 ? 1 : 0;
  std::map<int, int> slot;  // member id -> plan member index
  for (int i = 0; i < n_req; ++i) {
    const pdf_request& q = reqs[i];
    if (q.n < 0) return fail(PDF_ERR_ARG, "request %d: n < 0", i);
    if (q.n > 0 && (!q.x || !q.q2 || !q.out)) return fail(PDF_ERR_ARG, "request %d: null device pointer", i);
    Member* M = get_member(q.member);
    if (!M) return fail(PDF_ERR_MEMBER, "request %d: unknown member %d", i, q.member);
    ReqCols rcols{};
    if ((rc = build_req(*M, q.pids, q.n_pids, rcols)) != PDF_OK) return rc;
    if (!slot.count(q.member)) {
      slot[q.member] = (int)P.members.size();
      P.members.push_back(M->dev);
      P.member_ids.push_back({q.member, M->gen});
      P.invL01.push_back(M->invL01);
      P.max_tbl = std::max(P.max_tbl, M->dev.tbl_bytes);
      P.max_elems = std::max(P.max_elems, P.out_f64 ? M->dev.elems64 : M->dev.elems32);
    }
    BatchReq b{};
    b.member = slot[q.member];
    b.R = rcols.n;
    b.col_off = (int)P.cols.size();
    b.all_cols = rcols.n == M->dev.P;
    for (int j = 0; j < rcols.n; ++j) {
      P.cols.push_back(rcols.col[j]);
      if (rcols.col[j] != j) b.all_cols = 0;
    }
    b.x = q.x;
    b.q2 = q.q2;
    b.out = q.out;
    b.n = q.n;
    P.reqs.push_back(b);
  }
  P.lds = g_lds_policy != 1 &&
          batch_shared_bytes(P.max_tbl, !P.out_f64, true) + (size_t)P.max_elems * (P.out_f64 ? 8 : 4) <=
              kLdsBytes - 1024;
  P.blocks_per_cu = 1;
  const size_t br = align_up(sizeof(BatchReq) * std::max<size_t>(1, P.reqs.size()), 256);
  const size_t bc = align_up(sizeof(int) * std::max<size_t>(1, P.cols.size()), 256);
  const size_t bm = align_up(sizeof(MemberDev) * std::max<size_t>(1, P.members.size()), 256);
  const size_t bi = align_up(sizeof(double) * std::max<size_t>(1, P.invL01.size()), 256);
  hipError_t e = hipMalloc(&P.dmem, br + bc + bm + bi + 256);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(plan)");
  unsigned char* b = static_cast<unsigned char*>(P.dmem);
  P.d_reqs = reinterpret_cast<BatchReq*>(b);
  P.d_cols = reinterpret_cast<int*>(b + br);
  P.d_members = reinterpret_cast<MemberDev*>(b + br + bc);
  P.d_invL01 = reinterpret_cast<double*>(b + br + bc + bm);
  P.d_counter = reinterpret_cast<unsigned*>(b + br + bc + bm + bi);
  if (!P.reqs.empty() && (e = hipMemcpy(P.d_reqs, P.reqs.data(), sizeof(BatchReq) * P.reqs.size(),
                                        hipMemcpyHostToDevice)) != hipSuccess) {
    plan_release(P);
    return fail_hip(e, "hipMemcpy(plan)");
  }
  if (!P.cols.empty() &&
      (e = hipMemcpy(P.d_cols, P.cols.data(), sizeof(int) * P.cols.size(), hipMemcpyHostToDevice)) != hipSuccess) {
    plan_release(P);
    return fail_hip(e, "hipMemcpy(plan)");
  }
  if (!P.members.empty() && ((e = hipMemcpy(P.d_members, P.members.data(), sizeof(MemberDev) * P.members.size(),
                                            hipMemcpyHostToDevice)) != hipSuccess ||
                             (e = hipMemcpy(P.d_invL01, P.invL01.data(), sizeof(double) * P.invL01.size(),
                                            hipMemcpyHostToDevice)) != hipSuccess)) {
    plan_release(P);
    return fail_hip(e, "hipMemcpy(plan)");
  }
  if ((rc = plan_tiles(P)) != PDF_OK) {
    plan_release(P);
    return rc;
  }
  for (size_t i = 0; i < g_plans.size(); ++i)
    if (!g_plans[i].used) {
      g_plans[i] = P;
      *plan_out = (int32_t)i;
      return PDF_OK;
    }
  g_plans.push_back(P);
  *plan_out = (int32_t)(g_plans.size() - 1);
  return PDF_OK;
}

extern "C" int pdf_batch_configure(int32_t plan, int32_t tile_points, int32_t vector_cols, int32_t use_graph) {
  std::lock_guard<std::mutex> lock(g_mu);
  Plan* P = get_plan(plan);
  if (!P) return fail(PDF_ERR_ARG, "unknown plan %d", plan);
  if (tile_points < 64 || tile_points > (1 << 22) || (tile_points & 63))
    return fail(PDF_ERR_ARG, "tile_points must be a multiple of 64 in [64, 4194304]");
  if (vector_cols < 0 || vector_cols > 1 || use_graph < 0 || use_graph > 1)
    return fail(PDF_ERR_ARG, "flags must be 0 or 1");
  plan_free_graph(*P);
  P->vector_cols = vector_cols;
  P->use_graph = use_graph;
  if (tile_points != P->tile_points) {
    P->tile_points = tile_points;
    return plan_tiles(*P);
  }
  return PDF_OK;
}

extern "C" int pdf_batch_run(int32_t plan, pdf_stream_t stream) {
  std::lock_guard<std::mutex> lock(g_mu);
  Plan* P = get_plan(plan);
  if (!P) return fail(PDF_ERR_ARG, "unknown plan %d", plan);
  const int rc = plan_members_live(*P);
  if (rc != PDF_OK) return rc;
  return plan_run(*P, (hipStream_t)stream);
}

extern "C" int pdf_batch_autotune(int32_t plan, int32_t reps, pdf_stream_t stream, int32_t* tile_out,
                                  int32_t* vector_out) {
  if (reps < 1) return fail(PDF_ERR_ARG, "reps must be >= 1");
  std::lock_guard<std::mutex> lock(g_mu);
  Plan* P = get_plan(plan);
  if (!P) return fail(PDF_ERR_ARG, "unknown plan %d", plan);
  if (plan_members_live(*P) != PDF_OK) return PDF_ERR_MEMBER;
  hipStream_t s = (hipStream_t)stream;
  // signature of the work: request count, point total, flavour total, precision
  int64_t pts = 0, evals = 0;
  for (auto& r : P->reqs) {
    pts += r.n;
    evals += r.n * r.R;
  }
  char key[400];
  snprintf(key, sizeof key, "%s/%d/%zu/%lld/%lld/%d/%d", g_arch.c_str(), g_ncu, P->reqs.size(), (long long)pts,
           (long long)evals, P->out_f64, (int)P->lds);
  auto it = g_tune_cache.find(key);
  int best_tile = P->tile_points, best_vec = P->vector_cols;
  if (it != g_tune_cache.end()) {
    best_tile = it->second.first;
    best_vec = it->second.second;
  } else {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int saved_graph = P->use_graph;
    // the sweep; every exit path below restores the plan's graph flag and frees the events
    auto sweep = [&]() -> int {
      if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(PDF_ERR_DEVICE, "hipEventCreate");
      float best = 1e30f;
      P->use_graph = 0;
      for (int tp : {1024, 2048, 4096, 8192, 16384}) {
        for (int vec : {0, 1}) {
          P->tile_points = tp;
          P->vector_cols = vec;
          int rc = plan_tiles(*P);
          if (rc != PDF_OK) return rc;
          if ((rc = plan_run(*P, s)) != PDF_OK) return rc;  // warm-up
          float tot = 0.0f;
          for (int r = 0; r < reps; ++r) {
            (void)hipEventRecord(e0, s);
            if ((rc = plan_run(*P, s)) != PDF_OK) return rc;
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) return fail(PDF_ERR_DEVICE, "hipEventSynchronize");
            float ms = 0.0f;
            (void)hipEventElapsedTime(&ms, e0, e1);
            tot += ms;
          }
          if (tot < best) {
            best = tot;
            best_tile = tp;
            best_vec = vec;
          }
        }
      }
      return PDF_OK;
    };
    const int rc = sweep();
    P->use_graph = saved_graph;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (rc != PDF_OK) return rc;
    g_tune_cache[key] = {best_tile, best_vec};
    if (!g_tune_path.empty()) {  // best effort: a cache that cannot be written only costs a later sweep
      if (FILE* f = std::fopen(g_tune_path.c_str(), "a")) {
        std::fprintf(f, "%s %d %d\n", key, best_tile, best_vec);
        std::fclose(f);
      }
    }
  }
  plan_free_graph(*P);
  P->tile_points = best_tile;
  P->vector_cols = best_vec;
  int rc = plan_tiles(*P);
  if (rc != PDF_OK) return rc;
  if (tile_out) *tile_out = best_tile;
  if (vector_out) *vector_out = best_vec;
  return PDF_OK;
}

extern "C" int pdf_batch_destroy(int32_t plan) {
  std::lock_guard<std::mutex> lock(g_mu);
  Plan* P = get_plan(plan);
  if (!P) return fail(PDF_ERR_ARG, "unknown plan %d", plan);
  plan_release(*P);
  return PDF_OK;
}

namespace {
int batched_one_shot(const pdf_request* reqs, int32_t n_req, int32_t out_f64, pdf_stream_t stream) {
  int32_t plan = -1;
  int rc = pdf_batch_create(reqs, n_req, out_f64, &plan);
  if (rc != PDF_OK) return rc;
  rc = pdf_batch_run(plan, stream);
  if (rc == PDF_OK) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) rc = fail_hip(e, "hipStreamSynchronize");
  }
  pdf_batch_destroy(plan);
  return rc;
}
}  // namespace

extern "C" int pdf_xfxq2_batched(const pdf_request* reqs, int32_t n_req, pdf_stream_t stream) {
  return batched_one_shot(reqs, n_req, 0, stream);
}

extern "C" int pdf_xfxq2_batched_f64(const pdf_request* reqs, int32_t n_req, pdf_stream_t stream) {
  return batched_one_shot(reqs, n_req, 1, stream);
}

// ---------------------------------------------------------------------------------------
// MLP surrogates

namespace {

struct Surrogate {
  bool used = false;
  int member = -1;
  uint64_t member_gen = 0;   // load generation of the member the surrogate was built on
  SurDev sd{};
  SurBufs b{};
  void* pmem = nullptr;      // parameters, moments, gradients, envelope tables
  void* bmem = nullptr;      // training workspace (sized for batches of up to bcap rows)
  int bcap = 0;
  float* d_in = nullptr;     // training inputs [n][2]
  float* d_t = nullptr;      // training targets [n][kO]
  int64_t n_train = 0;
  int64_t step = 0;          // Adam steps taken
  uint64_t seed = 0;
  // one training step recorded as a graph (replayed per step), valid for g_batch and g_in
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int g_batch = 0;
  const float* g_in = nullptr;
  const void* g_bmem = nullptr;
};

std::vector<Surrogate> g_surs;

Surrogate* get_sur(int32_t id) {
  if (id < 0 || id >= (int32_t)g_surs.size() || !g_surs[id].used) return nullptr;
  return &g_surs[id];
}

// The surrogate's member, or null once it was unloaded (or its slot reused).
Member* sur_member(const Surrogate& S) {
  Member* M = get_member(S.member);
  return M && M->gen == S.member_gen ? M : nullptr;
}

void sur_free_graph(Surrogate& S) {
  if (S.exec) (void)hipGraphExecDestroy(S.exec);
  if (S.graph) (void)hipGraphDestroy(S.graph);
  S.exec = nullptr;
  S.graph = nullptr;
  S.g_batch = 0;
  S.g_in = nullptr;
  S.g_bmem = nullptr;
}

void sur_release(Surrogate& S) {
  sur_free_graph(S);
  if (S.cap) (void)hipStreamDestroy(S.cap);
  if (S.pmem) (void)hipFree(S.pmem);
  if (S.bmem) (void)hipFree(S.bmem);
  if (S.d_in) (void)hipFree(S.d_in);
  S = Surrogate();
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Glorot-uniform weights, zero biases, from a counter-based generator.
std::vector<float> sur_init_params(uint64_t seed) {
  const int H = sur_hidden(), O = sur_out_width();
  std::vector<float> p((size_t)sur_nparams(), 0.0f);
  uint64_t st = seed;
  auto fill = [&](size_t off, int fan_out, int fan_in) {
    const double a = std::sqrt(6.0 / (fan_in + fan_out));
    for (int i = 0; i < fan_out * fan_in; ++i) {
      const double u = (double)(splitmix64(st) >> 11) * (1.0 / 9007199254740992.0);
      p[off + i] = (float)((2.0 * u - 1.0) * a);
    }
  };
  size_t off = 0;
  fill(off, H, 2); off += (size_t)H * 2 + H;
  fill(off, H, H); off += (size_t)H * H + H;
  fill(off, H, H); off += (size_t)H * H + H;
  fill(off, O, H);
  return p;
}

int sur_ensure_batch(Surrogate& S, int B) {
  if (B <= S.bcap) return PDF_OK;
  if (S.bmem) (void)hipFree(S.bmem);
  S.bmem = nullptr;
  // the fused training step's per-slice partial gradients and losses
  hipError_t e = hipMalloc(&S.bmem, sur_workspace_floats(B) * 4);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(surrogate batch)");
  S.b.wpart = static_cast<float*>(S.bmem);
  S.bcap = B;
  return PDF_OK;
}

constexpr char kSurMagic[8] = {'P', 'D', 'F', 'M', 'I', 'S', 'R', '1'};

uint64_t fnv1a(const unsigned char* p, size_t n, uint64_t h = 1469598103934665603ull) {
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

}  // namespace

extern "C" int pdf_surrogate_param_count(int32_t* n_out) {
  if (!n_out) return fail(PDF_ERR_ARG, "null n_out");
  *n_out = sur_nparams();
  return PDF_OK;
}

extern "C" int pdf_surrogate_create(int32_t member, uint64_t seed, int32_t* sid_out) {
  if (!sid_out) return fail(PDF_ERR_ARG, "null sid_out");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_init();
  if (rc != PDF_OK) return rc;
  Member* M = get_member(member);
  if (!M) return fail(PDF_ERR_MEMBER, "unknown member %d", member);
  const int O = sur_out_width(), NP = sur_nparams();
  const int P = (int)M->pids.size();
  if (P > O) return fail(PDF_ERR_ARG, "surrogate supports at most %d stored flavours", O);
  const int K = (int)M->h_shape.size() / 2;
  const int nx0 = M->h_shape[0];
  const double* xk0 = M->h_knots.data();
  // envelope over sub-grid 0's x knots: at each, the value of largest magnitude over every Q^2 knot of every
  // sub-grid (signed); slopes d E / d ln x by finite differences (mean of the adjacent secants, one-sided at
  // the ends)
  std::vector<double> envv((size_t)nx0 * O, 0.0), enva((size_t)nx0 * O, -1.0), lxk(nx0);
  for (int i = 0; i < nx0; ++i) lxk[i] = std::log(xk0[i]);
  int64_t ko = 0, vo = 0;
  for (int k = 0; k < K; ++k) {
    const int nx = M->h_shape[2 * k], nq = M->h_shape[2 * k + 1];
    const double* xk = M->h_knots.data() + ko;
    for (int ix = 0; ix < nx; ++ix) {
      int i0 = 0;  // nearest sub-grid-0 knot
      for (int j = 0; j < nx0; ++j)
        if (std::fabs(std::log(xk0[j] / xk[ix])) < std::fabs(std::log(xk0[i0] / xk[ix]))) i0 = j;
      for (int iq = 0; iq < nq; ++iq)
        for (int c = 0; c < P; ++c) {
          const double v = M->h_values[vo + ((int64_t)ix * nq + iq) * P + c];
          if (std::fabs(v) > enva[(size_t)i0 * O + c]) {
            enva[(size_t)i0 * O + c] = std::fabs(v);
            envv[(size_t)i0 * O + c] = v;
          }
        }
    }
    ko += nx + nq;
    vo += (int64_t)nx * nq * P;
  }
  std::vector<float> env((size_t)nx0 * O), envd((size_t)nx0 * O);
  for (int i = 0; i < nx0; ++i)
    for (int c = 0; c < O; ++c) {
      auto sec = [&](int j) {  // secant over cell j
        return (envv[(size_t)(j + 1) * O + c] - envv[(size_t)j * O + c]) / (lxk[j + 1] - lxk[j]);
      };
      const double d = i == 0 ? sec(0) : i == nx0 - 1 ? sec(nx0 - 2) : 0.5 * (sec(i - 1) + sec(i));
      env[(size_t)i * O + c] = (float)envv[(size_t)i * O + c];
      envd[(size_t)i * O + c] = (float)d;
    }
  Surrogate S;
  S.used = true;
  S.member = member;
  S.member_gen = M->gen;
  S.seed = seed;
  S.sd.P = P;
  S.sd.nx = nx0;
  S.sd.lx0 = std::log(M->dev.xmin);
  S.sd.ilx = 1.0 / (std::log(M->dev.xmax) - std::log(M->dev.xmin));
  S.sd.lq0 = std::log(M->dev.qmin);
  S.sd.ilq = 1.0 / (std::log(M->dev.qmax) - std::log(M->dev.qmin));
  if (nx0 > kSurMaxEnvKnots)
    return fail(PDF_ERR_GRID, "surrogate envelope supports at most %d x knots", kSurMaxEnvKnots);
  {
    int64_t o = 0;
    for (int k = 0; k < K; ++k) {
      const int nx = M->h_shape[2 * k], nq = M->h_shape[2 * k + 1];
      const double* xk = M->h_knots.data() + o;
      const double* qk = xk + nx;
      S.sd.trust[k] = nx >= 4 && nq >= 4;
      S.sd.txlo[k] = S.sd.trust[k] ? xk[1] : 0.0;
      S.sd.txhi[k] = S.sd.trust[k] ? xk[nx - 2] : 0.0;
      S.sd.tqlo[k] = S.sd.trust[k] ? qk[1] : 0.0;
      S.sd.tqhi[k] = S.sd.trust[k] ? qk[nq - 2] : 0.0;
      o += nx + nq;
    }
  }
  const size_t bp = align_up((size_t)NP * 4, 256), bpb = align_up((size_t)NP * 4, 256);  // Pb: hi and lo halves
  const size_t be = align_up(env.size() * 4, 256), bl = align_up(lxk.size() * 8, 256);
  hipError_t e = hipMalloc(&S.pmem, 4 * bp + bpb + 2 * be + bl + 2048 + align_up(sizeof(SurStep), 256));
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(surrogate)");
  unsigned char* b = static_cast<unsigned char*>(S.pmem);
  S.b.P = reinterpret_cast<float*>(b);
  S.b.M = reinterpret_cast<float*>(b + bp);
  S.b.V = reinterpret_cast<float*>(b + 2 * bp);
  S.b.G = reinterpret_cast<float*>(b + 3 * bp);
  S.b.Pb = reinterpret_cast<unsigned short*>(b + 4 * bp);
  float* envdev = reinterpret_cast<float*>(b + 4 * bp + bpb);
  float* envddev = reinterpret_cast<float*>(b + 4 * bp + bpb + be);
  double* lxkd = reinterpret_cast<double*>(b + 4 * bp + bpb + 2 * be);
  S.b.loss = reinterpret_cast<float*>(b + 4 * bp + bpb + 2 * be + bl);
  S.b.st = reinterpret_cast<SurStep*>(b + 4 * bp + bpb + 2 * be + bl + 2048);
  S.sd.env = envdev;
  S.sd.envd = envddev;
  S.sd.lxk = lxkd;
  const std::vector<float> p0 = sur_init_params(seed);
  std::vector<float> zeros((size_t)NP, 0.0f);
  if ((e = hipMemcpy(S.b.P, p0.data(), (size_t)NP * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(S.b.M, zeros.data(), (size_t)NP * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(S.b.V, zeros.data(), (size_t)NP * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(envdev, env.data(), env.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(envddev, envd.data(), envd.size() * 4, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(lxkd, lxk.data(), lxk.size() * 8, hipMemcpyHostToDevice)) != hipSuccess ||
      (e = sur_refresh_bf16(S.b, nullptr)) != hipSuccess || (e = hipDeviceSynchronize()) != hipSuccess) {
    sur_release(S);
    return fail_hip(e, "surrogate upload");
  }
  for (size_t i = 0; i < g_surs.size(); ++i)
    if (!g_surs[i].used) {
      g_surs[i] = S;
      *sid_out = (int32_t)i;
      return PDF_OK;
    }
  g_surs.push_back(S);
  *sid_out = (int32_t)(g_surs.size() - 1);
  return PDF_OK;
}

extern "C" int pdf_surrogate_destroy(int32_t sid) {
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  sur_release(*S);
  return PDF_OK;
}

extern "C" int pdf_surrogate_set_data(int32_t sid, const double* x, const double* q2, int64_t n,
                                      pdf_stream_t stream) {
  if (n < 16 || !x || !q2) return fail(PDF_ERR_ARG, "need >= 16 device training points");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  Member* M = sur_member(*S);
  if (!M) return fail(PDF_ERR_MEMBER, "surrogate's member %d was unloaded", S->member);
  hipStream_t s = (hipStream_t)stream;
  const int O = sur_out_width(), P = (int)M->pids.size();
  // the old set is released first; until the new one is complete, training finds no data
  sur_free_graph(*S);
  if (S->d_in) (void)hipFree(S->d_in);
  S->d_in = nullptr;
  S->d_t = nullptr;
  S->n_train = 0;
  // every sample: inputs, targets, in-domain flag; then the in-domain samples, in order
  void* tmp = nullptr;
  const size_t b_in = align_up((size_t)n * (2 + O) * 4, 256), b_xf = align_up((size_t)n * P * 8, 256);
  hipError_t e = hipMalloc(&tmp, b_in + b_xf + align_up((size_t)n, 256) + (size_t)n * 8);
  if (e != hipSuccess) return fail_hip(e, "hipMalloc(training samples)");
  float* in_all = static_cast<float*>(tmp);
  float* t_all = in_all + 2 * n;
  double* xf = reinterpret_cast<double*>(static_cast<unsigned char*>(tmp) + b_in);
  unsigned char* keep = static_cast<unsigned char*>(tmp) + b_in + b_xf;
  int64_t* idx = reinterpret_cast<int64_t*>(keep + align_up((size_t)n, 256));
  ReqCols rc{};
  build_req(*M, nullptr, 0, rc);
  // targets from this library's FP64 interpolator
  const LaunchCfg cfg{g_ncu, g_blocks_per_cu, g_vector_cols};
  e = launch_xfxq2_f64(M->dev, rc, x, q2, n, xf, g_nerr, lds_grid_elems(*M, false, n), M->invL01, cfg, nullptr,
                       nullptr, s);
  if (e == hipSuccess) e = sur_prep(S->sd, M->dev, x, q2, xf, n, in_all, t_all, keep, s);
  std::vector<unsigned char> hkeep((size_t)n);
  if (e == hipSuccess) e = hipMemcpyAsync(hkeep.data(), keep, (size_t)n, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  std::vector<int64_t> hidx;
  if (e == hipSuccess) {
    hidx.reserve((size_t)n);
    for (int64_t i = 0; i < n; ++i)
      if (hkeep[(size_t)i]) hidx.push_back(i);
  }
  const int64_t nk = (int64_t)hidx.size();
  float* din = nullptr;
  if (e == hipSuccess && nk < 16) {
    (void)hipFree(tmp);
    return fail(PDF_ERR_ARG, "only %lld of the %lld points lie in the network's domain (need >= 16)",
                (long long)nk, (long long)n);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(idx, hidx.data(), (size_t)nk * 8, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMalloc(&din, (size_t)nk * (2 + O) * 4);
  if (e == hipSuccess) e = sur_gather(in_all, t_all, idx, nk, din, din + 2 * nk, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  (void)hipFree(tmp);
  if (e != hipSuccess) {
    if (din) (void)hipFree(din);
    return fail_hip(e, "surrogate targets");
  }
  S->d_in = din;
  S->d_t = din + 2 * nk;
  S->n_train = nk;
  return PDF_OK;
}

extern "C" int pdf_surrogate_train(int32_t sid, const pdf_train_opts* opts, pdf_stream_t stream) {
  if (!opts) return fail(PDF_ERR_ARG, "null opts");
  const int steps = opts->steps, batch = opts->batch;
  if (steps < 0 || batch < 16 || (batch & 15) || opts->total_steps < 1 || !(opts->lr >= 0.0f) ||
      !(opts->lr_final >= 0.0f))
    return fail(PDF_ERR_ARG, "bad training options");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  if (S->n_train < batch) return fail(PDF_ERR_STATE, "training data smaller than one batch (call set_data)");
  int rc = sur_ensure_batch(*S, batch);
  if (rc != PDF_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int64_t nb = S->n_train / batch;
  if (steps == 0) return PDF_OK;
  hipError_t e = sur_train_prepare();
  if (e != hipSuccess) return fail_hip(e, "surrogate training set-up");
  e = sur_train_begin(S->b, S->step, nb, opts->total_steps, opts->lr, opts->lr_final, opts->loss_out, s);
  if (e != hipSuccess) return fail_hip(e, "surrogate training start");
  if (opts->use_graph) {
    if (!S->exec || S->g_batch != batch || S->g_in != S->d_in || S->g_bmem != S->bmem) {
      sur_free_graph(*S);
      if (!S->cap && (e = hipStreamCreateWithFlags(&S->cap, hipStreamNonBlocking)) != hipSuccess)
        return fail_hip(e, "hipStreamCreate(capture)");
      if ((e = hipStreamBeginCapture(S->cap, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return fail_hip(e, "hipStreamBeginCapture");
      const hipError_t e1 = sur_train_step(S->b, S->d_in, S->d_t, batch, S->cap);
      e = hipStreamEndCapture(S->cap, &S->graph);
      if (e1 != hipSuccess || e != hipSuccess) {
        sur_free_graph(*S);
        return fail_hip(e1 != hipSuccess ? e1 : e, "capture of a training step");
      }
      if ((e = hipGraphInstantiate(&S->exec, S->graph, nullptr, nullptr, 0)) != hipSuccess) {
        sur_free_graph(*S);
        return fail_hip(e, "hipGraphInstantiate(training step)");
      }
      S->g_batch = batch;
      S->g_in = S->d_in;
      S->g_bmem = S->bmem;
    }
    for (int i = 0; i < steps; ++i)
      if ((e = hipGraphLaunch(S->exec, s)) != hipSuccess) return fail_hip(e, "hipGraphLaunch(training step)");
  } else {
    for (int i = 0; i < steps; ++i)
      if ((e = sur_train_step(S->b, S->d_in, S->d_t, batch, s)) != hipSuccess)
        return fail_hip(e, "surrogate training step");
  }
  S->step += steps;
  return PDF_OK;
}

extern "C" int pdf_surrogate_grad(int32_t sid, const float* in, const float* target, int32_t batch, float* grad_out,
                                  float* loss_out, pdf_stream_t stream) {
  if (!in || !target || !grad_out || !loss_out || batch < 16 || (batch & 15))
    return fail(PDF_ERR_ARG, "bad gradient arguments");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  int rc = sur_ensure_batch(*S, batch);
  if (rc != PDF_OK) return rc;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = sur_forward_backward(S->b, in, target, batch, loss_out, s);
  if (e == hipSuccess) e = hipMemcpyAsync(grad_out, S->b.G, (size_t)sur_nparams() * 4, hipMemcpyDeviceToDevice, s);
  if (e != hipSuccess) return fail_hip(e, "surrogate gradient");
  return PDF_OK;
}

extern "C" int pdf_surrogate_adam(int32_t sid, const float* grad, float lr, pdf_stream_t stream) {
  if (!grad || !(lr >= 0.0f)) return fail(PDF_ERR_ARG, "bad Adam arguments");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = hipMemcpyAsync(S->b.G, grad, (size_t)sur_nparams() * 4, hipMemcpyDeviceToDevice, s);
  if (e == hipSuccess) e = sur_adam(S->b, lr, (int)(S->step + 1), s);
  if (e != hipSuccess) return fail_hip(e, "surrogate Adam step");
  ++S->step;
  return PDF_OK;
}

extern "C" int pdf_surrogate_params(int32_t sid, float* host, int32_t write) {
  if (!host) return fail(PDF_ERR_ARG, "null host buffer");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  const size_t nb = (size_t)sur_nparams() * 4;
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) {
    if (write) {
      e = hipMemcpy(S->b.P, host, nb, hipMemcpyHostToDevice);
      if (e == hipSuccess) e = sur_refresh_bf16(S->b, nullptr);
      if (e == hipSuccess) e = hipDeviceSynchronize();
    } else {
      e = hipMemcpy(host, S->b.P, nb, hipMemcpyDeviceToHost);
    }
  }
  if (e != hipSuccess) return fail_hip(e, "surrogate parameters");
  return PDF_OK;
}

extern "C" int pdf_surrogate_xfxq2(int32_t sid, const int32_t* pids, int32_t n_pids, const double* x,
                                   const double* q2, int64_t n, float* out, pdf_stream_t stream) {
  int rc = check_stream_args(x, q2, n);
  if (rc != PDF_OK) return rc;
  if (n > 0 && !out) return fail(PDF_ERR_ARG, "null out");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  Member* M = sur_member(*S);
  if (!M) return fail(PDF_ERR_MEMBER, "surrogate's member %d was unloaded", S->member);
  ReqCols cols{};
  if ((rc = build_req(*M, pids, n_pids, cols)) != PDF_OK) return rc;
  if (n == 0 || cols.n == 0) return PDF_OK;
  hipError_t e = sur_infer(S->sd, M->dev, cols, S->b, x, q2, n, out, M->invL01, g_nerr, g_ncu, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch surrogate inference");
  return PDF_OK;
}

extern "C" int pdf_surrogate_save(int32_t sid, const char* path) {
  if (!path) return fail(PDF_ERR_ARG, "null path");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  const int NP = sur_nparams();
  std::vector<float> buf((size_t)3 * NP);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(buf.data(), S->b.P, (size_t)NP * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + NP, S->b.M, (size_t)NP * 4, hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(buf.data() + 2 * NP, S->b.V, (size_t)NP * 4, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return fail_hip(e, "surrogate save");
  const uint32_t version = 1, np = (uint32_t)NP;
  const int64_t step = S->step;
  uint64_t h = fnv1a(reinterpret_cast<const unsigned char*>(&step), 8);
  h = fnv1a(reinterpret_cast<const unsigned char*>(buf.data()), buf.size() * 4, h);
  FILE* f = fopen(path, "wb");
  if (!f) return fail(PDF_ERR_ARG, "cannot open %s for writing", path);
  bool ok = fwrite(kSurMagic, 1, 8, f) == 8 && fwrite(&version, 4, 1, f) == 1 && fwrite(&np, 4, 1, f) == 1 &&
            fwrite(&step, 8, 1, f) == 1 && fwrite(buf.data(), 4, buf.size(), f) == buf.size() &&
            fwrite(&h, 8, 1, f) == 1;
  ok = (fclose(f) == 0) && ok;
  if (!ok) return fail(PDF_ERR_ARG, "write to %s failed", path);
  return PDF_OK;
}

extern "C" int pdf_surrogate_load(int32_t sid, const char* path) {
  if (!path) return fail(PDF_ERR_ARG, "null path");
  std::lock_guard<std::mutex> lock(g_mu);
  Surrogate* S = get_sur(sid);
  if (!S) return fail(PDF_ERR_ARG, "unknown surrogate %d", sid);
  const int NP = sur_nparams();
  FILE* f = fopen(path, "rb");
  if (!f) return fail(PDF_ERR_ARG, "cannot open %s", path);
  char mg[8];
  uint32_t version = 0, np = 0;
  int64_t step = 0;
  uint64_t h = 0;
  std::vector<float> buf((size_t)3 * NP);
  bool ok = fread(mg, 1, 8, f) == 8 && fread(&version, 4, 1, f) == 1 && fread(&np, 4, 1, f) == 1;
  ok = ok && std::memcmp(mg, kSurMagic, 8) == 0 && version == 1 && np == (uint32_t)NP;
  ok = ok && fread(&step, 8, 1, f) == 1 && fread(buf.data(), 4, buf.size(), f) == buf.size() &&
       fread(&h, 8, 1, f) == 1;
  fclose(f);
  if (!ok) return fail(PDF_ERR_ARG, "%s is not a surrogate checkpoint of this layout", path);
  uint64_t h2 = fnv1a(reinterpret_cast<const unsigned char*>(&step), 8);
  h2 = fnv1a(reinterpret_cast<const unsigned char*>(buf.data()), buf.size() * 4, h2);
  if (h2 != h) return fail(PDF_ERR_ARG, "%s: checksum mismatch", path);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess) e = hipMemcpy(S->b.P, buf.data(), (size_t)NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(S->b.M, buf.data() + NP, (size_t)NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(S->b.V, buf.data() + 2 * NP, (size_t)NP * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = sur_refresh_bf16(S->b, nullptr);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) return fail_hip(e, "surrogate load");
  S->step = step;
  return PDF_OK;
}

extern "C" int pdf_mc_workspace_bytes(int64_t n, int64_t* bytes_out) {
  if (!bytes_out || n < 0) return fail(PDF_ERR_ARG, "bad argument");
  *bytes_out = (n == 0 ? 1 : mc_partials(n)) * (int64_t)sizeof(double);
  return PDF_OK;
}

template <typename T>
static int mc_sum_impl(const T* xf1, const T* xf2, int32_t n_pids, const double* alphas, int64_t n, double* workspace,
                       double* sum_out, pdf_stream_t stream) {
  if (n < 0 || n_pids < 1 || n_pids > kMaxReq) return fail(PDF_ERR_ARG, "bad n or n_pids");
  if (!sum_out || !workspace) return fail(PDF_ERR_ARG, "null output or workspace");
  if (n > 0 && (!xf1 || !xf2 || !alphas)) return fail(PDF_ERR_ARG, "null input");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_init();
  if (rc != PDF_OK) return rc;
  hipError_t e = launch_mc_sum<T>(xf1, xf2, n_pids, alphas, n, workspace, sum_out, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch mc sum");
  return PDF_OK;
}

extern "C" int pdf_mc_chunk_sum(const double* xf1, const double* xf2, int32_t n_pids, const double* alphas, int64_t n,
                                double* workspace, double* sum_out, pdf_stream_t stream) {
  return mc_sum_impl<double>(xf1, xf2, n_pids, alphas, n, workspace, sum_out, stream);
}

extern "C" int pdf_mc_chunk_sum_f32(const float* xf1, const float* xf2, int32_t n_pids, const double* alphas,
                                    int64_t n, double* workspace, double* sum_out, pdf_stream_t stream) {
  return mc_sum_impl<float>(xf1, xf2, n_pids, alphas, n, workspace, sum_out, stream);
}

template <typename T>
static int mc_fused_impl(int32_t member, const int32_t* pids, int32_t n_pids, const double* x1, const double* x2,
                         const double* q2, int64_t n, double* workspace, double* sum_out, pdf_stream_t stream) {
  if (n < 0) return fail(PDF_ERR_ARG, "n < 0");
  if (!sum_out || !workspace) return fail(PDF_ERR_ARG, "null output or workspace");
  if (n > 0 && (!x1 || !x2 || !q2)) return fail(PDF_ERR_ARG, "null input");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_init();
  if (rc != PDF_OK) return rc;
  Member* M = get_member(member);
  if (!M) return fail(PDF_ERR_MEMBER, "unknown member %d", member);
  if (!g_has_alphas) return fail(PDF_ERR_STATE, "no alpha_s table loaded");
  ReqCols rcols{};
  if ((rc = build_req(*M, pids, n_pids, rcols)) != PDF_OK) return rc;
  if (mc_fused_shared_bytes(M->dev, g_alphas, 0, sizeof(T) == 4) > kLdsBytes)
    return fail(PDF_ERR_GRID, "location tables too large for the fused kernel; use pdf_xfxq2 + pdf_mc_chunk_sum");
  hipError_t e = launch_mc_fused<T>(M->dev, rcols, g_alphas, x1, x2, q2, n, workspace, sum_out, g_nerr, M->invL01,
                                    g_ncu, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch fused mc sum");
  return PDF_OK;
}

extern "C" int pdf_mc_fused(int32_t member, const int32_t* pids, int32_t n_pids, const double* x1, const double* x2,
                            const double* q2, int64_t n, double* workspace, double* sum_out, pdf_stream_t stream) {
  return mc_fused_impl<double>(member, pids, n_pids, x1, x2, q2, n, workspace, sum_out, stream);
}

extern "C" int pdf_mc_fused_f32(int32_t member, const int32_t* pids, int32_t n_pids, const double* x1,
                                const double* x2, const double* q2, int64_t n, double* workspace, double* sum_out,
                                pdf_stream_t stream) {
  return mc_fused_impl<float>(member, pids, n_pids, x1, x2, q2, n, workspace, sum_out, stream);
}

extern "C" int pdf_fk_contract(const double* pdf, const double* fk, int32_t nrep, int32_t ndat, int64_t K,
                               double* out, pdf_stream_t stream) {
  if (nrep < 0 || ndat < 0 || K < 0) return fail(PDF_ERR_ARG, "negative size");
  if (nrep > (1 << 22)) return fail(PDF_ERR_ARG, "nrep above 4194304");
  if (nrep > 0 && ndat > 0 && (!out || (K > 0 && (!pdf || !fk)))) return fail(PDF_ERR_ARG, "null device pointer");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_init();
  if (rc != PDF_OK) return rc;
  if (nrep == 0 || ndat == 0) return PDF_OK;
  const int S = fk_slices(nrep, ndat, K, g_ncu);
  const size_t need = S > 1 ? (size_t)S * nrep * ndat * sizeof(double) : 0;
  if (need > g_fk_ws_bytes) {
    // the stream's earlier work may still read the old buffer
    hipError_t e = g_fk_ws ? hipStreamSynchronize((hipStream_t)stream) : hipSuccess;
    if (e != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
    if (g_fk_ws) (void)hipFree(g_fk_ws);
    g_fk_ws = nullptr;
    g_fk_ws_bytes = 0;
    e = hipMalloc(&g_fk_ws, need);
    if (e != hipSuccess) return fail_hip(e, "hipMalloc(fk workspace)");
    g_fk_ws_bytes = need;
  }
  hipError_t e = launch_fk_contract(pdf, fk, nrep, ndat, K, out, S, static_cast<double*>(g_fk_ws),
                                    (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch fk contraction");
  return PDF_OK;
}

extern "C" int pdf_fk_contract_noalloc(const double* pdf, const double* fk, int32_t nrep, int32_t ndat, int64_t K,
                                       double* out, pdf_stream_t stream) {
  if (nrep < 0 || ndat < 0 || K < 0) return fail(PDF_ERR_ARG, "negative size");
  if (nrep > (1 << 22)) return fail(PDF_ERR_ARG, "nrep above 4194304");
  if (nrep > 0 && ndat > 0 && (!out || (K > 0 && (!pdf || !fk)))) return fail(PDF_ERR_ARG, "null device pointer");
  std::lock_guard<std::mutex> lock(g_mu);
  int rc = ensure_device();
  if (rc != PDF_OK) return rc;
  if (nrep == 0 || ndat == 0) return PDF_OK;
  const int S = fk_slices(nrep, ndat, K, g_ncu);
  const size_t need = S > 1 ? (size_t)S * nrep * ndat * sizeof(double) : 0;
  if (need > fk_scratch_bytes())
    return fail(PDF_ERR_ARG, "partial sums of %d K slices x %d x %d doubles need %zu bytes, above the %zu-byte scratch",
                S, nrep, ndat, need, fk_scratch_bytes());
  // every partial sum is written by the contraction kernel before the reduction reads it: nothing to clear
  hipError_t e = launch_fk_contract(pdf, fk, nrep, ndat, K, out, S, g_fk_scratch, (hipStream_t)stream);
  if (e != hipSuccess) return fail_hip(e, "launch fk contraction");
  return PDF_OK;
}

extern "C" int pdf_set_lds_policy(int32_t policy) {
  if (policy < 0 || policy > 2) return fail(PDF_ERR_ARG, "policy must be 0, 1 or 2");
  std::lock_guard<std::mutex> lock(g_mu);
  g_lds_policy = policy;
  return PDF_OK;
}

extern "C" const char* pdf_last_error(void) { return g_err.c_str(); }

extern "C" int pdf_shutdown(void) {
  std::lock_guard<std::mutex> lock(g_mu);
  for (auto& M : g_members)
    if (M.used && M.dmem) (void)hipFree(M.dmem);
  g_members.clear();
  if (g_alphas_mem) (void)hipFree(g_alphas_mem);
  g_alphas_mem = nullptr;
  g_has_alphas = false;
  for (auto& P : g_plans)
    if (P.used) plan_release(P);
  g_plans.clear();
  for (auto& S : g_surs)
    if (S.used) sur_release(S);
  g_surs.clear();
  if (g_nerr) (void)hipFree(g_nerr);
  g_nerr = nullptr;
  if (g_fk_ws) (void)hipFree(g_fk_ws);
  g_fk_ws = nullptr;
  g_fk_ws_bytes = 0;
  g_fk_scratch = nullptr;  // the array itself stays with the process
  g_dev_ready = false;
  g_init = false;
  return PDF_OK;
}
