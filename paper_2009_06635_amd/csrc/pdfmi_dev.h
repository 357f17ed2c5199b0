// Device-side data layout shared by the host runtime (pdfmi.cpp) and the
// kernels (kernels.hip).  Not part of the public ABI.
#pragma once
#include <stdint.h>

#include <map>
#include <mutex>
#include <utility>

#include <hip/hip_runtime.h>

namespace pdfmi {

constexpr int kMaxSub = 16;      // Q^2 sub-grids per member
constexpr int kMaxReq = 64;      // flavours per query call
constexpr int kMaxSeg = 16;      // alpha_s segments

// Region / mode bits of a query point.
enum : int { kLowX = 1, kLowQ = 2, kHighQ = 4, kInvalid = 8, kXHigh = 16 };

// Per-cell Hermite data of one 1D knot table (cell i = [t_i, t_{i+1}]), FP64,
// computed on the host.  With Hermite basis h00,h10,h01,h11 of the cell
// parameter u, the weights of the four knots i-1..i+2 are
//   w(-1) = h10*am1
//   w(0)  = h00 + h10*a0 + h11*b0
//   w(1)  = h01 + h10*a1 + h11*b1
//   w(2)  = h11*b2
// where (am1,a0,a1) expand Delta_i * slope_i and (b0,b1,b2) expand
// Delta_i * slope_{i+1} over the knot values (finite-difference slopes:
// mean of adjacent secants inside the table, the one secant at its ends).
// Inside the table they depend only on hl = Delta_i / (2 Delta_{i-1}) and
// hr = Delta_i / (2 Delta_{i+1}):
//   am1 = -hl, a0 = hl - 1/2, a1 = 1/2;   b0 = -1/2, b1 = 1/2 - hr, b2 = hr;
// at the table's first cell (no left neighbour, hl < 0 marks it)
//   am1 = 0, a0 = -1, a1 = 1, and at its last cell (hr < 0)
//   b0 = -1, b1 = 1, b2 = 0.  48 bytes: three 16-byte LDS reads per cell.
struct CellCoef {
  double t0;      // knot i
  double t1;      // knot i+1
  double inv_t0;  // 1 / knot i
  double invD;    // 1 / ln(t1 / t0)
  double hl, hr;  // half ratios of the neighbouring cells' log-widths, or -1 at a table edge
};

// Knot search by bucket hints: positive doubles order like their IEEE-754
// bit patterns, so the key (bits >> shift) of a query selects a bucket of a
// 1D knot table; the bucket's hint is the largest cell index whose knot is
// <= the bucket's smallest value, and at most two more knots lie inside any
// bucket.  The cell of v is then the hint advanced over the next two knots
// that are <= v -- the same index as a binary search with the same raw FP64
// comparisons.  A table with no hint list (off < 0) is binary searched.
struct HintAxis {
  int off;        // first hint in MemberDev::hints, -1 for none
  int n;          // buckets
  int shift;      // key = (unsigned)(bits(v) >> shift)
  unsigned key0;  // key of the first knot
};

struct SubDesc {
  int nx, nq;        // knot counts
  int nxp, nqp;      // storage extents (>= 4; rows beyond the knots are zero)
  int xk_off, qk_off;  // knot offsets (doubles) into MemberDev::knots
  int xc_off, qc_off;  // cell offsets into MemberDev::cells
  HintAxis xh, qh;     // knot-search hints of the two axes
  int64_t val_off64;   // element offset of values[ix][iq][c] into v64 (row stride P64)
  int64_t val_off32;   // element offset into v32 (row stride P32)
  double qfirst;       // first Q^2 knot
};

// The point-location tables of a member (knots, cell coefficients, search
// hints, sub-grid descriptors) are one contiguous device block of tbl_bytes,
// copied whole into LDS by the kernels when it fits there.
struct MemberDev {
  int K;                 // sub-grids
  int P;                 // stored columns
  int P64, P32;          // row strides of v64 / v32 (zero padding; FP64 rows are whole 64/128-byte lines)
  int64_t elems64, elems32;  // value elements (padded) of v64 / v32
  int nknots;            // total knots (all sub-grids, x then Q^2 each; shared x tables stored once)
  int nknots_pad;        // nknots rounded up to an even count
  int tbl_bytes;         // bytes of the location-table block (multiple of 16)
  int cells_off, hints_off, subs_off;  // byte offsets of cells, hints and sub-grid descriptors in it
  double xmin, xmax;     // x range (shared by all sub-grids)
  double qmin, qmax;     // Q^2 range (first knot of sub-grid 0, last of K-1)
  const unsigned char* tables;  // device, the location-table block
  const double* knots;   // device, = tables
  const CellCoef* cells; // device, = tables + cells_off
  const short* hints;    // device, = tables + hints_off
  const SubDesc* subs;   // device, = tables + subs_off
  const double* v64;     // device, FP64 values
  const float* v32;      // device, FP32-rounded values
  SubDesc sub[kMaxSub];
};

struct ReqCols {
  int n;             // requested flavours
  int col[kMaxReq];  // stored column, or -1 for a valid flavour absent from the grid
};

struct LaunchCfg {
  int n_cu;           // compute units
  int blocks_per_cu;  // workgroups per CU for the global-grid kernels
  int vector_cols;    // use G-wide column groups for all-column requests
};

struct AlphasDev {
  int n;                   // knots
  int nseg;
  int nhints;              // search hints (all segments)
  int seg_lo[kMaxSeg];     // first knot index of each segment
  int seg_hi[kMaxSeg];     // last knot index of each segment
  double seg_first[kMaxSeg];
  HintAxis seg_hint[kMaxSeg];  // knot-search hints of each segment (off < 0: binary search)
  const double* knots;     // device, n
  const double* vals;      // device, n
  const CellCoef* cells;   // device, cell j = [knot j, knot j+1] (within a segment)
  const short* hints;      // device, nhints
};

}  // namespace pdfmi

namespace pdfmi {

// One request of a batched plan (device copy).
struct BatchReq {
  int member;        // index into the plan's member table
  int R;             // requested flavours
  int col_off;       // offset of this request's column list in the plan's column array
  int all_cols;      // 1 if the request is every stored column in load order
  const double* x;
  const double* q2;
  void* out;         // FP32 or FP64 point-major [n][R], per the plan
  int64_t n;
};

// A tile: tile_points consecutive points of one request (the last tile of a
// request may be shorter).
struct BatchTile {
  int req;
  int count;
  int64_t start;
};

// Kernel node parameters of one batched run (counter reset + persistent kernel).
struct BatchLaunch {
  const void* reset_fn;
  const void* main_fn;
  unsigned grid;
  size_t shm;
};

// Surrogate input normalisation and output envelope (device tables).  The
// envelope of column c is a signed cubic Hermite in ln x through one value
// per sub-grid-0 x knot (the grid value of largest magnitude over every Q^2
// knot at that x), with finite-difference slopes (mean of the adjacent
// secants, the one secant at the ends).
struct SurDev {
  int P;              // stored columns (<= 16)
  int nx;             // envelope knots (sub-grid 0 x knots)
  double lx0, ilx;    // u = 2 (ln x - lx0) * ilx - 1
  double lq0, ilq;    // v = 2 (ln Q^2 - lq0) * ilq - 1
  const double* lxk;  // [nx] ln of the envelope knots
  const float* env;   // [nx][16] envelope values
  const float* envd;  // [nx][16] envelope slopes d E / d ln x
  // inference trusts the network inside sub-grid k for txlo[k] <= x < txhi[k]
  // and tqlo[k] <= Q^2 < tqhi[k] (second to second-last knots) when trust[k]
  int trust[kMaxSub];
  double txlo[kMaxSub], txhi[kMaxSub], tqlo[kMaxSub], tqhi[kMaxSub];
};

// Device-side state of a surrogate's training call.  The training kernels
// read the global step (which batch slice, which learning rate) from here,
// so every step is the same launch sequence and can be replayed as a graph.
struct SurStep {
  int64_t step;      // global step: batch (step % nb), learning rate, Adam update number step + 1
  int64_t call;      // step index within the current train call (index into loss_out)
  int64_t nb;        // batches in the training set
  int total;         // cosine schedule length
  float lr0, lrf;    // schedule end points
  float* loss_out;   // the call's per-step losses, or null
  unsigned done;     // workgroups of the step's update kernel that have finished (the last one advances the step)
};

// Surrogate device buffers (parameters, Adam moments, gradient, training workspace).
// Matrix operands are BF16 pairs (hi, lo) with value = hi + lo.
struct SurBufs {
  float* P;                 // FP32 master parameters
  unsigned short* Pb;       // BF16 halves of the parameters: [0, n) hi, [n, 2n) lo
  float *M, *V, *G;         // Adam moments, gradient
  float* loss;              // [1]
  float* wpart;             // per-slice partial gradients and losses of a training step
  SurStep* st;              // training-call state
};

// hipFuncSetAttribute(MaxDynamicSharedMemorySize) only when a launch needs
// more dynamic LDS than the kernel was last allowed on this device: repeated
// launches of the same shape make no extra runtime call (it costs several
// microseconds, the whole duration of a small evaluation).
inline hipError_t allow_dynamic_lds(const void* fn, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, size_t> allowed;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lock(mu);
  size_t& a = allowed[{fn, dev}];
  if (bytes <= a) return hipSuccess;
  e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) a = bytes;
  return e;
}

}  // namespace pdfmi
