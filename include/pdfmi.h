/*
 * pdfmi.h -- C ABI of libpdfmi.so: parton-distribution and alpha_s
 * interpolation on AMD MI355X (gfx950).
 *
 * The operations are those of Carrazza, Cruz-Martinez, Rossi, "PDFFlow: parton
 * distribution functions on GPU": evaluate x*f(x,Q^2) for arrays of points and
 * a set of flavours (section 2.1, the xfxQ2 / xfxQ2_allpid methods of figure 1)
 * by log-bicubic interpolation on knot grids split into Q^2 sub-grids at
 * flavour thresholds, with extrapolation outside the grid (section 2.2, figure
 * 1 INTERPOLATE / EXTRAPOLATE), and alpha_s(Q^2) by log-cubic interpolation
 * with constant extrapolation (section 2.3).
 *
 * Interpolation rule (the paper defers to LHAPDF6 and prints no formula; this
 * library's reading): cubic Hermite in ln x, then in ln Q^2, with slopes from
 * finite differences (mean of the two adjacent secants inside a sub-grid, the
 * single secant at a sub-grid edge).  Knot search compares raw FP64 values.  A
 * Q^2 equal to a threshold knot belongs to the upper sub-grid.  Below x_min the
 * value is continued in ln x from the first two x knots; above Q^2_max in
 * ln Q^2 from the last two Q^2 knots; below Q^2_min by an anomalous-dimension
 * power law; corners take x first.
 *
 * Conventions
 *   - Return value: PDF_OK (0) or a negative pdf_status.  pdf_last_error()
 *     gives a message for the last failure on the calling thread.
 *   - Load inputs are host memory and are copied; the caller may free them on
 *     return.  Query inputs and outputs are device pointers owned by the caller
 *     that must stay valid until the work queued on `stream` has completed.
 *   - Query calls are asynchronous on `stream` (a hipStream_t; NULL = the
 *     default stream).  Argument errors are detected before anything is queued
 *     and nothing is written then.
 *   - Per-point domain errors (x <= 0, x > x_max, Q^2 <= 0, NaN/inf) are not
 *     API errors: those points get NaN in every requested column and add one
 *     to a device-side counter read with pdf_error_count().
 *   - Flavours are PDG ids: -6..-1, 1..6 quarks, 21 gluon; 0 is accepted as
 *     the gluon.  A valid flavour that the grid does not store evaluates to 0.
 *   - Loading/unloading must not race with queries that use the same member
 *     (single writer).  All calls use the HIP device current on the calling
 *     thread when the library initialises (device 0 by default).
 */
#ifndef PDFMI_H
#define PDFMI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PDF_OK = 0,
    PDF_ERR_ARG = -1,     /* bad argument (null pointer, negative size, ...) */
    PDF_ERR_GRID = -2,    /* malformed grid passed to a load call */
    PDF_ERR_MEMBER = -3,  /* unknown member id */
    PDF_ERR_PID = -4,     /* flavour id outside {-6..6, 21} or duplicated in a load */
    PDF_ERR_NOMEM = -5,   /* device or host allocation failed */
    PDF_ERR_DEVICE = -6,  /* HIP runtime / launch failure, or no usable GPU */
    PDF_ERR_STATE = -7    /* call not valid in the current state (e.g. no alpha_s table) */
} pdf_status;

/* hipStream_t, passed as an opaque pointer so this header needs no HIP include */
typedef void* pdf_stream_t;

/*
 * Load one member's grid (section 2.2 data: LHAPDF-style sub-grids).
 *   n_subgrids     K >= 1 sub-grids in increasing Q^2 order
 *   subgrid_shape  [K][2] = {nx, nq}, each >= 2
 *   n_pids, pids   the stored flavour columns, in column order (no duplicates)
 *   knots          for each sub-grid: nx x knots then nq Q^2 knots, all strictly
 *                  increasing; x knots in (0, 1]; every sub-grid has the same
 *                  first and last x knot; the last Q^2 knot of sub-grid k equals
 *                  the first of sub-grid k+1 (the threshold is repeated)
 *   values         for each sub-grid: x*f as [ix][iq][column] (column fastest),
 *                  finite, concatenated over sub-grids; at most 8192 knots in
 *                  total, and the device copy (each sub-grid padded to >= 4
 *                  knots per axis, columns to an even count, FP64) within 2 GiB
 *   member_out     receives the member id (>= 0)
 * Errors: PDF_ERR_ARG (null pointers), PDF_ERR_GRID (shape/knots/values),
 * PDF_ERR_PID, PDF_ERR_NOMEM, PDF_ERR_DEVICE.  Synchronous: the grid is
 * resident on the device when the call returns.
 */
int pdf_load_grid(int32_t n_subgrids, const int32_t* subgrid_shape,
                  int32_t n_pids, const int32_t* pids,
                  const double* knots, const double* values,
                  int32_t* member_out);

/* Release a member's device memory.  PDF_ERR_MEMBER if unknown. */
int pdf_unload(int32_t member);

/*
 * Load the alpha_s table (section 2.3: nodes from the set's metadata).
 * q2_knots non-decreasing, > 0; a value repeated once starts a new segment
 * (flavour threshold) and a Q^2 equal to it uses the upper segment; every
 * segment has >= 2 knots; at most 256 knots.  alphas finite.  Replaces any
 * previous table.
 */
int pdf_load_alphas(int32_t n_knots, const double* q2_knots, const double* alphas);

/*
 * x*f for n points and n_pids flavours, FP64 arithmetic (sections 2.1-2.2).
 *   member        id from pdf_load_grid
 *   pids, n_pids  HOST array of requested flavours (copied into the launch);
 *                 pids == NULL requests every stored column in load order
 *                 (n_pids is then ignored)
 *   x, q2         DEVICE arrays of n doubles (momentum fraction, Q^2 in GeV^2)
 *   out           DEVICE array of n * P doubles, point-major:
 *                 out[i * P + j] = x f_{pid j}(x[i], q2[i]), P = number of
 *                 requested flavours
 * n == 0 is a no-op.  Errors: PDF_ERR_MEMBER, PDF_ERR_PID, PDF_ERR_ARG,
 * PDF_ERR_DEVICE.
 */
int pdf_xfxq2(int32_t member, const int32_t* pids, int32_t n_pids,
              const double* x, const double* q2, int64_t n,
              double* out, pdf_stream_t stream);

/*
 * As pdf_xfxq2 with FP32 bulk arithmetic: validation, sub-grid choice, knot
 * search and the log transforms in FP64; Hermite weights, grid values (rounded
 * to FP32 at load) and the accumulation in FP32; extrapolation combined in
 * FP64 from the FP32 anchor values; FP32 output.
 */
int pdf_xfxq2_f32(int32_t member, const int32_t* pids, int32_t n_pids,
                  const double* x, const double* q2, int64_t n,
                  float* out, pdf_stream_t stream);

/*
 * alpha_s(Q^2) for n points (section 2.3): cubic Hermite in ln Q^2 inside a
 * segment, constant below the first and above the last knot; NaN (and the
 * error counter) for Q^2 <= 0 or non-finite.  q2 and out are DEVICE arrays of
 * n doubles.  PDF_ERR_STATE if no table is loaded.
 */
int pdf_alphas_q2(const double* q2, int64_t n, double* out, pdf_stream_t stream);

/*
 * Location of each point in a member's grid, as used by pdf_xfxq2: sub-grid k
 * (the largest whose first Q^2 knot is <= q2, clamped), x cell ix and Q^2 cell
 * iq (largest i <= n-2 with knot_i <= value, clamped to the grid), and region
 * bits (1 x < x_min, 2 Q^2 < Q^2_min, 4 Q^2 > Q^2_max, 8 invalid; an invalid
 * point gets k = ix = iq = -1).  All four outputs are DEVICE arrays of n.
 */
int pdf_locate(int32_t member, const double* x, const double* q2, int64_t n,
               int32_t* subgrid, int32_t* ix, int32_t* iq, int8_t* region,
               pdf_stream_t stream);

/*
 * Number of invalid query points seen since the last reset (all query entry
 * points add to it).  Synchronises `stream` first.  reset != 0 zeroes it.
 */
int pdf_error_count(int64_t* count_out, int32_t reset, pdf_stream_t stream);

/*
 * Host-only checks run by pdf_load_grid / pdf_load_alphas before any device
 * work (same arguments, same error codes); they touch no GPU state and can be
 * called on a machine without a GPU.
 */
int pdf_validate_grid(int32_t n_subgrids, const int32_t* subgrid_shape,
                      int32_t n_pids, const int32_t* pids,
                      const double* knots, const double* values);
int pdf_validate_alphas(int32_t n_knots, const double* q2_knots, const double* alphas);

/*
 * Tuning: whether pdf_xfxq2 / pdf_xfxq2_f32 stage a member's whole grid in
 * each workgroup's LDS (160 KB per CU on gfx950) when it fits.
 *   0 = automatic (stage when it fits and the call has enough points to pay
 *       for one grid copy per workgroup), 1 = never, 2 = whenever it fits.
 * A batch plan takes the policy in force when it is created: 1 reads the
 * grids from global memory, 0 and 2 stage them whenever the largest fits.
 * Results are identical under every policy.
 */
int pdf_set_lds_policy(int32_t policy);

/*
 * Launch-shape knobs (results are identical under every setting; they only
 * change speed).  Process-wide; set them before queueing work.
 *   PDF_TUNE_LDS_POLICY      as pdf_set_lds_policy (0, 1, 2)
 *   PDF_TUNE_VECTOR_COLUMNS  1: a request for every stored flavour in load
 *                            order is served by lanes that each own a
 *                            16-byte group of columns (2 FP64 / 4 FP32);
 *                            0: one lane per (point, flavour)
 *   PDF_TUNE_BLOCKS_PER_CU   workgroups launched per compute unit when the
 *                            grid is read from global memory (1..4096;
 *                            capped at one 64-point tile per wave)
 * PDF_ERR_ARG for an unknown knob or value out of range.
 */
enum { PDF_TUNE_LDS_POLICY = 0, PDF_TUNE_VECTOR_COLUMNS = 1, PDF_TUNE_BLOCKS_PER_CU = 2 };
int pdf_set_tuning(int32_t knob, int32_t value);
int pdf_get_tuning(int32_t knob, int32_t* value);

/*
 * Batched evaluation: many requests, each on its own member and flavour list
 * (the multi-member evaluation of section 4.3), served by one persistent
 * launch.  Workgroups take tiles (tile_points consecutive points of one
 * request) from a device counter, stage the tile's member grid in LDS when it
 * is not the one already staged, and evaluate it like pdf_xfxq2 (FP32 bulk
 * arithmetic like pdf_xfxq2_f32 when out_f64 == 0, FP64 otherwise).
 * Results are identical to the per-request calls for every tile size.
 */
typedef struct {
    int32_t member;        /* id from pdf_load_grid */
    int32_t n_pids;        /* requested flavours (ignored when pids == NULL) */
    const int32_t* pids;   /* HOST list; NULL = every stored flavour in load order */
    const double* x;       /* DEVICE [n] */
    const double* q2;      /* DEVICE [n] */
    int64_t n;             /* points (>= 0) */
    void* out;             /* DEVICE point-major [n][P], float (out_f64 == 0) or double */
} pdf_request;

/*
 * Build a plan (request, flavour and tile tables copied to the device).  The
 * members and the x / q2 / out buffers named by the requests must stay valid
 * for the plan's lifetime; running the plan again evaluates whatever the x
 * and q2 buffers then hold.  *plan_out receives the plan id.
 */
int pdf_batch_create(const pdf_request* reqs, int32_t n_req, int32_t out_f64, int32_t* plan_out);
/*
 * Plan settings: tile_points (multiple of 64, default 4096), vector_cols
 * (1: 16-byte column groups for requests of every stored flavour in order),
 * use_graph (1: pdf_batch_run replays a hipGraph holding the counter reset
 * and the persistent kernel, built on first use).  A change of tile_points
 * rebuilds the tile table and first waits for the device to be idle (a run
 * of the plan may still be reading the old table).
 */
int pdf_batch_configure(int32_t plan, int32_t tile_points, int32_t vector_cols, int32_t use_graph);
/* Queue one evaluation of every request of the plan on stream. */
int pdf_batch_run(int32_t plan, pdf_stream_t stream);
/*
 * Time the plan on stream for each tile size in {1024, 2048, 4096, 8192,
 * 16384} and vector_cols in {0, 1} (reps timed runs each, after one warm-up;
 * outputs are overwritten with identical values), keep the fastest, and
 * remember it for plans with the same request signature in this process.
 * Synchronises stream.  tile_out / vector_out (nullable) receive the choice.
 */
int pdf_batch_autotune(int32_t plan, int32_t reps, pdf_stream_t stream, int32_t* tile_out, int32_t* vector_out);
/*
 * Autotune choices kept on disk, for later processes with the same workload:
 * reads path (a text file of "key tile_points vector_cols" lines; a missing
 * file holds none, lines that do not parse are skipped) into the choices
 * pdf_batch_autotune remembers, and from then on appends every choice a
 * sweep makes.  Keys are the request signature (request count, point and
 * evaluation totals, output precision, grid staging) and the device
 * (architecture name, compute units), so a file can serve several GPUs and
 * workloads; a later line for a key replaces an earlier one on reading.
 * path NULL or "" stops the appending (choices already read stay).  Host
 * only: no device work.  Errors: PDF_ERR_ARG when path exists but cannot be
 * read.  A file that cannot be appended to is ignored (the choice is then
 * remembered in this process only).
 */
int pdf_batch_tune_cache(const char* path);
int pdf_batch_destroy(int32_t plan);
/* One-shot: create a plan with FP32 outputs (the FP32 bulk path of many
 * members), run it on stream, synchronise stream, destroy it.  Errors as
 * pdf_batch_create / pdf_batch_run; nothing is written when creation fails. */
int pdf_xfxq2_batched(const pdf_request* reqs, int32_t n_req, pdf_stream_t stream);
/* The same with FP64 outputs (every out pointer a double[n][n_pids]). */
int pdf_xfxq2_batched_f64(const pdf_request* reqs, int32_t n_req, pdf_stream_t stream);

/*
 * MLP surrogate of one member's PDFs (an alternative evaluator grown on top
 * of the interpolator; the interpolator remains the reference for its error).
 * A surrogate is created on one loaded member and identified by its own id
 * (sid): several surrogates may share a member; every call that needs the
 * member's grid (set_data, xfxq2) returns PDF_ERR_MEMBER once that member
 * was unloaded, even if a later load reuses its id.
 * Network (ln x, ln Q^2) normalised to [-1,1]^2 -> 64 -> 64 -> 64 -> 16,
 * tanh hidden activations.  The first layer runs in FP32; layers 2-4 on the
 * BF16 matrix cores with FP32 accumulation, every operand carried as a BF16
 * pair (value = hi + lo, products hi*hi + lo*hi + hi*lo: about 16 significant
 * bits); FP32 master weights trained with Adam.  Output c is scaled by an
 * envelope E_c(x) of the grid (a signed cubic Hermite in ln x through the
 * value of largest magnitude over Q^2 at each x knot), so the network
 * predicts xf_c / E_c.  At most 16 stored flavours and 512 x knots.  Flat
 * FP32 parameter layout: W1[64][2], b1[64], W2[64][64], b2[64], W3[64][64],
 * b3[64], W4[16][64], b4[16].
 */
int pdf_surrogate_param_count(int32_t* n_out);
/* New surrogate for a member; Glorot-uniform weights from a counter-based
 * generator seeded by seed, zero biases and Adam moments. */
int pdf_surrogate_create(int32_t member, uint64_t seed, int32_t* sid_out);
int pdf_surrogate_destroy(int32_t sid);
/* Training set: n DEVICE points (x, q2); targets are computed by the
 * library's FP64 interpolator.  Only the points inside the network's domain
 * (see pdf_surrogate_xfxq2) are kept, in order, on the device; PDF_ERR_ARG if
 * fewer than 16 remain.  Synchronises stream. */
int pdf_surrogate_set_data(int32_t sid, const double* x, const double* q2, int64_t n, pdf_stream_t stream);
/* Options of pdf_surrogate_train. */
typedef struct {
    int32_t steps;        /* Adam steps to take in this call (>= 0) */
    int32_t batch;        /* samples per step, a multiple of 16 (consecutive slices of the training set) */
    float lr;             /* learning rate at global step 0 */
    float lr_final;       /* learning rate from global step total_steps on */
    int32_t total_steps;  /* length of the cosine schedule (>= 1) */
    float* loss_out;      /* NULL, or DEVICE [steps]: each step's batch loss before its update */
    int32_t use_graph;    /* 1: the steps replay one recorded HIP graph of a training step (fewer launch
                             costs); 0: the same launches queued one by one.  Results are identical. */
} pdf_train_opts;
/* opts->steps Adam steps (beta 0.9 / 0.999, eps 1e-8); learning rate on a
 * cosine schedule from lr to lr_final over total_steps, indexed by the
 * surrogate's global step (as is the batch slice), so a run split across
 * calls (or across a save/load) is identical to one call.  Asynchronous on
 * stream; the recorded step graph is kept with the surrogate and rebuilt
 * when the batch size or the training set changes.  PDF_ERR_STATE without a
 * training set of at least one batch. */
int pdf_surrogate_train(int32_t sid, const pdf_train_opts* opts, pdf_stream_t stream);
/* One forward + backward pass on DEVICE inputs in[batch][2] (normalised) and
 * targets[batch][16]: writes the flat FP32 gradient (param_count floats) and
 * the mean-squared-error loss (1 float) to DEVICE memory.  No update. */
int pdf_surrogate_grad(int32_t sid, const float* in, const float* target, int32_t batch,
                       float* grad_out, float* loss_out, pdf_stream_t stream);
/* One Adam update of the parameters with a caller-supplied DEVICE gradient
 * (param_count floats) at learning rate lr (for losses of the caller's own);
 * advances the global step like a training step.  Asynchronous on stream. */
int pdf_surrogate_adam(int32_t sid, const float* grad, float lr, pdf_stream_t stream);
/* Read (write == 0) or replace (write != 0) the FP32 master parameters
 * (HOST array of param_count floats).  Synchronises the device. */
int pdf_surrogate_params(int32_t sid, float* host, int32_t write);
/* x*f of the requested flavours at n DEVICE points, FP32 point-major
 * [n][P] (pids, n_pids as in pdf_xfxq2: a HOST list, NULL = every stored
 * flavour in load order; a valid flavour the grid does not store gives 0).
 * Points outside the grid or in the first/last x or Q^2 cell of a sub-grid
 * (which includes the cells at flavour thresholds) are evaluated by the FP32
 * interpolator instead of the network; invalid points give NaN and count in
 * pdf_error_count.  Asynchronous on stream. */
int pdf_surrogate_xfxq2(int32_t sid, const int32_t* pids, int32_t n_pids, const double* x, const double* q2,
                        int64_t n, float* out, pdf_stream_t stream);
/* Checkpoint: parameters, Adam moments and step count, with a checksum. */
int pdf_surrogate_save(int32_t sid, const char* path);
int pdf_surrogate_load(int32_t sid, const char* path);

/*
 * Monte-Carlo luminosity chunk sum (the integrand-shaped use of section 4.1:
 * PDFs of both incoming partons at one scale, weighted by alpha_s):
 *   *sum_out = sum_i alphas[i] * sum_j xf1[i*n_pids + j] * xf2[i*n_pids + j]
 * in FP64, with a fixed summation order that depends only on n (the result
 * is bit-identical from run to run).  xf1, xf2 (point-major [n][n_pids]),
 * alphas, workspace and sum_out are DEVICE pointers; workspace holds at least
 * pdf_mc_workspace_bytes(n) bytes and is overwritten.  n == 0 writes 0.
 */
int pdf_mc_workspace_bytes(int64_t n, int64_t* bytes_out);
int pdf_mc_chunk_sum(const double* xf1, const double* xf2, int32_t n_pids,
                     const double* alphas, int64_t n, double* workspace,
                     double* sum_out, pdf_stream_t stream);
/* The same sum over FP32 PDF values (products and sums in FP64). */
int pdf_mc_chunk_sum_f32(const float* xf1, const float* xf2, int32_t n_pids,
                         const double* alphas, int64_t n, double* workspace,
                         double* sum_out, pdf_stream_t stream);

/*
 * PDFs and alpha_s at the same points in one pass (the shape of an
 * integrand, which needs both at every phase-space point; sections 2.2 and
 * 2.3): out as pdf_xfxq2 (or pdf_xfxq2_f32), alphas_out[i] = alpha_s(q2[i])
 * as pdf_alphas_q2 -- both bit-identical to the separate calls; q2 is read
 * once.  alphas_out: device [n].  Invalid points add to pdf_error_count as
 * the two separate calls would (once for x*f, once for alpha_s).  Errors as
 * pdf_xfxq2, plus PDF_ERR_ARG for a null alphas_out (n > 0) and
 * PDF_ERR_STATE when no alpha_s table is loaded.  Asynchronous on stream.
 */
int pdf_xfxq2_alphas(int32_t member, const int32_t* pids, int32_t n_pids,
                     const double* x, const double* q2, int64_t n, double* out,
                     double* alphas_out, pdf_stream_t stream);
int pdf_xfxq2_alphas_f32(int32_t member, const int32_t* pids, int32_t n_pids,
                         const double* x, const double* q2, int64_t n, float* out,
                         double* alphas_out, pdf_stream_t stream);

/*
 * LHAPDF6 data files (section 2: the set folders are loaded directly, with
 * the same layout as LHAPDF).  Host-only parsing; no device work except the
 * final pdf_load_grid / pdf_load_alphas of the load calls.
 *
 * Member file ("lhagrid1"): a header of "key: value" lines ended by "---",
 * then per sub-grid a block ended by "---": the x knots, the Q knots and the
 * flavour ids on one line each, then nx*nq lines of one value per flavour,
 * the Q index running fastest.  Q knots are squared (FP64) on reading.
 *
 * pdf_lhapdf_read(path, sizes, shape, pids, knots, values):
 *   sizes[4] receives {K, P, knot count, value count}.  With all four arrays
 *   NULL only the sizes are returned; otherwise all four must be non-NULL and
 *   hold shape[2K], pids[P], knots[knot count], values[value count], filled
 *   in pdf_load_grid's argument layout.  Errors: PDF_ERR_ARG (null pointers,
 *   unreadable file), PDF_ERR_GRID (malformed file: the message names the
 *   sub-grid and line).  Nothing is validated beyond the layout: a load call
 *   applies pdf_validate_grid.
 * pdf_load_lhapdf(path, member_out): read and pdf_load_grid in one call.
 * pdf_lhapdf_read_alphas(info_path, n_out, q2_knots, alphas): the AlphaS_Qs
 *   (squared) and AlphaS_Vals lists of a set's .info file; with both arrays
 *   NULL only *n_out is set, otherwise both must hold *n_out entries.
 * pdf_load_lhapdf_alphas(info_path): read and pdf_load_alphas in one call.
 */
int pdf_lhapdf_read(const char* path, int64_t* sizes, int32_t* shape, int32_t* pids,
                    double* knots, double* values);
int pdf_load_lhapdf(const char* path, int32_t* member_out);
int pdf_lhapdf_read_alphas(const char* info_path, int32_t* n_out, double* q2_knots,
                           double* alphas);
int pdf_load_lhapdf_alphas(const char* info_path);

/*
 * Fused Monte-Carlo chunk sum (section 4.1 integrand load, one kernel): for
 * points (x1[i], x2[i], q2[i]) of a member and the loaded alpha_s table,
 *   S = sum_i alpha_s(q2[i]) * sum_j xf(x1[i], q2[i])_j * xf(x2[i], q2[i])_j
 * over the requested flavours (pids as in pdf_xfxq2; NULL = all stored),
 * without writing the PDF values: the result is bit-identical to pdf_xfxq2
 * (x1), pdf_xfxq2 (x2), pdf_alphas_q2 and pdf_mc_chunk_sum on the same
 * inputs (same per-value arithmetic, same summation order).  The _f32 form
 * matches pdf_xfxq2_f32 + pdf_mc_chunk_sum_f32.  x1, x2, q2: device [n];
 * workspace: device, pdf_mc_workspace_bytes(n); sum_out: device double.
 * Invalid points count in the error counter as in the unfused calls.
 * Errors: PDF_ERR_ARG, PDF_ERR_MEMBER, PDF_ERR_PID, PDF_ERR_STATE (no
 * alpha_s table), PDF_ERR_GRID (location tables beyond LDS), PDF_ERR_DEVICE.
 * Asynchronous on stream.
 */
int pdf_mc_fused(int32_t member, const int32_t* pids, int32_t n_pids,
                 const double* x1, const double* x2, const double* q2, int64_t n,
                 double* workspace, double* sum_out, pdf_stream_t stream);
int pdf_mc_fused_f32(int32_t member, const int32_t* pids, int32_t n_pids,
                     const double* x1, const double* x2, const double* q2, int64_t n,
                     double* workspace, double* sum_out, pdf_stream_t stream);

/*
 * FastKernel-style contraction of PDF members (section 4.3: predictions are
 * convolutions of FK tables with PDFs on an x grid, for many members at once):
 *   out[r][d] = sum_k pdf[r][k] * fk[d][k]      (FP64, fixed summation order)
 * pdf: device [nrep][K] (member r's values flattened, e.g. [x point][flavour]
 * as pdf_xfxq2 writes them), fk: device [ndat][K] in the same k order, out:
 * device [nrep][ndat].  K = 0 gives zeros.  For long K the sum is split into
 * slices whose partial sums the library keeps in a workspace it allocates on
 * first need and reuses (grown, after synchronising the stream, when a
 * larger one is needed; freed by pdf_shutdown).  Every call uses that one
 * workspace: calls on different streams must not run concurrently (calls on
 * one stream are ordered by the stream).  Errors: PDF_ERR_ARG
 * (negative sizes, nrep > 2^22, null pointers), PDF_ERR_NOMEM,
 * PDF_ERR_DEVICE.  Asynchronous on stream.
 */
int pdf_fk_contract(const double* pdf, const double* fk, int32_t nrep, int32_t ndat, int64_t K,
                    double* out, pdf_stream_t stream);

/*
 * For callers that cannot allocate device memory (code recorded into a HIP
 * graph, serving loops, harnesses that forbid hipMalloc): pdf_fk_contract
 * with the partial sums of its K slices kept in a fixed 64 MiB device array
 * that the library holds on each GPU it runs on until the process ends,
 * instead of a workspace it allocates.  Same arguments, kernels and results
 * (bit-identical to pdf_fk_contract); no allocation, no free and no
 * synchronisation.  PDF_ERR_ARG when the partial sums (S slices x nrep x ndat
 * doubles, S chosen from the sizes and the number of compute units, at most
 * 64; S = 1 needs none) exceed 64 MiB: nothing is queued then.  Every call on
 * a GPU shares that array and leaves its partial sums there: calls that
 * overlap on one GPU (different streams or threads) race and must not be
 * issued.  Asynchronous on stream.
 */
int pdf_fk_contract_noalloc(const double* pdf, const double* fk, int32_t nrep, int32_t ndat, int64_t K,
                            double* out, pdf_stream_t stream);

/* Message of the last failure on the calling thread ("" if none). */
const char* pdf_last_error(void);

/* Release every member, the alpha_s table and library state. */
int pdf_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* PDFMI_H */
