/*
 * oracle.c -- plain FP64 CPU reference for PDF and alpha_s interpolation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no source with the HIP implementation.
 *
 * What it computes (Carrazza, Cruz-Martinez, Rossi, "PDFFlow: parton
 * distribution functions on GPU"):
 *   - section 2.2 (PDF evaluation procedure): x*f(x,Q^2) by log-bicubic
 *     interpolation in (x, Q^2) on knot grids, following the LHAPDF6
 *     prescription; query points in different Q^2 sub-grids are evaluated
 *     independently, with one-sided treatment where a sub-grid edge (flavour
 *     threshold, x edge) leaves fewer than four knots;
 *   - figure 1 (EXTRAPOLATE box) and section 2.2: evaluation outside the grid;
 *   - section 2.3 (alpha_s evaluation procedure): log-cubic interpolation of
 *     alpha_s with constant extrapolation, sub-grids split at repeated knots.
 * The paper prints no formula for any of these.  The readings taken here are:
 *   - interpolate x*f as stored, in the coordinates ln x and ln Q^2;
 *   - 1D step = cubic Hermite on a cell, value and finite-difference slope at
 *     both ends; slope at an interior knot = mean of the two adjacent secant
 *     slopes, at a sub-grid end = the one adjacent secant slope;
 *   - 2D = the 1D step along x on each Q^2 row that the Q^2 step needs, then
 *     the 1D step along Q^2 on those row values (x first, then Q^2);
 *   - knot search = comparison of raw FP64 values (same order as comparing
 *     exact logarithms); a query equal to the last knot lies in the last cell;
 *   - a Q^2 equal to a threshold knot (repeated in both sub-grids) belongs to
 *     the upper sub-grid;
 *   - extrapolation: continuation in ln x below x_min, continuation in ln Q^2
 *     above Q^2_max, an anomalous-dimension power law below Q^2_min, corners
 *     by x first; constants TAU_X, TAU_Q and X_HIGH below;
 *   - invalid queries (x <= 0, x > x_max, Q^2 <= 0, non-finite) give NaN.
 *
 * The extrapolation constants (TAU_X, TAU_Q, X_HIGH) and the agreement with
 * LHAPDF are "parity unpinned" against the paper (it prints neither); the
 * test-suite pins every part against closed forms, invariants and brute force
 * instead.
 *
 * Arithmetic: FP64 throughout, libm log/exp/pow, built with
 * -O2 -ffp-contract=off and no fast-math.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define TAU_X 1e-3   /* log-linear vs linear switch of the x / high-Q^2 continuation */
#define TAU_Q 1e-5   /* positivity threshold for the low-Q^2 anomalous dimension */
#define X_HIGH 0.9   /* above this x the low-Q^2 anomalous dimension is 1 */

enum { REG_LOWX = 1, REG_LOWQ = 2, REG_HIGHQ = 4, REG_INVALID = 8 };

/* One member's grid, as flat host arrays. */
typedef struct {
    int K;               /* number of Q^2 sub-grids */
    const int32_t* shape;/* [K][2] = {nx, nq} */
    int P;               /* number of stored flavour columns */
    const int32_t* pids; /* column -> pid */
    const double** xk;   /* per sub-grid x knots */
    const double** qk;   /* per sub-grid Q^2 knots */
    const double** val;  /* per sub-grid values [ix][iq][P] */
} grid_t;

/* value + error scale (the largest magnitude any rounding in this value is
 * proportional to; carried so tests can derive a tolerance) */
typedef struct { double v, s; } vs_t;

/* ---- 1D cubic Hermite with finite-difference slopes (section 2.2) -------- */

/* Secant slope between knots j and j+1 of a 1D table (t = knot positions,
 * f = values read with stride `st`). */
static double secant(const double* t, const double* f, long st, int j)
{
    return (f[(long)(j + 1) * st] - f[(long)j * st]) / log(t[j + 1] / t[j]);
}

/* Finite-difference slope d f / d ln t at knot j of an n-knot table. */
static double fd_slope(const double* t, const double* f, long st, int n, int j)
{
    if (j == 0) return secant(t, f, st, 0);
    if (j == n - 1) return secant(t, f, st, n - 2);
    return 0.5 * (secant(t, f, st, j - 1) + secant(t, f, st, j));
}

/* Cubic Hermite on cell i (knots i, i+1) at parameter u in [0,1]:
 * h00 f_i + h10 D d_i + h01 f_{i+1} + h11 D d_{i+1}, D = ln(t_{i+1}/t_i),
 * with the basis h00 = 2u^3 - 3u^2 + 1, h10 = u^3 - 2u^2 + u,
 * h01 = -2u^3 + 3u^2, h11 = u^3 - u^2 evaluated in factored form (v = 1 - u
 * is exact, so each keeps its relative precision at both ends of the cell). */
static double hermite_cell(const double* t, const double* f, long st, int n, int i, double u)
{
    double D = log(t[i + 1] / t[i]);
    double v = 1.0 - u, u2 = u * u, v2 = v * v;
    double h00 = v2 * (1 + 2 * u);
    double h10 = u * v2;
    double h01 = u2 * (3 - 2 * u);
    double h11 = -u2 * v;
    return h00 * f[(long)i * st] + h10 * D * fd_slope(t, f, st, n, i)
         + h01 * f[(long)(i + 1) * st] + h11 * D * fd_slope(t, f, st, n, i + 1);
}

/* Cell search: largest i in [0, n-2] with t[i] <= v (raw FP64 comparisons);
 * 0 if v < t[0]. */
static int find_cell(const double* t, int n, double v)
{
    int i = 0;
    for (int j = 0; j <= n - 2; ++j)
        if (t[j] <= v) i = j;
    return i;
}

/* Hermite parameter: ln(v / t_i) / ln(t_{i+1} / t_i). */
static double cell_param(const double* t, int i, double v)
{
    return log(v / t[i]) / log(t[i + 1] / t[i]);
}

/* Sub-grid holding Q^2 = q2: the largest k whose first knot is <= q2,
 * clamped to [0, K-1] (a repeated threshold knot goes to the upper grid). */
static int find_subgrid(const grid_t* g, double q2)
{
    int k = 0;
    for (int j = 0; j < g->K; ++j)
        if (g->qk[j][0] <= q2) k = j;
    return k;
}

/* ---- 2D log-bicubic inside sub-grid k (section 2.2) ----------------------- */

/* x*f for column c at (x, q2) inside sub-grid k: the x step on each Q^2 row
 * the Q^2 step needs (rows iq-1..iq+2 that exist), then the Q^2 step on those
 * row values with the same slope rule, one-sided at the sub-grid edges. */
static vs_t interp_k(const grid_t* g, int k, int c, double x, double q2)
{
    int nx = g->shape[2 * k], nq = g->shape[2 * k + 1], P = g->P;
    const double* xk = g->xk[k];
    const double* qk = g->qk[k];
    const double* V = g->val[k];
    int ix = find_cell(xk, nx, x), iq = find_cell(qk, nq, q2);
    double ux = cell_param(xk, ix, x), uq = cell_param(qk, iq, q2);

    int r0 = iq - 1 < 0 ? 0 : iq - 1;
    int r1 = iq + 2 > nq - 1 ? nq - 1 : iq + 2;
    double G[512];          /* x-step value on each needed Q^2 row, by row */
    double M = 0.0;
    for (int r = r0; r <= r1; ++r) {
        /* column c of row r seen as a 1D table over x: stride nq*P */
        const double* fr = V + (long)r * P + c;
        G[r] = hermite_cell(xk, fr, (long)nq * P, nx, ix, ux);
        int a0 = ix - 1 < 0 ? 0 : ix - 1, a1 = ix + 2 > nx - 1 ? nx - 1 : ix + 2;
        for (int a = a0; a <= a1; ++a) {
            double m = fabs(fr[(long)a * nq * P]);
            if (m > M) M = m;
        }
    }
    /* Q^2 step on the row values; it reads only rows iq-1..iq+2 */
    vs_t out = { hermite_cell(qk, G, 1, nq, iq, uq), M };
    return out;
}

/* ---- extrapolation (figure 1 EXTRAPOLATE; section 2.2) -------------------- */

/* Error scale of v = f0^e0 f1^e1 (log-linear) or e0 f0 + e1 f1 (linear),
 * propagated from the anchors' own scales. */
static double cont_scale(vs_t f0, vs_t f1, double v, double e0, double e1, int loglin)
{
    if (loglin) return fabs(v) * (fabs(e0) * f0.s / f0.v + fabs(e1) * f1.s / f1.v);
    return fabs(e0) * f0.s + fabs(e1) * f1.s;
}

/* x below x_min at a Q^2 inside sub-grid k: continuation in ln x from the
 * first two x knots, s = ln(x/x_0) / ln(x_1/x_0):
 * log-linear f0 (f1/f0)^s when both anchors exceed TAU_X, else linear
 * f0 + s (f1 - f0). */
static vs_t extrap_lowx(const grid_t* g, int k, int c, double x, double q2)
{
    const double* xk = g->xk[k];
    vs_t f0 = interp_k(g, k, c, xk[0], q2);
    vs_t f1 = interp_k(g, k, c, xk[1], q2);
    double s = log(x / xk[0]) / log(xk[1] / xk[0]);
    int loglin = f0.v > TAU_X && f1.v > TAU_X;
    vs_t r;
    r.v = loglin ? f0.v * pow(f1.v / f0.v, s) : f0.v + s * (f1.v - f0.v);
    r.s = cont_scale(f0, f1, r.v, 1.0 - s, s, loglin);
    return r;
}

/* value at x (in range or below x_min) on Q^2 knot row r of sub-grid k */
static vs_t at_qrow(const grid_t* g, int k, int c, double x, int r)
{
    double qr = g->qk[k][r];
    if (x < g->xk[k][0]) return extrap_lowx(g, k, c, x, qr);
    return interp_k(g, k, c, x, qr);
}

/* Q^2 above the last knot: continuation in ln Q^2 from the last two knots of
 * the last sub-grid, anchored at the last knot, s = ln(q2/q_{n-1}) /
 * ln(q_{n-1}/q_{n-2}): log-linear f1 (f1/f0)^s when both anchors exceed
 * TAU_X, else linear f1 + s (f1 - f0). */
static vs_t extrap_highq(const grid_t* g, int c, double x, double q2)
{
    int k = g->K - 1, nq = g->shape[2 * k + 1];
    const double* qk = g->qk[k];
    vs_t f0 = at_qrow(g, k, c, x, nq - 2);
    vs_t f1 = at_qrow(g, k, c, x, nq - 1);
    double s = log(q2 / qk[nq - 1]) / log(qk[nq - 1] / qk[nq - 2]);
    int loglin = f0.v > TAU_X && f1.v > TAU_X;
    vs_t r;
    r.v = loglin ? f1.v * pow(f1.v / f0.v, s) : f1.v + s * (f1.v - f0.v);
    r.s = cont_scale(f0, f1, r.v, -s, 1.0 + s, loglin);
    return r;
}

/* Q^2 below the first knot: anomalous-dimension power law
 * v = f0 * r^(gamma r + 1 - r), r = q2/q_0, gamma = d ln f / d ln Q^2 from the
 * first two knots (1 if either value <= TAU_Q, or x > X_HIGH).  Continuous at
 * q_0 with log-slope gamma there, and vanishing as Q^2 -> 0. */
static vs_t extrap_lowq(const grid_t* g, int c, double x, double q2)
{
    const double* qk = g->qk[0];
    vs_t f0 = at_qrow(g, 0, c, x, 0);
    vs_t f1 = at_qrow(g, 0, c, x, 1);
    double r = q2 / qk[0];
    double L01 = log(qk[1] / qk[0]);
    int use_gamma = (f0.v > TAU_Q && f1.v > TAU_Q && x <= X_HIGH);
    vs_t out;
    if (use_gamma) {
        double gamma = log(f1.v / f0.v) / L01;
        out.v = f0.v * pow(r, gamma * r + 1.0 - r);
        /* ln v = (1 - b) ln f0 + b ln f1 + (1-r) ln r,  b = r ln r / L01 */
        double b = r * log(r) / L01;
        out.s = fabs(out.v) * (fabs(1.0 - b) * f0.s / f0.v + fabs(b) * f1.s / f1.v);
    } else {
        out.v = f0.v * r;
        out.s = f0.s * r;
    }
    return out;
}

/* ---- one query ------------------------------------------------------------ */

static int region_of(const grid_t* g, double x, double q2)
{
    double xmax = g->xk[0][g->shape[0] - 1];
    if (!isfinite(x) || !isfinite(q2) || !(x > 0.0) || !(q2 > 0.0) || x > xmax) return REG_INVALID;
    int kl = g->K - 1, nql = g->shape[2 * kl + 1];
    int reg = 0;
    if (x < g->xk[0][0]) reg |= REG_LOWX;
    if (q2 < g->qk[0][0]) reg |= REG_LOWQ;
    if (q2 > g->qk[kl][nql - 1]) reg |= REG_HIGHQ;
    return reg;
}

static vs_t eval_one(const grid_t* g, int c, double x, double q2, int reg)
{
    if (reg & REG_LOWQ) return extrap_lowq(g, c, x, q2);
    if (reg & REG_HIGHQ) return extrap_highq(g, c, x, q2);
    int k = find_subgrid(g, q2);
    if (reg & REG_LOWX) return extrap_lowx(g, k, c, x, q2);
    return interp_k(g, k, c, x, q2);
}

static int pid_known(int pid)
{
    return (pid >= -6 && pid <= 6) || pid == 21;
}

/* column of a requested pid, -1 if a known pid absent from the grid,
 * -2 if not a valid pid; pid 0 is the gluon (21). */
static int column_of(const grid_t* g, int pid)
{
    if (pid == 0) pid = 21;
    for (int c = 0; c < g->P; ++c)
        if (g->pids[c] == pid || (g->pids[c] == 0 && pid == 21)) return c;
    return pid_known(pid) ? -1 : -2;
}

static int build_grid(grid_t* g, int32_t K, const int32_t* shape, int32_t P,
                      const int32_t* pids, const double* knots, const double* values)
{
    if (K < 1 || K > 64 || P < 1) return -1;
    g->K = K; g->shape = shape; g->P = P; g->pids = pids;
    g->xk = malloc(sizeof(double*) * K);
    g->qk = malloc(sizeof(double*) * K);
    g->val = malloc(sizeof(double*) * K);
    long ko = 0, vo = 0;
    for (int k = 0; k < K; ++k) {
        int nx = shape[2 * k], nq = shape[2 * k + 1];
        if (nx < 2 || nq < 2 || nq > 500) return -1;
        g->xk[k] = knots + ko; ko += nx;
        g->qk[k] = knots + ko; ko += nq;
        g->val[k] = values + vo; vo += (long)nx * nq * P;
    }
    return 0;
}

static void free_grid(grid_t* g)
{
    free(g->xk); free(g->qk); free(g->val);
}

/*
 * x*f for n queries and nreq requested pids.  Output point-major:
 * out[i*nreq + j].  scale (nullable) receives the error scale of each value:
 * the largest stencil magnitude for an interpolated value, propagated through
 * the extrapolation formula otherwise.  Returns 0, or -1 for a malformed
 * grid, -4 for an invalid pid (nothing written).
 */
int oracle_xfxq2(int32_t K, const int32_t* shape, int32_t P, const int32_t* pids,
                 const double* knots, const double* values,
                 int32_t nreq, const int32_t* req_pids,
                 const double* x, const double* q2, int64_t n,
                 double* out, double* scale, int32_t n_threads)
{
    grid_t g;
    if (build_grid(&g, K, shape, P, pids, knots, values) != 0) { free_grid(&g); return -1; }
    int* col = malloc(sizeof(int) * (nreq > 0 ? nreq : 1));
    for (int j = 0; j < nreq; ++j) {
        col[j] = column_of(&g, req_pids[j]);
        if (col[j] == -2) { free(col); free_grid(&g); return -4; }
    }
    if (n_threads < 1) n_threads = 1;
    #pragma omp parallel for schedule(static) num_threads(n_threads)
    for (int64_t i = 0; i < n; ++i) {
        int reg = region_of(&g, x[i], q2[i]);
        for (int j = 0; j < nreq; ++j) {
            vs_t r;
            if (reg & REG_INVALID) { r.v = NAN; r.s = 0.0; }
            else if (col[j] < 0) { r.v = 0.0; r.s = 0.0; }
            else r = eval_one(&g, col[j], x[i], q2[i], reg);
            out[i * nreq + j] = r.v;
            if (scale) scale[i * nreq + j] = r.s;
        }
    }
    free(col);
    free_grid(&g);
    return 0;
}

/*
 * Location of each query: sub-grid k, x cell ix, Q^2 cell iq (each search
 * clamped to the grid) and region bits (1 low x, 2 low Q^2, 4 high Q^2,
 * 8 invalid; invalid points get k = ix = iq = -1).
 */
int oracle_locate(int32_t K, const int32_t* shape, const double* knots,
                  const double* x, const double* q2, int64_t n,
                  int32_t* k_out, int32_t* ix_out, int32_t* iq_out, int8_t* region)
{
    int32_t pid0 = 21;
    double dummy = 0.0;
    grid_t g;
    /* values are not read here; point them at a dummy */
    if (build_grid(&g, K, shape, 1, &pid0, knots, &dummy) != 0) { free_grid(&g); return -1; }
    for (int64_t i = 0; i < n; ++i) {
        int reg = region_of(&g, x[i], q2[i]);
        region[i] = (int8_t)reg;
        if (reg & REG_INVALID) { k_out[i] = ix_out[i] = iq_out[i] = -1; continue; }
        int k = find_subgrid(&g, q2[i]);
        k_out[i] = k;
        ix_out[i] = find_cell(g.xk[k], shape[2 * k], x[i]);
        iq_out[i] = find_cell(g.qk[k], shape[2 * k + 1], q2[i]);
    }
    free_grid(&g);
    return 0;
}

/*
 * alpha_s(Q^2) (section 2.3): knots q2k[0..nk) non-decreasing, a repeated
 * value starts a new segment (flavour threshold); a Q^2 equal to it belongs to
 * the upper segment.  Inside a segment: cubic Hermite in ln Q^2 with the
 * finite-difference slopes above, one-sided at segment ends.  Outside the
 * knots: constant (first / last value).  Invalid Q^2 (<= 0, non-finite): NaN.
 */
int oracle_alphas_q2(int32_t nk, const double* q2k, const double* a,
                     const double* q2, int64_t n, double* out)
{
    if (nk < 2) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double v = q2[i];
        if (!isfinite(v) || !(v > 0.0)) { out[i] = NAN; continue; }
        if (v < q2k[0]) { out[i] = a[0]; continue; }
        if (v > q2k[nk - 1]) { out[i] = a[nk - 1]; continue; }
        /* segment: [s0, s1] index range, split where q2k repeats */
        int s0 = 0;
        for (int j = 1; j < nk; ++j)
            if (q2k[j] == q2k[j - 1] && q2k[j] <= v) s0 = j;
        int s1 = s0;
        while (s1 + 1 < nk && q2k[s1 + 1] != q2k[s1]) ++s1;
        int m = s1 - s0 + 1;
        if (m < 2) { out[i] = a[s0]; continue; }
        int c = find_cell(q2k + s0, m, v);
        double u = cell_param(q2k + s0, c, v);
        out[i] = hermite_cell(q2k + s0, a + s0, 1, m, c, u);
    }
    return 0;
}
