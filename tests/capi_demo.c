/*
 * A plain C program using libpdfmi.so through include/pdfmi.h only (no
 * Python, no torch): device memory from the HIP runtime, the null stream.
 *
 *   capi_demo <input file> <output file>
 *
 * Input (native-endian binary, written by the test): int32 K, int32 P,
 * int32 shape[2K], int32 pids[P], int64 nknots, double knots[nknots],
 * int64 nvalues, double values[nvalues], int32 nalpha, double q2a[nalpha],
 * double alpha[nalpha], int64 n, double x[n], double q2[n].
 * Output: double xf[n][P] (all stored flavours, pids = NULL), double
 * alpha_s[n], int64 invalid-point count; then, from an MLP surrogate of the
 * member trained for 5 steps on the query points, float sur[n][P] (every
 * stored flavour), float sub[n][3] (flavours 21, the last stored one, -1:
 * a subset in another order) and float loss[5] (the per-step losses).
 * Exit status 0 on success, 1 with a message on stderr for any library or
 * runtime error.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "pdfmi.h"

#define LIBCHECK(call)                                                              \
  do {                                                                              \
    int rc_ = (call);                                                               \
    if (rc_ != PDF_OK) {                                                            \
      fprintf(stderr, "%s failed: %d %s\n", #call, rc_, pdf_last_error());          \
      return 1;                                                                     \
    }                                                                               \
  } while (0)
#define HIPCHECK(call)                                                              \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));             \
      return 1;                                                                     \
    }                                                                               \
  } while (0)

static void* read_array(FILE* f, size_t count, size_t size) {
  void* p = malloc(count * size + 1);
  if (p && fread(p, size, count, f) != count) {
    free(p);
    return NULL;
  }
  return p;
}

int main(int argc, char** argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s <input> <output>\n", argv[0]);
    return 1;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) {
    fprintf(stderr, "cannot open %s\n", argv[1]);
    return 1;
  }
  int32_t K = 0, P = 0, nalpha = 0;
  int64_t nknots = 0, nvalues = 0, n = 0;
  if (fread(&K, 4, 1, f) != 1 || fread(&P, 4, 1, f) != 1 || K < 1 || K > 64 || P < 1 || P > 64) return 1;
  int32_t* shape = read_array(f, 2 * (size_t)K, 4);
  int32_t* pids = read_array(f, (size_t)P, 4);
  if (!shape || !pids || fread(&nknots, 8, 1, f) != 1 || nknots < 4) return 1;
  double* knots = read_array(f, (size_t)nknots, 8);
  if (!knots || fread(&nvalues, 8, 1, f) != 1 || nvalues < 1) return 1;
  double* values = read_array(f, (size_t)nvalues, 8);
  if (!values || fread(&nalpha, 4, 1, f) != 1 || nalpha < 2) return 1;
  double* q2a = read_array(f, (size_t)nalpha, 8);
  double* alpha = read_array(f, (size_t)nalpha, 8);
  if (!q2a || !alpha || fread(&n, 8, 1, f) != 1 || n < 1) return 1;
  double* x = read_array(f, (size_t)n, 8);
  double* q2 = read_array(f, (size_t)n, 8);
  fclose(f);
  if (!x || !q2) return 1;

  int32_t member = -1;
  LIBCHECK(pdf_load_grid(K, shape, P, pids, knots, values, &member));
  LIBCHECK(pdf_load_alphas(nalpha, q2a, alpha));

  double *dx = NULL, *dq = NULL, *dout = NULL, *da = NULL;
  HIPCHECK(hipMalloc((void**)&dx, (size_t)n * 8));
  HIPCHECK(hipMalloc((void**)&dq, (size_t)n * 8));
  HIPCHECK(hipMalloc((void**)&dout, (size_t)n * P * 8));
  HIPCHECK(hipMalloc((void**)&da, (size_t)n * 8));
  HIPCHECK(hipMemcpy(dx, x, (size_t)n * 8, hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(dq, q2, (size_t)n * 8, hipMemcpyHostToDevice));

  int64_t nerr = 0;
  LIBCHECK(pdf_error_count(&nerr, 1, NULL));
  LIBCHECK(pdf_xfxq2(member, NULL, 0, dx, dq, n, dout, NULL));
  LIBCHECK(pdf_alphas_q2(dq, n, da, NULL));
  LIBCHECK(pdf_error_count(&nerr, 1, NULL));  /* synchronises the null stream */

  double* out = malloc((size_t)n * P * 8);
  double* a = malloc((size_t)n * 8);
  if (!out || !a) return 1;
  HIPCHECK(hipMemcpy(out, dout, (size_t)n * P * 8, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(a, da, (size_t)n * 8, hipMemcpyDeviceToHost));

  /* surrogate: a few training steps through the options struct, then every
   * stored flavour and a subset */
  enum { kSteps = 5, kSub = 3 };
  int32_t sid = -1;
  const int32_t sub_pids[kSub] = {21, pids[P - 1], -1};
  float *dsur = NULL, *dsub = NULL, *dloss = NULL;
  HIPCHECK(hipMalloc((void**)&dsur, (size_t)n * P * 4));
  HIPCHECK(hipMalloc((void**)&dsub, (size_t)n * kSub * 4));
  HIPCHECK(hipMalloc((void**)&dloss, kSteps * 4));
  LIBCHECK(pdf_surrogate_create(member, 1, &sid));
  LIBCHECK(pdf_surrogate_set_data(sid, dx, dq, n, NULL));
  pdf_train_opts opts = {kSteps, 256, 3e-3f, 3e-4f, kSteps, dloss, 1};
  LIBCHECK(pdf_surrogate_train(sid, &opts, NULL));
  LIBCHECK(pdf_surrogate_xfxq2(sid, NULL, 0, dx, dq, n, dsur, NULL));
  LIBCHECK(pdf_surrogate_xfxq2(sid, sub_pids, kSub, dx, dq, n, dsub, NULL));
  HIPCHECK(hipDeviceSynchronize());
  float* sur = malloc((size_t)n * P * 4);
  float* sub = malloc((size_t)n * kSub * 4);
  float loss[kSteps];
  if (!sur || !sub) return 1;
  HIPCHECK(hipMemcpy(sur, dsur, (size_t)n * P * 4, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(sub, dsub, (size_t)n * kSub * 4, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(loss, dloss, kSteps * 4, hipMemcpyDeviceToHost));
  LIBCHECK(pdf_surrogate_destroy(sid));
  HIPCHECK(hipFree(dsur));
  HIPCHECK(hipFree(dsub));
  HIPCHECK(hipFree(dloss));
  LIBCHECK(pdf_unload(member));
  LIBCHECK(pdf_shutdown());
  HIPCHECK(hipFree(dx));
  HIPCHECK(hipFree(dq));
  HIPCHECK(hipFree(dout));
  HIPCHECK(hipFree(da));

  FILE* g = fopen(argv[2], "wb");
  if (!g) return 1;
  if (fwrite(out, 8, (size_t)n * P, g) != (size_t)n * P || fwrite(a, 8, (size_t)n, g) != (size_t)n ||
      fwrite(&nerr, 8, 1, g) != 1 || fwrite(sur, 4, (size_t)n * P, g) != (size_t)n * P ||
      fwrite(sub, 4, (size_t)n * kSub, g) != (size_t)n * kSub || fwrite(loss, 4, kSteps, g) != kSteps)
    return 1;
  fclose(g);
  printf("capi_demo: %lld points x %d flavours, %lld invalid\n", (long long)n, P, (long long)nerr);
  return 0;
}
