/*
 * A plain C caller of the CoFEM library (include/cofem.h): reads a dense problem from
 * a binary file, runs one fit on the default device through the C ABI only, and
 * writes mu, s and alpha.  Used by tests/test_gpu_c_caller.py, which compares the
 * result with the FP64 oracle.
 *
 * usage: fit_smoke IN OUT K T U TOL SEED
 *   IN:  int64 N, int64 D, float64 beta, then N*D float32 (Phi, row-major), N float32 (y)
 *   OUT: D float32 mu, D float32 s, D float32 alpha, int32 total CG steps
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cofem.h"

static int fail(const char* what) {
  fprintf(stderr, "fit_smoke: %s (%s)\n", what, cofem_last_error());
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 8) {
    fprintf(stderr, "usage: fit_smoke IN OUT K T U TOL SEED\n");
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return fail("cannot open input");
  int64_t N = 0, D = 0;
  double beta = 0.0;
  if (fread(&N, 8, 1, f) != 1 || fread(&D, 8, 1, f) != 1 || fread(&beta, 8, 1, f) != 1) return fail("short header");
  float* phi = (float*)malloc(sizeof(float) * (size_t)(N * D));
  float* y = (float*)malloc(sizeof(float) * (size_t)N);
  float* out = (float*)malloc(sizeof(float) * (size_t)(3 * D));
  if (!phi || !y || !out) return fail("host allocation");
  if (fread(phi, sizeof(float), (size_t)(N * D), f) != (size_t)(N * D) || fread(y, sizeof(float), (size_t)N, f) != (size_t)N)
    return fail("short data");
  fclose(f);

  cofem_params p = {0};
  p.N = N;
  p.D = D;
  p.beta = beta;
  p.K = atoi(argv[3]);
  p.T = atoi(argv[4]);
  p.U = atoi(argv[5]);
  p.tol = atof(argv[6]);
  p.theta_mode = COFEM_THETA_ONES;
  p.stop_mode = COFEM_STOP_JOINT;
  p.op_kind = COFEM_OP_DENSE;
  p.phi_dtype = COFEM_PHI_FP32;
  p.refine_last = 0;
  p.seed = (uint64_t)strtoull(argv[7], NULL, 10);
  p.alpha_floor = 1e-30;
  p.mstep_mode = COFEM_MSTEP_GAUSSIAN;
  if (cofem_abi_version() != COFEM_ABI_VERSION) return fail("ABI version mismatch");

  float *d_phi = NULL, *d_y = NULL, *d_out = NULL;
  if (hipMalloc((void**)&d_phi, sizeof(float) * (size_t)(N * D)) != hipSuccess ||
      hipMalloc((void**)&d_y, sizeof(float) * (size_t)N) != hipSuccess ||
      hipMalloc((void**)&d_out, sizeof(float) * (size_t)(3 * D)) != hipSuccess)
    return fail("hipMalloc");
  if (hipMemcpy(d_phi, phi, sizeof(float) * (size_t)(N * D), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(d_y, y, sizeof(float) * (size_t)N, hipMemcpyHostToDevice) != hipSuccess)
    return fail("hipMemcpy");

  cofem_ctx* c = NULL;
  if (cofem_create(&p, NULL, &c) != COFEM_OK) return fail("cofem_create");
  if (cofem_set_dictionary(c, d_phi) != COFEM_OK) return fail("cofem_set_dictionary");
  if (cofem_fit(c, d_y) != COFEM_OK) return fail("cofem_fit");
  cofem_stats st;
  if (cofem_posterior(c, d_out, d_out + D, d_out + 2 * D, &st) != COFEM_OK) return fail("cofem_posterior");
  cofem_destroy(c);
  if (hipMemcpy(out, d_out, sizeof(float) * (size_t)(3 * D), hipMemcpyDeviceToHost) != hipSuccess)
    return fail("hipMemcpy back");
  (void)hipFree(d_phi);
  (void)hipFree(d_y);
  (void)hipFree(d_out);

  f = fopen(argv[2], "wb");
  if (!f) return fail("cannot open output");
  const int32_t steps = st.total_cg_steps;
  if (fwrite(out, sizeof(float), (size_t)(3 * D), f) != (size_t)(3 * D) || fwrite(&steps, 4, 1, f) != 1)
    return fail("short write");
  fclose(f);
  free(phi);
  free(y);
  free(out);
  printf("fit_smoke: N=%lld D=%lld, %d CG steps\n", (long long)N, (long long)D, (int)steps);
  return 0;
}
