/*
 * Plain C user of libqkrylov through include/qk.h alone (no Python, no
 * torch): the survival probability of the Neel state of a spin-1/2 XXZ ring
 * with quasiperiodic fields (Sec. 2, Eq. (1); Sec. 4), evolved by Krylov
 * steps.  Device memory comes from the HIP runtime.  Prints one line
 * "t P(t)" per step.
 *
 * Usage: qk_demo L h phi m dt n_steps
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "qk.h"

#define HIP_OK(call)                                                   \
  do {                                                                 \
    if ((call) != hipSuccess) {                                        \
      fprintf(stderr, "%s failed\n", #call);                          \
      return 1;                                                        \
    }                                                                  \
  } while (0)

static int fail(const char* what, qk_status s) {
  fprintf(stderr, "%s failed with status %d: %s\n", what, (int)s, qk_last_error());
  return 1;
}

int main(int argc, char** argv) {
  if (argc != 7) {
    fprintf(stderr, "usage: %s L h phi m dt n_steps\n", argv[0]);
    return 2;
  }
  const int L = atoi(argv[1]), m = atoi(argv[4]), n_steps = atoi(argv[6]);
  const double h = atof(argv[2]), phi = atof(argv[3]), dt = atof(argv[5]);
  if (L < 2 || L > 32 || L % 2 != 0 || m < 1 || n_steps < 1) {
    fprintf(stderr, "need an even 2 <= L <= 32, m >= 1 and n_steps >= 1\n");
    return 2;
  }
  const double beta = 0.5 * (sqrt(5.0) - 1.0);
  double* fields = (double*)malloc(sizeof(double) * (size_t)L);
  qk_status s = qk_fields_quasiperiodic(L, h, beta, &phi, 1, fields);
  if (s != QK_OK) return fail("qk_fields_quasiperiodic", s);

  qk_basis* b = NULL;
  s = qk_basis_build(L, L / 2, NULL, &b);
  if (s != QK_OK) return fail("qk_basis_build", s);
  int64_t D = 0;
  qk_basis_dim(b, &D);
  const qk_ham_params hp = {1.0, 1.0, 1, QK_MATFREE};
  qk_ham* H = NULL;
  s = qk_ham_create(b, &hp, fields, 1, NULL, &H);
  if (s != QK_OK) return fail("qk_ham_create", s);
  qk_krylov* k = NULL;
  s = qk_krylov_create(H, m, QK_C128, 0, &k);
  if (s != QK_OK) return fail("qk_krylov_create", s);

  uint64_t neel = 0;
  for (int i = 0; i < L; i += 2) neel |= 1ull << i;
  int64_t r0 = -1;
  s = qk_basis_rank(b, &neel, 1, &r0);
  if (s != QK_OK || r0 < 0) return fail("qk_basis_rank", s);

  // psi = e_r0 (interleaved complex doubles)
  double* psi_h = (double*)calloc((size_t)D * 2, sizeof(double));
  psi_h[2 * r0] = 1.0;
  void* psi = NULL;
  double* P_d = NULL;
  HIP_OK(hipMalloc(&psi, sizeof(double) * 2 * (size_t)D));
  HIP_OK(hipMalloc((void**)&P_d, sizeof(double)));
  HIP_OK(hipMemcpy(psi, psi_h, sizeof(double) * 2 * (size_t)D, hipMemcpyHostToDevice));
  for (int n = 1; n <= n_steps; ++n) {
    s = qk_krylov_expm_step(k, psi, dt, NULL, NULL);
    if (s != QK_OK) return fail("qk_krylov_expm_step", s);
    s = qk_return_prob(b, r0, NULL, psi, QK_C128, 1, P_d, NULL);
    if (s != QK_OK) return fail("qk_return_prob", s);
    double P = 0.0;
    HIP_OK(hipMemcpy(&P, P_d, sizeof(double), hipMemcpyDeviceToHost));
    printf("%.6f %.17g\n", n * dt, P);
  }
  HIP_OK(hipFree(psi));
  HIP_OK(hipFree(P_d));
  free(psi_h);
  free(fields);
  qk_krylov_destroy(k);
  qk_ham_destroy(H);
  qk_basis_destroy(b);
  return 0;
}
