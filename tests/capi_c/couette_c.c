/*
 * A plain C user of libhrlb (test program): one Couette instance set up and advanced through
 * the C ABI of include/hrlb.h alone -- device buffers from hipMalloc, one HIP stream of its
 * own, no Python and no torch -- and its moment table printed for comparison with the oracle.
 *
 *   couette_c Qx Qy Qz S scheme kn u_w pr omega A dt steps
 *
 * Prints "residual R" and then S lines of the 14 moments of hrlb_moments (n, u_x, u_y, u_z,
 * T, P_xx, P_yy, P_zz, P_xy, P_xz, P_yz, q_x, q_y, q_z), all with 17 significant digits.
 * The start is the library's equilibrium at rest; the power viscosity law.
 */
#include <hip/hip_runtime_api.h>
#include <stdio.h>
#include <stdlib.h>

#include "hrlb.h"

#define CHECK(call)                                                                \
  do {                                                                             \
    int rc_ = (call);                                                              \
    if (rc_ != HRLB_OK) {                                                          \
      fprintf(stderr, "%s failed (%d): %s\n", #call, rc_, hrlb_last_error());     \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

#define HCHECK(call)                                                               \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess) {                                                        \
      fprintf(stderr, "%s failed: %s\n", #call, hipGetErrorString(e_));            \
      return 1;                                                                    \
    }                                                                              \
  } while (0)

int main(int argc, char** argv) {
  if (argc != 13) {
    fprintf(stderr, "usage: %s Qx Qy Qz S scheme kn u_w pr omega A dt steps\n", argv[0]);
    return 2;
  }
  const int Qx = atoi(argv[1]), Qy = atoi(argv[2]), Qz = atoi(argv[3]), S = atoi(argv[4]);
  const int scheme = atoi(argv[5]), steps = atoi(argv[12]);
  hrlb_params p;
  p.kn = atof(argv[6]);
  p.u_w = atof(argv[7]);
  p.T_w = 1.0;
  p.n0 = 1.0;
  p.pr = atof(argv[8]);
  p.omega = atof(argv[9]);
  p.suth_S = 0.0;
  p.A = atof(argv[10]);
  p.dt = atof(argv[11]);
  p.law = HRLB_LAW_POWER;
  p.collisionless = 0;

  /* the library's default expansion orders: N_x = min(6, Qx - 1), N_y = Qy - 1, N_z = Qz - 1 */
  hrlb_quad* q = NULL;
  CHECK(hrlb_init_quadrature(Qx, Qx - 1 < 6 ? Qx - 1 : 6, Qy, Qy - 1, Qz, Qz - 1, &q));
  size_t state_bytes = 0, work_bytes = 0;
  CHECK(hrlb_state_bytes(q, S, 1, &state_bytes, &work_bytes));
  void *d_state = NULL, *d_work = NULL;
  double* d_mom = NULL;
  HCHECK(hipMalloc(&d_state, state_bytes));
  HCHECK(hipMalloc(&d_work, work_bytes));
  HCHECK(hipMalloc((void**)&d_mom, (size_t)S * 14 * sizeof(double)));
  hipStream_t stream;
  HCHECK(hipStreamCreate(&stream));

  hrlb_sim* sim = NULL;
  CHECK(hrlb_init_state(q, S, scheme, &p, 1, d_state, state_bytes, d_work, work_bytes, (void*)stream, NULL, 0.0,
                        &sim));
  CHECK(hrlb_step(sim, steps));
  double R = 0.0;
  CHECK(hrlb_residual(sim, &R));
  CHECK(hrlb_moments(sim, d_mom));
  double* mom = (double*)malloc((size_t)S * 14 * sizeof(double));
  if (!mom) return 1;
  HCHECK(hipMemcpyAsync(mom, d_mom, (size_t)S * 14 * sizeof(double), hipMemcpyDeviceToHost, stream));
  HCHECK(hipStreamSynchronize(stream));

  printf("residual %.17g\n", R);
  for (int s = 0; s < S; ++s) {
    for (int k = 0; k < 14; ++k) printf(k ? " %.17g" : "%.17g", mom[s * 14 + k]);
    printf("\n");
  }

  free(mom);
  hrlb_sim_free(sim);
  hrlb_quad_free(q);
  HCHECK(hipStreamDestroy(stream));
  HCHECK(hipFree(d_mom));
  HCHECK(hipFree(d_work));
  HCHECK(hipFree(d_state));
  return 0;
}
