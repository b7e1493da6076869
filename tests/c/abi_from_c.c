/* The C ABI driven from C alone (no Python): a 24 x 20 x 18 D3Q27 FP64 lattice
 * with a uniform force, stepped through cmlbm_run and through the in-place
 * calls from the same initial state.  Checks:
 *   - total mass is conserved and total momentum grows by N F per step
 *     (Eqs. densitycalculation, velocitycalculation: the collision conserves
 *     mass and momentum, the source adds F at every node);
 *   - the in-place run ends in the same FP64 totals as the two-buffer run,
 *     and neither final buffer holds a non-finite population;
 *   - argument errors (aliasing, counts, rates, misaligned pointers) come back
 *     as CMLBM_EINVAL with a message, before any launch.
 * Prints "abi_from_c ok" and exits 0 on success. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "cmlbm.h"

#define CHECK(cond, ...)                                \
  do {                                                  \
    if (!(cond)) {                                      \
      fprintf(stderr, "abi_from_c: " __VA_ARGS__);      \
      fprintf(stderr, "\n");                            \
      exit(1);                                          \
    }                                                   \
  } while (0)

static void ok(cmlbm_sim *s, cmlbm_status st, const char *what) {
  CHECK(st == CMLBM_OK, "%s failed: %d (%s)", what, (int)st, cmlbm_last_error(s));
}

int main(void) {
  const int nx = 24, ny = 20, nz = 18, q = 27, steps = 10;
  const size_t N = (size_t)nx * ny * nz;
  const double F[3] = {1e-5, -2e-6, 3e-6};
  double *rho_h = (double *)malloc(N * sizeof(double));
  double *u_h = (double *)malloc(3 * N * sizeof(double));
  CHECK(rho_h && u_h, "host allocation");
  srand(7);
  for (size_t i = 0; i < N; ++i) {
    rho_h[i] = 1.0 + 0.01 * ((double)rand() / RAND_MAX - 0.5);
    for (int c = 0; c < 3; ++c) u_h[c * N + i] = 0.05 * ((double)rand() / RAND_MAX - 0.5);
  }
  void *rho, *u, *fa, *fb, *fpre, *fin;
  CHECK(hipMalloc(&rho, N * sizeof(double)) == hipSuccess, "hipMalloc");
  CHECK(hipMalloc(&u, 3 * N * sizeof(double)) == hipSuccess, "hipMalloc");
  CHECK(hipMalloc(&fa, q * N * sizeof(double)) == hipSuccess, "hipMalloc");
  CHECK(hipMalloc(&fb, q * N * sizeof(double)) == hipSuccess, "hipMalloc");
  CHECK(hipMalloc(&fpre, q * N * sizeof(double)) == hipSuccess, "hipMalloc");
  CHECK(hipMalloc(&fin, q * N * sizeof(double)) == hipSuccess, "hipMalloc");
  CHECK(hipMemcpy(rho, rho_h, N * sizeof(double), hipMemcpyHostToDevice) == hipSuccess, "copy");
  CHECK(hipMemcpy(u, u_h, 3 * N * sizeof(double), hipMemcpyHostToDevice) == hipSuccess, "copy");

  cmlbm_sim *s = NULL;
  CHECK(cmlbm_create(q, nx, ny, nz, CMLBM_F64, &s) == CMLBM_OK, "create: %s", cmlbm_last_error(NULL));
  double omega[23];
  for (int b = 0; b < 23; ++b) omega[b] = b < 5 ? 1.7 : 1.1;
  ok(s, cmlbm_set_rates(s, omega, 23), "set_rates");
  ok(s, cmlbm_set_force_uniform(s, F[0], F[1], F[2]), "set_force_uniform");

  /* two buffers */
  double t0[4], t1[4];
  ok(s, cmlbm_init_equilibrium(s, rho, u, fpre, fa, NULL), "init_equilibrium");
  ok(s, cmlbm_totals(s, fa, t0, NULL), "totals");
  int in_b = 0;
  ok(s, cmlbm_run(s, fa, fb, steps, NULL, &in_b), "run");
  ok(s, cmlbm_totals(s, in_b ? fb : fa, t1, NULL), "totals");
  CHECK(fabs(t1[0] - t0[0]) <= 1e-11 * t0[0], "mass drift %.3e", t1[0] - t0[0]);
  for (int c = 0; c < 3; ++c) {
    const double want = t0[1 + c] + (double)steps * (double)N * F[c];
    CHECK(fabs(t1[1 + c] - want) <= 1e-10 * (fabs(want) + (double)N * 1e-5), "momentum %d: %.12e vs %.12e", c,
          t1[1 + c], want);
  }

  /* in place, from the same initial state */
  double t2[4];
  ok(s, cmlbm_init_equilibrium_inplace(s, rho, u, fin, NULL), "init_equilibrium_inplace");
  ok(s, cmlbm_run_inplace(s, fin, steps, NULL), "run_inplace");
  ok(s, cmlbm_totals_pre(s, fin, t2, NULL), "totals_pre");
  for (int c = 0; c < 4; ++c) CHECK(t2[c] == t1[c], "in-place total %d: %.17g vs %.17g", c, t2[c], t1[c]);
  int64_t nonfinite = -1;
  ok(s, cmlbm_check_finite(s, in_b ? fb : fa, &nonfinite, NULL), "check_finite");
  CHECK(nonfinite == 0, "%lld non-finite populations after the two-buffer run", (long long)nonfinite);
  ok(s, cmlbm_check_finite(s, fin, &nonfinite, NULL), "check_finite");
  CHECK(nonfinite == 0, "%lld non-finite populations after the in-place run", (long long)nonfinite);

  /* errors */
  CHECK(cmlbm_step(s, fa, fa, NULL) == CMLBM_EINVAL, "aliased step accepted");
  CHECK(cmlbm_last_error(s)[0] != '\0', "no message for the aliased step");
  CHECK(cmlbm_run_inplace(s, fin, 3, NULL) == CMLBM_EINVAL, "odd in-place run accepted");
  /* an FP64 buffer at a 4-byte offset: refused before any launch */
  CHECK(cmlbm_step(s, fa, (char *)fb + 4, NULL) == CMLBM_EINVAL, "misaligned buffer accepted");
  CHECK(cmlbm_macroscopic(s, fa, (char *)rho + 4, u, NULL) == CMLBM_EINVAL, "misaligned field accepted");
  CHECK(cmlbm_set_rates(s, omega, 22) == CMLBM_EINVAL, "wrong rate count accepted");
  omega[0] = 2.0;
  CHECK(cmlbm_set_rates(s, omega, 23) == CMLBM_EINVAL, "rate 2 accepted");
  cmlbm_sim *bad = NULL;
  CHECK(cmlbm_create(21, nx, ny, nz, CMLBM_F64, &bad) == CMLBM_EINVAL && bad == NULL, "q = 21 accepted");

  cmlbm_destroy(s);
  cmlbm_destroy(NULL);
  hipFree(rho);
  hipFree(u);
  hipFree(fa);
  hipFree(fb);
  hipFree(fpre);
  hipFree(fin);
  free(rho_h);
  free(u_h);
  printf("abi_from_c ok (mass %.15g, momentum %.6e %.6e %.6e after %d steps)\n", t1[0], t1[1], t1[2], t1[3], steps);
  return 0;
}
