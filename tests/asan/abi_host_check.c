/* Host-side checks of the C ABI (include/dngd.h) for an AddressSanitizer and
 * UndefinedBehaviorSanitizer build of the library's host code. Every call
 * here returns before any device work: argument validation and its error
 * messages, the default options, and the host-only footprint computation
 * over many problem descriptions and step options. Needs no GPU.
 * Prints "ok <checks>" and exits 0, or names the first failing check. */
#include <stdio.h>
#include <string.h>

#include "dngd.h"

static int n_checks = 0;

#define CHECK(cond)                                                        \
  do {                                                                     \
    ++n_checks;                                                            \
    if (!(cond)) {                                                         \
      fprintf(stderr, "check failed at line %d: %s (last error: %s)\n",   \
              __LINE__, #cond, dngd_last_error());                         \
      return 1;                                                            \
    }                                                                      \
  } while (0)

static dngd_problem_desc desc(int pde, int L, const int* widths, long n_int, long n_bdy,
                              long n_init) {
  dngd_problem_desc d;
  memset(&d, 0, sizeof(d));
  d.pde = pde;
  d.n_layers = L;
  d.widths = (const int32_t*)widths;
  d.kappa = 0.1;
  d.n_int = n_int;
  d.n_bdy = n_bdy;
  d.n_init = n_init;
  return d;
}

int main(void) {
  CHECK(dngd_version() != NULL && strlen(dngd_version()) > 0);

  dngd_step_opts o;
  memset(&o, 0x5a, sizeof(o));
  dngd_step_opts_default(&o);
  CHECK(o.precision == DNGD_MIXED && o.solver == DNGD_DENSE && o.ga == 1 && o.ir_sweeps == 2);
  CHECK(o.pcg_kvp == DNGD_F64 && o.nystrom_reuse == 0 && o.landmarks == NULL);
  dngd_step_opts_default(NULL);

  /* footprints: every solver and precision on Poisson, heat and Navier-Stokes shapes */
  const int w_p5[] = {5, 256, 256, 256, 1};
  const int w_p2[] = {2, 48, 1};
  const int w_h[] = {3, 40, 24, 1};
  const int w_ns[] = {2, 50, 50, 50, 50, 3};
  const int w_big[] = {5, 2048, 2048, 2048, 2048, 1};
  dngd_problem_desc ds[5];
  ds[0] = desc(DNGD_POISSON, 4, w_p5, 4000, 1000, 0);
  ds[1] = desc(DNGD_POISSON, 2, w_p2, 77, 31, 0);
  ds[2] = desc(DNGD_HEAT, 3, w_h, 91, 37, 29);
  ds[3] = desc(DNGD_NAVIER_STOKES, 5, w_ns, 400, 400, 0);
  ds[4] = desc(DNGD_POISSON, 5, w_big, 45000, 5000, 0);
  const int solvers[] = {DNGD_DENSE, DNGD_PCG, DNGD_PRIMAL, DNGD_DENSE_AUTO, DNGD_STRUCTURED};
  for (int i = 0; i < 5; ++i) {
    size_t prev = 0;
    for (int s = 0; s < 5; ++s)
      for (int prec = 0; prec < 2; ++prec)
        for (int kv = 0; kv < 2; ++kv) {
          dngd_step_opts_default(&o);
          o.solver = solvers[s];
          o.precision = prec;
          o.n_landmarks = 60;
          o.pcg_kvp = kv ? DNGD_BF16 : DNGD_F64;
          size_t b = 0;
          CHECK(dngd_footprint_desc(&ds[i], &o, &b) == DNGD_OK);
          CHECK(b > 0);
          if (s == 1 && kv == 1) CHECK(b > prev); /* bf16 products add their buffers */
          prev = b;
        }
    size_t b0 = 0;
    CHECK(dngd_footprint_desc(&ds[i], NULL, &b0) == DNGD_OK && b0 > 0);
  }

  /* invalid descriptions: rejected before anything touches a device */
  dngd_problem* h = NULL;
  dngd_problem_desc bad = ds[0];
  CHECK(dngd_problem_create(NULL, &h) == DNGD_EINVAL);
  CHECK(dngd_problem_create(&bad, NULL) == DNGD_EINVAL);
  bad.pde = 7;
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL && h == NULL);
  CHECK(strstr(dngd_last_error(), "pde") != NULL);
  bad = ds[0];
  bad.n_layers = 0;
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  bad = ds[0];
  bad.widths = NULL;
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  const int w_two_out[] = {5, 32, 2};
  bad = desc(DNGD_POISSON, 2, w_two_out, 10, 10, 0);
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  const int w_wide[] = {5, 5000, 1};
  bad = desc(DNGD_POISSON, 2, w_wide, 10, 10, 0);
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  bad = desc(DNGD_POISSON, 2, w_p2, 10, 10, 3);  /* initial points need the heat equation */
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  bad = desc(DNGD_POISSON, 2, w_p2, 0, 0, 0);
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  bad = ds[0]; /* valid shape, but no point arrays */
  CHECK(dngd_problem_create(&bad, &h) == DNGD_EINVAL);
  CHECK(strstr(dngd_last_error(), "null") != NULL);
  CHECK(dngd_footprint_desc(NULL, NULL, NULL) == DNGD_EINVAL);

  /* entry points taking a handle: null handles and arguments */
  double x = 0.0;
  dngd_step_stats st;
  CHECK(dngd_step(NULL, &x, 1e-3, NULL, &x, &st, NULL) == DNGD_EINVAL);
  CHECK(dngd_kvp(NULL, &x, 1e-3, &x, &x, DNGD_F64, NULL) == DNGD_EINVAL);
  CHECK(dngd_vjp(NULL, &x, &x, &x, NULL) == DNGD_EINVAL);
  CHECK(dngd_jvp(NULL, &x, &x, &x, NULL) == DNGD_EINVAL);
  CHECK(dngd_fvv(NULL, &x, &x, &x, NULL) == DNGD_EINVAL);
  CHECK(dngd_num_params(NULL) == -1 && dngd_num_residuals(NULL) == -1);
  CHECK(dngd_problem_destroy(NULL) == DNGD_OK);

  /* stateless calls: sizes, dtypes and passes checked before any allocation */
  int64_t info = 0;
  CHECK(dngd_gram(10, 10, NULL, 10, DNGD_F64, 1, 1e-3, &x, 10, NULL) == DNGD_EINVAL);
  CHECK(dngd_gram(10, 10, &x, 5, DNGD_F64, 1, 1e-3, &x, 10, NULL) == DNGD_EINVAL);
  CHECK(dngd_gram(10, 10, &x, 12, DNGD_F32, 2, 1e-3, &x, 10, NULL) == DNGD_EINVAL);
  CHECK(dngd_gram(10, 10, &x, 10, DNGD_F32, 3, 1e-3, &x, 10, NULL) == DNGD_EINVAL);
  CHECK(dngd_gram(10, 10, &x, 12, 9, 3, 1e-3, &x, 10, NULL) == DNGD_EINVAL);
  CHECK(dngd_cholesky_solve(0, &x, 1, 0, 1, &x, 1, &info, NULL) == DNGD_EINVAL);
  CHECK(dngd_cholesky_solve(4, &x, 2, 0, 1, &x, 4, &info, NULL) == DNGD_EINVAL);
  CHECK(dngd_cholesky_solve(4, &x, 4, 0, 1, NULL, 4, &info, NULL) == DNGD_EINVAL);
  CHECK(dngd_cholesky_solve_noalloc(4, NULL, 4, 0, 1, &x, 4, &info, NULL) == DNGD_EINVAL);
  CHECK(dngd_cholesky_solve_noalloc(100000, &x, 100000, 0, 1, &x, 100000, &info, NULL) ==
        DNGD_EINVAL);
  CHECK(strstr(dngd_last_error(), "scratch") != NULL);
  CHECK(dngd_nystrom_pcg(NULL, &x, 1e-3, NULL, 1, 1e-6, 10, &x, &x, NULL, NULL) == DNGD_EINVAL);
  CHECK(dngd_losses(NULL, &x, &x, 1, &x, &x, NULL) == DNGD_EINVAL);
  CHECK(dngd_iterate(NULL, &x, 1e-3, 0.0, NULL, 1, &x, NULL, NULL, NULL) == DNGD_EINVAL);

  printf("ok %d\n", n_checks);
  return 0;
}
