/*
 * Driver for running the CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
 * tests/test_oracle.py::test_oracle_under_sanitizers).  It calls every entry point of oracle/oracle.h on small
 * grids (cubes, unequal counts, one- and two-grid hierarchies, every initial guess and stopping-norm reading, the
 * level-dependent tolerance, the adjoint) and the argument checks, and exits non-zero on an unexpected return code or
 * a non-finite output; the sanitizers abort on any invalid access or undefined operation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/oracle.h"

static int failures = 0;

#define CHECK(cond, what)                                    \
  do {                                                       \
    if (!(cond)) {                                           \
      fprintf(stderr, "FAILED: %s (line %d)\n", what, __LINE__); \
      ++failures;                                            \
    }                                                        \
  } while (0)

static size_t nodes(int nx, int ny, int nz) { return (size_t)(nx + 1) * (size_t)(ny + 1) * (size_t)(nz + 1); }

/* u = sin(pi x) sin(2 pi y / ly) sin(pi z / lz) + exp(x + y + z) / 10 and f = its Laplacian, on the node grid */
static void field(int nx, int ny, int nz, double lx, double ly, double lz, double *u, double *f) {
  const double pi = 3.14159265358979323846;
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        const double x = i * lx / nx, y = j * ly / ny, z = k * lz / nz;
        const double ax = pi / lx, ay = 2.0 * pi / ly, az = pi / lz;
        const double s = sin(ax * x) * sin(ay * y) * sin(az * z), e = exp(x + y + z) / 10.0;
        const size_t m = ((size_t)k * (ny + 1) + j) * (nx + 1) + i;
        u[m] = s + e;
        f[m] = -(ax * ax + ay * ay + az * az) * s + 3.0 * e;
      }
}

static int finite_all(const double *a, size_t n) {
  for (size_t q = 0; q < n; ++q)
    if (!isfinite(a[q])) return 0;
  return 1;
}

static double max_err(const double *a, const double *b, size_t n) {
  double m = 0.0;
  for (size_t q = 0; q < n; ++q) m = fmax(m, fabs(a[q] - b[q]));
  return m;
}

static void cascade_case(int nx, int ny, int nz, double lx, double ly, double lz, int ncx, int ncy, int ncz,
                         int levels) {
  const size_t n = nodes(nx, ny, nz);
  double *u = malloc(n * sizeof(double)), *f = malloc(n * sizeof(double)), *uh = malloc(n * sizeof(double));
  double *ut = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double)), *relres = malloc(16 * sizeof(double));
  int *iters = malloc(16 * sizeof(int));
  field(nx, ny, nz, lx, ly, lz, u, f);
  double sec[2] = {0.0, 0.0};  /* total and CG seconds */
  int e = orc_excmg(nx, ny, nz, lx, ly, lz, ncx, ncy, ncz, f, u, 1e-10, 10000, NULL, uh, levels >= 2 ? ut : NULL,
                    levels >= 3 ? w : NULL, iters, relres, sec);
  CHECK(e == ORC_OK, "orc_excmg");
  CHECK(finite_all(uh, n), "orc_excmg output finite");
  CHECK(max_err(uh, u, n) < 1e-2, "orc_excmg error against the exact field");
  for (int guess = 0; guess < 3; ++guess)
    for (int sn = 0; sn < 2; ++sn) {
      e = orc_excmg_variant(guess, sn, nx, ny, nz, lx, ly, lz, ncx, ncy, ncz, f, u, 1e-10, sn ? 6.0 : 0.0, 10000,
                            NULL, uh, levels >= 2 ? ut : NULL, levels >= 3 ? w : NULL, iters, relres);
      CHECK(e == ORC_OK, "orc_excmg_variant");
      CHECK(finite_all(uh, n), "orc_excmg_variant output finite");
    }
  /* adjoint of the same hierarchy with G = u - (the exact field) */
  double *G = malloc(n * sizeof(double)), *dLdf = malloc(n * sizeof(double)), *dLdg = malloc(n * sizeof(double));
  double *lam = malloc(n * sizeof(double));
  for (size_t q = 0; q < n; ++q) G[q] = uh[q] - u[q] + 1e-3 * sin((double)q);
  e = orc_adjoint(nx, ny, nz, lx, ly, lz, ncx, ncy, ncz, G, 1e-10, 10000, NULL, dLdf, dLdg, lam, iters, relres);
  CHECK(e == ORC_OK, "orc_adjoint");
  CHECK(finite_all(dLdf, n) && finite_all(dLdg, n) && finite_all(lam, n), "orc_adjoint outputs finite");
  free(G);
  free(dLdf);
  free(dLdg);
  free(lam);
  free(u);
  free(f);
  free(uh);
  free(ut);
  free(w);
  free(relres);
  free(iters);
}

static void operator_case(int nx, int ny, int nz) {
  const double hx = 1.0 / nx, hy = 0.7 / ny, hz = 1.3 / nz;
  const size_t n = nodes(nx, ny, nz);
  double *u = malloc(n * sizeof(double)), *f = malloc(n * sizeof(double)), *a = malloc(n * sizeof(double));
  double *b = malloc(n * sizeof(double)), *c = malloc(n * sizeof(double)), *d = malloc(n * sizeof(double));
  field(nx, ny, nz, 1.0, 0.7, 1.3, u, f);
  CHECK(orc_apply_L(nx, ny, nz, hx, hy, hz, u, a) == ORC_OK, "orc_apply_L");
  CHECK(orc_apply_R(nx, ny, nz, hx, hy, hz, f, b) == ORC_OK, "orc_apply_R");
  CHECK(orc_apply_M(nx, ny, nz, hx, hy, hz, u, c) == ORC_OK, "orc_apply_M");
  CHECK(orc_banded_M_apply(nx, ny, nz, hx, hy, hz, u, d) == ORC_OK, "orc_banded_M_apply");
  CHECK(max_err(c, d, n) < 1e-9 * (1.0 / (hx * hx)), "banded and stencil M agree");
  CHECK(orc_rhs(nx, ny, nz, hx, hy, hz, f, u, b) == ORC_OK, "orc_rhs");
  for (size_t q = 0; q < n; ++q) a[q] = 0.0;
  int it = 0;
  double rr = 0.0;
  const int e = orc_cg(nx, ny, nz, hx, hy, hz, b, a, 1e-12, 10000, -1, &it, &rr, NULL);
  CHECK(e == ORC_OK, "orc_cg");
  CHECK(orc_direct_solve(nx, ny, nz, hx, hy, hz, b, c) == ORC_OK, "orc_direct_solve");
  CHECK(finite_all(a, n) && finite_all(c, n), "solutions finite");
  if (nx >= 4 && ny >= 4 && nz >= 4) {
    double *gx = malloc(n * sizeof(double)), *gy = malloc(n * sizeof(double)), *gz = malloc(n * sizeof(double));
    CHECK(orc_gradient(nx, ny, nz, hx, hy, hz, u, gx, gy, gz) == ORC_OK, "orc_gradient");
    CHECK(finite_all(gx, n) && finite_all(gy, n) && finite_all(gz, n), "gradient finite");
    free(gx);
    free(gy);
    free(gz);
  }
  CHECK(orc_apply_RT(nx, ny, nz, u, a) == ORC_OK, "orc_apply_RT");
  CHECK(orc_apply_LIBT(nx, ny, nz, hx, hy, hz, u, a) == ORC_OK, "orc_apply_LIBT");
  free(u);
  free(f);
  free(a);
  free(b);
  free(c);
  free(d);
}

static void transfer_case(int nx, int ny, int nz) {
  const size_t n = nodes(nx, ny, nz), n2 = nodes(nx / 2, ny / 2, nz / 2), n4 = nodes(nx / 4, ny / 4, nz / 4);
  double *u = malloc(n * sizeof(double)), *f = malloc(n * sizeof(double)), *w = malloc(n * sizeof(double));
  double *u2 = malloc(n2 * sizeof(double)), *f2 = malloc(n2 * sizeof(double));
  double *u4 = malloc(n4 * sizeof(double)), *f4 = malloc(n4 * sizeof(double));
  field(nx, ny, nz, 1.0, 1.0, 1.0, u, f);
  field(nx / 2, ny / 2, nz / 2, 1.0, 1.0, 1.0, u2, f2);
  field(nx / 4, ny / 4, nz / 4, 1.0, 1.0, 1.0, u4, f4);
  CHECK(orc_exp_finite(nx, ny, nz, u2, u4, u, w) == ORC_OK, "orc_exp_finite");
  CHECK(max_err(w, u, n) < 1e-2, "EXP_finite near the field");
  for (int kind = 0; kind < 3; ++kind) {
    CHECK(orc_initial_guess(kind, nx, ny, nz, u2, u4, u, w) == ORC_OK, "orc_initial_guess");
    CHECK(finite_all(w, n), "initial guess finite");
  }
  CHECK(orc_exp_true(nx, ny, nz, u, u2, w) == ORC_OK, "orc_exp_true");
  CHECK(finite_all(w, n), "EXP_true finite");
  free(u);
  free(f);
  free(w);
  free(u2);
  free(f2);
  free(u4);
  free(f4);
}

int main(void) {
  orc_set_threads(2);
  /* argument checks: no access through bad arguments */
  double x[8] = {0};
  CHECK(orc_apply_M(8, 8, 8, 0.1, 0.1, 0.1, NULL, x) == ORC_ERR_ARG, "null input rejected");
  CHECK(orc_excmg(12, 12, 12, 1, 1, 1, 3, 3, 3, x, x, 1e-10, 100, NULL, x, NULL, NULL, (int *)x, x, NULL) ==
            ORC_ERR_SHAPE,
        "odd coarsest grid under three grids rejected");
  CHECK(orc_excmg_variant(7, 0, 16, 16, 16, 1, 1, 1, 4, 4, 4, x, x, 1e-10, 0.0, 100, NULL, x, NULL, NULL, (int *)x,
                          x) == ORC_ERR_ARG,
        "unknown guess rejected");
  CHECK(orc_excmg_variant(0, 0, 16, 16, 16, 1, 1, 1, 4, 4, 4, x, x, 1e-10, -1.0, 100, NULL, x, NULL, NULL, (int *)x,
                          x) == ORC_ERR_ARG,
        "negative tolerance order rejected");
  operator_case(5, 4, 6);
  operator_case(8, 12, 6);
  transfer_case(32, 16, 32);
  cascade_case(16, 16, 16, 1.0, 1.0, 1.0, 4, 4, 4, 3);
  cascade_case(32, 16, 8, 1.0, 0.5, 0.25, 8, 4, 2, 3);
  cascade_case(8, 8, 8, 1.0, 1.0, 1.0, 4, 4, 4, 2);
  cascade_case(6, 10, 14, 0.6, 1.0, 1.4, 6, 10, 14, 1);
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("oracle under sanitizers: all checks passed\n");
  return 0;
}
