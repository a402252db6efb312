/*
 * Driver for the host logic of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer (built and run by
 * tests/test_abi.py::test_host_logic_under_sanitizers, against a host-only build of the library with the sanitizers
 * on its host code).  It needs no GPU: it calls the host-only entry points (level plan, workspace size, error
 * strings) over many problem shapes, flags and invalid arguments, and the argument checks of the device entry points,
 * which must return their error codes before touching any device.
 */
#include <stdio.h>
#include <string.h>

#include "../include/excmg.h"

static int failures = 0;

#define CHECK(cond, what)                                        \
  do {                                                           \
    if (!(cond)) {                                               \
      fprintf(stderr, "FAILED: %s (line %d)\n", what, __LINE__); \
      ++failures;                                                \
    }                                                            \
  } while (0)

static excmg_problem problem(int nx, int ny, int nz, int cx, int cy, int cz) {
  excmg_problem p;
  memset(&p, 0, sizeof(p));
  p.box[0] = 1.0;
  p.box[1] = 0.5;
  p.box[2] = 2.0;
  p.n[0] = nx;
  p.n[1] = ny;
  p.n[2] = nz;
  p.n_coarse[0] = cx;
  p.n_coarse[1] = cy;
  p.n_coarse[2] = cz;
  p.tol = 1e-10;
  return p;
}

int main(void) {
  /* every shape from 1 to 40 cells per axis in steps, automatic and explicit coarsest grids, both precisions */
  int ok = 0, rejected = 0;
  for (int nx = 1; nx <= 40; nx += 3)
    for (int ny = 2; ny <= 40; ny += 5)
      for (int nz = 2; nz <= 40; nz += 7)
        for (int prec = 0; prec < 2; ++prec) {
          excmg_problem p = problem(nx, ny, nz, 0, 0, 0);
          p.precision = prec;
          int32_t levels = 0, nc[3] = {0, 0, 0};
          size_t bytes = 0;
          const int e = excmg_plan(&p, &levels, nc);
          const int w = excmg_workspace_bytes(&p, &bytes);
          CHECK(e == w, "plan and workspace agree on validity");
          if (e == EXCMG_OK) {
            ++ok;
            CHECK(levels >= 1 && levels <= EXCMG_MAX_LEVELS, "level count");
            CHECK(nc[0] << (levels - 1) == nx && nc[1] << (levels - 1) == ny && nc[2] << (levels - 1) == nz,
                  "coarsest grid times 2^(levels-1) is the finest");
            CHECK(bytes > 8u * (size_t)(nx + 1) * (size_t)(ny + 1) * (size_t)(nz + 1), "workspace size");
            excmg_problem q = problem(nx, ny, nz, nc[0], nc[1], nc[2]);
            q.precision = prec;
            int32_t l2 = 0, nc2[3];
            CHECK(excmg_plan(&q, &l2, nc2) == EXCMG_OK && l2 == levels, "the automatic plan given explicitly");
          } else {
            ++rejected;
            CHECK(e == EXCMG_ERR_SHAPE || e == EXCMG_ERR_ARG, "rejection code");
          }
        }
  CHECK(ok > 0 && rejected > 0, "both accepted and rejected shapes");
  /* invalid parameters */
  excmg_problem p = problem(64, 64, 64, 0, 0, 0);
  int32_t levels;
  int32_t nc[3];
  size_t bytes;
  p.tol = -1.0;
  CHECK(excmg_plan(&p, &levels, nc) == EXCMG_ERR_ARG, "negative tolerance");
  p = problem(64, 64, 64, 0, 0, 0);
  p.flags = 1u << 20;
  CHECK(excmg_workspace_bytes(&p, &bytes) == EXCMG_ERR_ARG, "unknown flag");
  p = problem(64, 64, 64, 0, 0, 0);
  p.tol_order = 17.0;
  CHECK(excmg_workspace_bytes(&p, &bytes) == EXCMG_ERR_ARG, "tolerance order above 16");
  p = problem(64, 64, 64, 3, 3, 3);
  CHECK(excmg_plan(&p, &levels, nc) == EXCMG_ERR_SHAPE, "coarsest counts that do not divide");
  p = problem(64, 64, 64, 0, 0, 0);
  p.box[1] = 0.0;
  CHECK(excmg_plan(&p, &levels, nc) == EXCMG_ERR_ARG, "zero box edge");
  CHECK(excmg_plan(NULL, &levels, nc) == EXCMG_ERR_ARG, "null problem");
  CHECK(excmg_workspace_bytes(NULL, &bytes) == EXCMG_ERR_ARG, "null problem (workspace)");
  /* device entry points reject bad arguments before touching a device */
  excmg_handle *h = NULL;
  CHECK(excmg_setup(NULL, NULL, 0, NULL, &h) == EXCMG_ERR_ARG && h == NULL, "setup without a problem");
  p = problem(64, 64, 64, 0, 0, 0);
  CHECK(excmg_setup(&p, NULL, 0, NULL, &h) == EXCMG_ERR_WORKSPACE && h == NULL, "setup without a workspace");
  CHECK(excmg_solve(NULL, NULL, NULL, NULL, NULL, NULL) == EXCMG_ERR_ARG, "solve without a handle");
  CHECK(excmg_gradient(NULL, NULL, NULL, NULL, NULL) == EXCMG_ERR_ARG, "gradient without a handle");
  CHECK(excmg_adjoint(NULL, NULL, NULL, NULL, NULL, NULL) == EXCMG_ERR_ARG, "adjoint without a handle");
  excmg_destroy(NULL);
  for (int code = 1; code >= -10; --code) CHECK(excmg_strerror(code) != NULL, "error string");
  if (failures) {
    fprintf(stderr, "%d check(s) failed\n", failures);
    return 1;
  }
  printf("host logic under sanitizers: %d shapes accepted, %d rejected, all checks passed\n", ok, rejected);
  return 0;
}
