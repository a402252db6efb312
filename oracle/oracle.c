/*
 * Plain FP64 CPU oracle for EXCMG + 19-point compact scheme (arXiv 1507.05063).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test suite, the smoke check and the benchmark's CPU-baseline leg, never by
 * the GPU library.  Every routine is written for checking by eye against the paper: no blocking, no fusion, no
 * reordering beyond splitting the plane loop over OpenMP threads (each dot product is summed plane by plane, in
 * plane order, so results do not depend on the thread count).
 *
 * Pinning (what checks this oracle against something other than itself) is listed in the oracle's test file; every
 * function here has at least one pin there.
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------------------------------------------ */
/* grid helpers                                                                                                 */
/* ------------------------------------------------------------------------------------------------------------ */

typedef struct {
  int nx, ny, nz;
} dims_t;

static size_t node_count(int nx, int ny, int nz) { return (size_t)(nx + 1) * (size_t)(ny + 1) * (size_t)(nz + 1); }

#define NID(i, j, k) ((((size_t)(k)) * (size_t)(ny + 1) + (size_t)(j)) * (size_t)(nx + 1) + (size_t)(i))

static int is_bnd(int nx, int ny, int nz, int i, int j, int k) {
  return i == 0 || j == 0 || k == 0 || i == nx || j == ny || k == nz;
}

static double now_s(void) {
  struct timespec ts;
  clock_gettime(CLOCK_MONOTONIC, &ts);
  return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

static int g_progress = 0;

/* progress lines on stderr after each grid of a cascade (for long full-size runs) */
void orc_set_progress(int on) { g_progress = on; }

void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static int bad_grid(int nx, int ny, int nz) { return nx < 2 || ny < 2 || nz < 2; }

/* sum over interior nodes of x*y, summed per plane then over planes in order */
static double dot_interior(int nx, int ny, int nz, const double *x, const double *y) {
  double *part = (double *)calloc((size_t)nz + 1, sizeof(double));
  if (!part) return NAN;
#pragma omp parallel for schedule(static)
  for (int k = 1; k < nz; ++k) {
    double s = 0.0;
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) s += x[NID(i, j, k)] * y[NID(i, j, k)];
    part[k] = s;
  }
  double s = 0.0;
  for (int k = 1; k < nz; ++k) s += part[k];
  free(part);
  return s;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* the compact scheme, eq. (compact)                                                                            */
/* ------------------------------------------------------------------------------------------------------------ */

int orc_apply_L(int nx, int ny, int nz, double hx, double hy, double hz, const double *u, double *out) {
  if (bad_grid(nx, ny, nz) || !u || !out) return ORC_ERR_ARG;
  const double a = 1.0 / (hx * hx), b = 1.0 / (hy * hy), c = 1.0 / (hz * hz);
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        if (is_bnd(nx, ny, nz, i, j, k)) {
          out[NID(i, j, k)] = 0.0;
          continue;
        }
#define U(di, dj, dk) u[NID(i + (di), j + (dj), k + (dk))]
        double v = -8.0 * (a + b + c) * U(0, 0, 0);
        v += (4.0 * a - b - c) * (U(1, 0, 0) + U(-1, 0, 0));
        v += (4.0 * b - a - c) * (U(0, 1, 0) + U(0, -1, 0));
        v += (4.0 * c - a - b) * (U(0, 0, 1) + U(0, 0, -1));
        v += 0.5 * (a + b) * (U(1, 1, 0) + U(1, -1, 0) + U(-1, 1, 0) + U(-1, -1, 0));
        v += 0.5 * (a + c) * (U(1, 0, 1) + U(1, 0, -1) + U(-1, 0, 1) + U(-1, 0, -1));
        v += 0.5 * (b + c) * (U(0, 1, 1) + U(0, -1, 1) + U(0, 1, -1) + U(0, -1, -1));
#undef U
        out[NID(i, j, k)] = v;
      }
  return ORC_OK;
}

int orc_apply_R(int nx, int ny, int nz, double hx, double hy, double hz, const double *f, double *out) {
  (void)hx; (void)hy; (void)hz;
  if (bad_grid(nx, ny, nz) || !f || !out) return ORC_ERR_ARG;
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        if (is_bnd(nx, ny, nz, i, j, k)) {
          out[NID(i, j, k)] = 0.0;
          continue;
        }
#define F(di, dj, dk) f[NID(i + (di), j + (dj), k + (dk))]
        out[NID(i, j, k)] = 0.5 * (6.0 * F(0, 0, 0) + F(1, 0, 0) + F(-1, 0, 0) + F(0, 1, 0) + F(0, -1, 0) +
                                   F(0, 0, -1) + F(0, 0, 1));
#undef F
      }
  return ORC_OK;
}

/* copy of x with every boundary entry set to zero */
static double *interior_copy(int nx, int ny, int nz, const double *x) {
  double *t = (double *)malloc(node_count(nx, ny, nz) * sizeof(double));
  if (!t) return NULL;
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) t[NID(i, j, k)] = is_bnd(nx, ny, nz, i, j, k) ? 0.0 : x[NID(i, j, k)];
  return t;
}

/* y = -L x for an x whose boundary entries are already zero */
static void apply_M_zero_bnd(int nx, int ny, int nz, double hx, double hy, double hz, const double *x, double *y) {
  orc_apply_L(nx, ny, nz, hx, hy, hz, x, y);
  const size_t n = node_count(nx, ny, nz);
#pragma omp parallel for schedule(static)
  for (size_t m = 0; m < n; ++m) y[m] = -y[m];
}

int orc_apply_M(int nx, int ny, int nz, double hx, double hy, double hz, const double *x, double *y) {
  if (bad_grid(nx, ny, nz) || !x || !y) return ORC_ERR_ARG;
  double *t = interior_copy(nx, ny, nz, x);
  if (!t) return ORC_ERR_NOMEM;
  apply_M_zero_bnd(nx, ny, nz, hx, hy, hz, t, y);
  free(t);
  return ORC_OK;
}

int orc_rhs(int nx, int ny, int nz, double hx, double hy, double hz, const double *f, const double *g,
            double *b) {
  if (bad_grid(nx, ny, nz) || !f || !g || !b) return ORC_ERR_ARG;
  const size_t n = node_count(nx, ny, nz);
  double *gb = (double *)malloc(n * sizeof(double));
  double *lg = (double *)malloc(n * sizeof(double));
  if (!gb || !lg) {
    free(gb);
    free(lg);
    return ORC_ERR_NOMEM;
  }
  /* g restricted to the boundary: L applied to it gives L_IB g at the interior nodes */
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) gb[NID(i, j, k)] = is_bnd(nx, ny, nz, i, j, k) ? g[NID(i, j, k)] : 0.0;
  orc_apply_L(nx, ny, nz, hx, hy, hz, gb, lg);
  orc_apply_R(nx, ny, nz, hx, hy, hz, f, b);
  for (size_t m = 0; m < n; ++m) b[m] = -b[m] + lg[m];
  free(gb);
  free(lg);
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* conjugate gradients (Algorithm 1, relaxation)                                                                 */
/* ------------------------------------------------------------------------------------------------------------ */

int orc_cg(int nx, int ny, int nz, double hx, double hy, double hz, const double *b, double *u, double tol,
           int max_iters, int fixed_iters, int *iters_out, double *relres_out, double *hist) {
  if (bad_grid(nx, ny, nz) || !b || !u || max_iters < 0) return ORC_ERR_ARG;
  const size_t n = node_count(nx, ny, nz);
  double *r = interior_copy(nx, ny, nz, u);
  double *p = (double *)calloc(n, sizeof(double));
  double *q = (double *)calloc(n, sizeof(double));
  if (!r || !p || !q) {
    free(r); free(p); free(q);
    return ORC_ERR_NOMEM;
  }
  /* r = b - M u */
  apply_M_zero_bnd(nx, ny, nz, hx, hy, hz, r, q);
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) r[NID(i, j, k)] = b[NID(i, j, k)] - q[NID(i, j, k)];
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i)
        if (is_bnd(nx, ny, nz, i, j, k)) r[NID(i, j, k)] = 0.0;

  const double bnorm = sqrt(dot_interior(nx, ny, nz, b, b));
  int status = ORC_OK;
  int it = 0;
  if (bnorm == 0.0) {
    /* b = 0: the solution is u = 0 */
    for (int k = 1; k < nz; ++k)
      for (int j = 1; j < ny; ++j)
        for (int i = 1; i < nx; ++i) u[NID(i, j, k)] = 0.0;
    if (hist) hist[0] = 0.0;
    if (iters_out) *iters_out = 0;
    if (relres_out) *relres_out = 0.0;
    free(r); free(p); free(q);
    return ORC_OK;
  }
  double rho = dot_interior(nx, ny, nz, r, r);
  double rho_old = rho;
  if (hist) hist[0] = sqrt(rho) / bnorm;
  for (;;) {
    int go = (fixed_iters >= 0) ? (it < fixed_iters) : (sqrt(rho) > tol * bnorm);
    if (!go) break;
    if (it >= max_iters) {
      status = ORC_ERR_NOCONV;
      break;
    }
    if (it == 0) {
      for (size_t m = 0; m < n; ++m) p[m] = r[m];
    } else {
      const double beta = rho / rho_old;
      for (size_t m = 0; m < n; ++m) p[m] = r[m] + beta * p[m];
    }
    apply_M_zero_bnd(nx, ny, nz, hx, hy, hz, p, q);
    const double pq = dot_interior(nx, ny, nz, p, q);
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = ORC_ERR_BREAKDOWN;
      break;
    }
    const double alpha = rho / pq;
    for (int k = 1; k < nz; ++k)
      for (int j = 1; j < ny; ++j)
        for (int i = 1; i < nx; ++i) {
          u[NID(i, j, k)] += alpha * p[NID(i, j, k)];
          r[NID(i, j, k)] -= alpha * q[NID(i, j, k)];
        }
    rho_old = rho;
    rho = dot_interior(nx, ny, nz, r, r);
    ++it;
    if (hist) hist[it] = sqrt(rho) / bnorm;
  }
  /* true residual at exit */
  double *t = interior_copy(nx, ny, nz, u);
  if (t) {
    apply_M_zero_bnd(nx, ny, nz, hx, hy, hz, t, q);
    for (int k = 1; k < nz; ++k)
      for (int j = 1; j < ny; ++j)
        for (int i = 1; i < nx; ++i) q[NID(i, j, k)] = b[NID(i, j, k)] - q[NID(i, j, k)];
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i)
          if (is_bnd(nx, ny, nz, i, j, k)) q[NID(i, j, k)] = 0.0;
    if (relres_out) *relres_out = sqrt(dot_interior(nx, ny, nz, q, q)) / bnorm;
    free(t);
  }
  if (iters_out) *iters_out = it;
  free(r); free(p); free(q);
  return status;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* DSOLVE: banded Cholesky of M                                                                                  */
/* ------------------------------------------------------------------------------------------------------------ */

/* interior unknowns numbered lexicographically, x fastest */
static size_t uid(int nx, int ny, int i, int j, int k) {
  return (((size_t)(k - 1)) * (size_t)(ny - 1) + (size_t)(j - 1)) * (size_t)(nx - 1) + (size_t)(i - 1);
}

/* entry of M = -L for neighbour offset (di,dj,dk); the 19 offsets of eq. (compact), 0 for any other offset */
static double M_coef(double a, double b, double c, int di, int dj, int dk) {
  const int s = abs(di) + abs(dj) + abs(dk);
  if (abs(di) > 1 || abs(dj) > 1 || abs(dk) > 1) return 0.0;
  if (s == 0) return 8.0 * (a + b + c);
  if (s == 1) {
    if (di) return -(4.0 * a - b - c);
    if (dj) return -(4.0 * b - a - c);
    return -(4.0 * c - a - b);
  }
  if (s == 2) {
    if (!dk) return -0.5 * (a + b);
    if (!dj) return -0.5 * (a + c);
    return -0.5 * (b + c);
  }
  return 0.0;
}

/* lower band of M: band[m*(w+1) + (m-col)] = M[m][col] for m-w <= col <= m */
static double *assemble_band(int nx, int ny, int nz, double hx, double hy, double hz, size_t *w_out,
                             size_t *n_out) {
  const double a = 1.0 / (hx * hx), b = 1.0 / (hy * hy), c = 1.0 / (hz * hz);
  const size_t n = (size_t)(nx - 1) * (size_t)(ny - 1) * (size_t)(nz - 1);
  const size_t w = (size_t)(nx - 1) * (size_t)(ny - 1) + (size_t)(nx - 1);
  double *band = (double *)calloc(n * (w + 1), sizeof(double));
  if (!band) return NULL;
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        const size_t row = uid(nx, ny, i, j, k);
        for (int dk = -1; dk <= 1; ++dk)
          for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
              const int ii = i + di, jj = j + dj, kk = k + dk;
              if (is_bnd(nx, ny, nz, ii, jj, kk)) continue;
              const double v = M_coef(a, b, c, di, dj, dk);
              if (v == 0.0) continue;
              const size_t col = uid(nx, ny, ii, jj, kk);
              if (col > row) continue;
              band[row * (w + 1) + (row - col)] = v;
            }
      }
  *w_out = w;
  *n_out = n;
  return band;
}

int orc_banded_M_apply(int nx, int ny, int nz, double hx, double hy, double hz, const double *x, double *y) {
  if (bad_grid(nx, ny, nz) || !x || !y) return ORC_ERR_ARG;
  size_t w, n;
  double *band = assemble_band(nx, ny, nz, hx, hy, hz, &w, &n);
  if (!band) return ORC_ERR_NOMEM;
  double *xv = (double *)malloc(n * sizeof(double));
  double *yv = (double *)calloc(n, sizeof(double));
  if (!xv || !yv) {
    free(band); free(xv); free(yv);
    return ORC_ERR_NOMEM;
  }
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) xv[uid(nx, ny, i, j, k)] = x[NID(i, j, k)];
  for (size_t r = 0; r < n; ++r)
    for (size_t d = 0; d <= w && d <= r; ++d) {
      const double v = band[r * (w + 1) + d];
      if (v == 0.0) continue;
      yv[r] += v * xv[r - d];
      if (d) yv[r - d] += v * xv[r];
    }
  memset(y, 0, node_count(nx, ny, nz) * sizeof(double));
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) y[NID(i, j, k)] = yv[uid(nx, ny, i, j, k)];
  free(band); free(xv); free(yv);
  return ORC_OK;
}

int orc_direct_solve(int nx, int ny, int nz, double hx, double hy, double hz, const double *b, double *u) {
  if (bad_grid(nx, ny, nz) || !b || !u) return ORC_ERR_ARG;
  size_t w, n;
  double *L = assemble_band(nx, ny, nz, hx, hy, hz, &w, &n);
  if (!L) return ORC_ERR_NOMEM;
  const size_t W = w + 1;
  /* Cholesky M = L L^T on the band, column by column */
  for (size_t j = 0; j < n; ++j) {
    const size_t k0 = (j > w) ? j - w : 0;
    double s = L[j * W + 0];
    for (size_t k = k0; k < j; ++k) s -= L[j * W + (j - k)] * L[j * W + (j - k)];
    if (!(s > 0.0)) {
      free(L);
      return ORC_ERR_BREAKDOWN;
    }
    const double d = sqrt(s);
    L[j * W + 0] = d;
    const size_t iend = (j + w < n - 1) ? j + w : n - 1;
    for (size_t i = j + 1; i <= iend; ++i) {
      const size_t kk0 = (i > w) ? i - w : 0;
      double t = L[i * W + (i - j)];
      for (size_t k = (kk0 > k0 ? kk0 : k0); k < j; ++k) t -= L[i * W + (i - k)] * L[j * W + (j - k)];
      L[i * W + (i - j)] = t / d;
    }
  }
  double *y = (double *)malloc(n * sizeof(double));
  if (!y) {
    free(L);
    return ORC_ERR_NOMEM;
  }
  for (int k = 1; k < nz; ++k)
    for (int jj = 1; jj < ny; ++jj)
      for (int i = 1; i < nx; ++i) y[uid(nx, ny, i, jj, k)] = b[NID(i, jj, k)];
  /* forward: L y = b */
  for (size_t i = 0; i < n; ++i) {
    double s = y[i];
    const size_t k0 = (i > w) ? i - w : 0;
    for (size_t k = k0; k < i; ++k) s -= L[i * W + (i - k)] * y[k];
    y[i] = s / L[i * W + 0];
  }
  /* backward: L^T x = y */
  for (size_t ii = n; ii-- > 0;) {
    double s = y[ii];
    const size_t kend = (ii + w < n - 1) ? ii + w : n - 1;
    for (size_t k = ii + 1; k <= kend; ++k) s -= L[k * W + (k - ii)] * y[k];
    y[ii] = s / L[ii * W + 0];
  }
  for (int k = 1; k < nz; ++k)
    for (int jj = 1; jj < ny; ++jj)
      for (int i = 1; i < nx; ++i) u[NID(i, jj, k)] = y[uid(nx, ny, i, jj, k)];
  free(y);
  free(L);
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* extrapolation and tri-quartic interpolation (Sections 4.2 and 4.3)                                           */
/* ------------------------------------------------------------------------------------------------------------ */

double orc_lagrange4(int a, double t) {
  double v = 1.0;
  for (int m = 0; m <= 4; ++m) {
    if (m == a) continue;
    v *= (t - (double)m) / ((double)a - (double)m);
  }
  return v;
}

/* Mean over the 2^(m-1) diagonals through a node whose odd axes are listed in ax[0..m-1]: each diagonal joins the
 * two opposite corners base+s and base-s (s = +-1 on the odd axes, 0 on the even ones), and contributes
 * center + weight*(delta(base+s) + delta(base-s)).  delta is read through dfun at coarse-grid corners.
 * With m = 1 this is the midpoint formula itself; m = 2 the face-centre rule; m = 3 the element-centre rule. */
typedef double (*delta_fn)(const void *ctx, int I, int J, int K);

static double diagonal_mean(double center, double weight, int I, int J, int K, const int *odd, int m,
                            delta_fn dfun, const void *ctx) {
  double acc = 0.0;
  int count = 0;
  const int patterns = 1 << (m - 1);
  for (int p = 0; p < patterns; ++p) {
    int s[3] = {0, 0, 0};
    /* first odd axis fixed to -1 so each diagonal is taken once; the rest take both signs */
    s[odd[0]] = -1;
    for (int q = 1; q < m; ++q) s[odd[q]] = ((p >> (q - 1)) & 1) ? 1 : -1;
    const double da = dfun(ctx, I + s[0], J + s[1], K + s[2]);
    const double db = dfun(ctx, I - s[0], J - s[1], K - s[2]);
    acc += center + weight * (da + db);
    ++count;
  }
  return acc / (double)count;
}

typedef struct {
  const double *fine; /* the finer of the two solutions, on its own grid */
  const double *coarse;
  dims_t fd, cd; /* dims of fine and coarse arrays */
} delta_ctx;

/* delta at a node (I,J,K) of the finer grid that is also a coarse node: finer - coarser */
static double delta_at(const void *vctx, int I, int J, int K) {
  const delta_ctx *c = (const delta_ctx *)vctx;
  const size_t fi = (((size_t)K) * (size_t)(c->fd.ny + 1) + (size_t)J) * (size_t)(c->fd.nx + 1) + (size_t)I;
  const int Ic = I / 2, Jc = J / 2, Kc = K / 2;
  const size_t ci = (((size_t)Kc) * (size_t)(c->cd.ny + 1) + (size_t)Jc) * (size_t)(c->cd.nx + 1) + (size_t)Ic;
  return c->fine[fi] - c->coarse[ci];
}

/* The known values of the fine grid's interpolation: the extrapolated value at every node of the 2h grid (which is a
 * fine node with all offsets even), written into w there.  nx, ny, nz multiples of 4. */
static void extrapolate_2h_nodes(int nx, int ny, int nz, const double *u2h, const double *u4h, double *w) {
  const int mx = nx / 2, my = ny / 2, mz = nz / 2; /* 2h grid */
  delta_ctx ctx;
  ctx.fine = u2h;
  ctx.coarse = u4h;
  ctx.fd.nx = mx; ctx.fd.ny = my; ctx.fd.nz = mz;
  ctx.cd.nx = mx / 2; ctx.cd.ny = my / 2; ctx.cd.nz = mz / 2;

  /* 1. the 125 known nodes of every cell = every node of the 2h grid: eq. (jiedian) at 4h nodes, eq. (zhongdian)
   *    at edge midpoints, mean over 2 face diagonals at face centres, mean over 4 space diagonals at centres. */
#pragma omp parallel for schedule(static)
  for (int K = 0; K <= mz; ++K)
    for (int J = 0; J <= my; ++J)
      for (int I = 0; I <= mx; ++I) {
        const size_t ci = (((size_t)K) * (size_t)(my + 1) + (size_t)J) * (size_t)(mx + 1) + (size_t)I;
        int odd[3], m = 0;
        if (I & 1) odd[m++] = 0;
        if (J & 1) odd[m++] = 1;
        if (K & 1) odd[m++] = 2;
        double v;
        if (m == 0) {
          const size_t qi = (((size_t)(K / 2)) * (size_t)(my / 2 + 1) + (size_t)(J / 2)) * (size_t)(mx / 2 + 1) +
                            (size_t)(I / 2);
          v = (17.0 * u2h[ci] - u4h[qi]) / 16.0;
        } else {
          v = diagonal_mean(u2h[ci], 1.0 / 32.0, I, J, K, odd, m, delta_at, &ctx);
        }
        w[NID(2 * I, 2 * J, 2 * K)] = v;
      }
}

int orc_exp_finite(int nx, int ny, int nz, const double *u2h, const double *u4h, const double *g, double *w) {
  if (!u2h || !u4h || !g || !w) return ORC_ERR_ARG;
  if (nx % 8 || ny % 8 || nz % 8 || nx < 8 || ny < 8 || nz < 8) return ORC_ERR_SHAPE;
  extrapolate_2h_nodes(nx, ny, nz, u2h, u4h, w);

  /* 2. tri-quartic Lagrange interpolation (eq. inter) on each cell of 2x2x2 elements of the 4h grid (8x8x8 fine
   *    elements): the 604 remaining nodes of the cell from its 125 known nodes, natural coordinate t = offset/2. */
  double lw[9][5];
  for (int o = 0; o <= 8; ++o)
    for (int a = 0; a <= 4; ++a) lw[o][a] = orc_lagrange4(a, 0.5 * (double)o);
  const int cx = nx / 8, cy = ny / 8, cz = nz / 8;
#pragma omp parallel for schedule(static)
  for (int ck = 0; ck < cz; ++ck)
    for (int cj = 0; cj < cy; ++cj)
      for (int ci = 0; ci < cx; ++ci)
        for (int ok = 0; ok <= 8; ++ok)
          for (int oj = 0; oj <= 8; ++oj)
            for (int oi = 0; oi <= 8; ++oi) {
              if (!(oi & 1) && !(oj & 1) && !(ok & 1)) continue; /* a known node */
              double s = 0.0;
              for (int c = 0; c <= 4; ++c)
                for (int b = 0; b <= 4; ++b)
                  for (int a = 0; a <= 4; ++a)
                    s += lw[oi][a] * lw[oj][b] * lw[ok][c] * w[NID(8 * ci + 2 * a, 8 * cj + 2 * b, 8 * ck + 2 * c)];
              w[NID(8 * ci + oi, 8 * cj + oj, 8 * ck + ok)] = s;
            }

  /* 3. Dirichlet values on the boundary */
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i)
        if (is_bnd(nx, ny, nz, i, j, k)) w[NID(i, j, k)] = g[NID(i, j, k)];
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* the other initial guesses the paper compares with (its remark on the interpolation order, Section 4.3, and the   */
/* CMG method of Section 3)                                                                                     */
/* ------------------------------------------------------------------------------------------------------------ */

double orc_lagrange2(int a, double t) {
  double v = 1.0;
  for (int m = 0; m <= 2; ++m) {
    if (m == a) continue;
    v *= (t - (double)m) / ((double)a - (double)m);
  }
  return v;
}

int orc_initial_guess(int kind, int nx, int ny, int nz, const double *u2h, const double *u4h, const double *g,
                      double *w) {
  if (!u2h || !g || !w) return ORC_ERR_ARG;
  if (kind == ORC_GUESS_QUARTIC) {
    if (!u4h) return ORC_ERR_ARG;
    return orc_exp_finite(nx, ny, nz, u2h, u4h, g, w);
  }
  if (kind == ORC_GUESS_QUADRATIC) {
    if (!u4h) return ORC_ERR_ARG;
    if (nx % 4 || ny % 4 || nz % 4 || nx < 4 || ny < 4 || nz < 4) return ORC_ERR_SHAPE;
    extrapolate_2h_nodes(nx, ny, nz, u2h, u4h, w);
    /* tri-quadratic Lagrange interpolation on each cell of 2x2x2 elements of the 2h grid (4x4x4 fine elements):
     * the nodes of the cell with an odd offset from its 27 known nodes, natural coordinate t = offset/2 */
    double lw[5][3];
    for (int o = 0; o <= 4; ++o)
      for (int a = 0; a <= 2; ++a) lw[o][a] = orc_lagrange2(a, 0.5 * (double)o);
    const int cx = nx / 4, cy = ny / 4, cz = nz / 4;
#pragma omp parallel for schedule(static)
    for (int ck = 0; ck < cz; ++ck)
      for (int cj = 0; cj < cy; ++cj)
        for (int ci = 0; ci < cx; ++ci)
          for (int ok = 0; ok <= 4; ++ok)
            for (int oj = 0; oj <= 4; ++oj)
              for (int oi = 0; oi <= 4; ++oi) {
                if (!(oi & 1) && !(oj & 1) && !(ok & 1)) continue; /* a known node */
                double s = 0.0;
                for (int c = 0; c <= 2; ++c)
                  for (int b = 0; b <= 2; ++b)
                    for (int a = 0; a <= 2; ++a)
                      s += lw[oi][a] * lw[oj][b] * lw[ok][c] * w[NID(4 * ci + 2 * a, 4 * cj + 2 * b, 4 * ck + 2 * c)];
                w[NID(4 * ci + oi, 4 * cj + oj, 4 * ck + ok)] = s;
              }
  } else if (kind == ORC_GUESS_LINEAR) {
    if (nx % 2 || ny % 2 || nz % 2 || nx < 2 || ny < 2 || nz < 2) return ORC_ERR_SHAPE;
    /* trilinear interpolation of u_2h itself (no extrapolation): a fine node at 2h coordinates (i/2, j/2, k/2) is the
     * weighted sum over the corners of the 2h element that holds it */
    const int mx = nx / 2, my = ny / 2;
#pragma omp parallel for schedule(static)
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
          const int I0 = i / 2, J0 = j / 2, K0 = k / 2;
          const double fx = 0.5 * (i % 2), fy = 0.5 * (j % 2), fz = 0.5 * (k % 2);
          double s = 0.0;
          for (int dk = 0; dk <= 1; ++dk)
            for (int dj = 0; dj <= 1; ++dj)
              for (int di = 0; di <= 1; ++di) {
                const double wgt = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
                if (wgt == 0.0) continue; /* the corner past the grid's last node carries no weight */
                const size_t ci = (((size_t)(K0 + dk)) * (size_t)(my + 1) + (size_t)(J0 + dj)) * (size_t)(mx + 1) +
                                  (size_t)(I0 + di);
                s += wgt * u2h[ci];
              }
          w[NID(i, j, k)] = s;
        }
  } else {
    return ORC_ERR_ARG;
  }
  /* Dirichlet values on the boundary */
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i)
        if (is_bnd(nx, ny, nz, i, j, k)) w[NID(i, j, k)] = g[NID(i, j, k)];
  return ORC_OK;
}

int orc_exp_true(int nx, int ny, int nz, const double *uh, const double *u2h, double *ut) {
  if (!uh || !u2h || !ut) return ORC_ERR_ARG;
  if (nx % 2 || ny % 2 || nz % 2 || nx < 2 || ny < 2 || nz < 2) return ORC_ERR_SHAPE;
  delta_ctx ctx;
  ctx.fine = uh;
  ctx.coarse = u2h;
  ctx.fd.nx = nx; ctx.fd.ny = ny; ctx.fd.nz = nz;
  ctx.cd.nx = nx / 2; ctx.cd.ny = ny / 2; ctx.cd.nz = nz / 2;
#pragma omp parallel for schedule(static)
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i) {
        int odd[3], m = 0;
        if (i & 1) odd[m++] = 0;
        if (j & 1) odd[m++] = 1;
        if (k & 1) odd[m++] = 2;
        double v;
        if (m == 0) {
          const size_t qi = (((size_t)(k / 2)) * (size_t)(ny / 2 + 1) + (size_t)(j / 2)) * (size_t)(nx / 2 + 1) +
                            (size_t)(i / 2);
          v = (16.0 * uh[NID(i, j, k)] - u2h[qi]) / 15.0; /* eq. (t1) */
        } else {
          v = diagonal_mean(uh[NID(i, j, k)], 1.0 / 30.0, i, j, k, odd, m, delta_at, &ctx); /* eq. (chenlin) */
        }
        ut[NID(i, j, k)] = v;
      }
  return ORC_OK;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* compact fourth-order gradient (Section 5.1)                                                                  */
/* ------------------------------------------------------------------------------------------------------------ */

/* one grid line: u[0..N] with stride s -> v[0..N] with stride s */
static void gradient_line(int N, double h, const double *u, size_t s, double *v, double *cp, double *dp) {
#define UL(t) u[(size_t)(t) * s]
#define VL(t) v[(size_t)(t) * s]
  VL(0) = (-25.0 / 12.0 * UL(0) + 4.0 * UL(1) - 3.0 * UL(2) + 4.0 / 3.0 * UL(3) - 0.25 * UL(4)) / h;
  VL(N) = (25.0 / 12.0 * UL(N) - 4.0 * UL(N - 1) + 3.0 * UL(N - 2) - 4.0 / 3.0 * UL(N - 3) + 0.25 * UL(N - 4)) / h;
  /* (1/6) v_{i-1} + (4/6) v_i + (1/6) v_{i+1} = (u_{i+1} - u_{i-1}) / (2h), i = 1..N-1; Thomas algorithm */
  const double lo = 1.0 / 6.0, di = 4.0 / 6.0, up = 1.0 / 6.0;
  for (int i = 1; i <= N - 1; ++i) {
    double d = (UL(i + 1) - UL(i - 1)) / (2.0 * h);
    if (i == 1) d -= lo * VL(0);
    if (i == N - 1) d -= up * VL(N);
    if (i == 1) {
      cp[i] = up / di;
      dp[i] = d / di;
    } else {
      const double m = di - lo * cp[i - 1];
      cp[i] = up / m;
      dp[i] = (d - lo * dp[i - 1]) / m;
    }
  }
  VL(N - 1) = dp[N - 1];
  for (int i = N - 2; i >= 1; --i) VL(i) = dp[i] - cp[i] * VL(i + 1);
#undef UL
#undef VL
}

int orc_gradient(int nx, int ny, int nz, double hx, double hy, double hz, const double *u, double *ux,
                 double *uy, double *uz) {
  if (!u || !ux || !uy || !uz) return ORC_ERR_ARG;
  if (nx < 4 || ny < 4 || nz < 4) return ORC_ERR_SHAPE;
  const int nmax = (nx > ny ? (nx > nz ? nx : nz) : (ny > nz ? ny : nz)) + 1;
  int err = ORC_OK;
#pragma omp parallel
  {
    double *cp = (double *)malloc((size_t)nmax * sizeof(double));
    double *dp = (double *)malloc((size_t)nmax * sizeof(double));
    if (!cp || !dp) {
#pragma omp atomic write
      err = ORC_ERR_NOMEM;
    } else {
#pragma omp for schedule(static)
      for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= ny; ++j) gradient_line(nx, hx, u + NID(0, j, k), 1, ux + NID(0, j, k), cp, dp);
#pragma omp for schedule(static)
      for (int k = 0; k <= nz; ++k)
        for (int i = 0; i <= nx; ++i)
          gradient_line(ny, hy, u + NID(i, 0, k), (size_t)(nx + 1), uy + NID(i, 0, k), cp, dp);
#pragma omp for schedule(static)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i)
          gradient_line(nz, hz, u + NID(i, j, 0), (size_t)(nx + 1) * (size_t)(ny + 1), uz + NID(i, j, 0), cp, dp);
    }
    free(cp);
    free(dp);
  }
  return err;
}

/* ------------------------------------------------------------------------------------------------------------ */
/* Algorithm 1 (EXCMG)                                                                                          */
/* ------------------------------------------------------------------------------------------------------------ */

/* number of halvings Lt with nc*2^Lt = n on every axis, or -1 */
static int level_count(int nx, int ny, int nz, int ncx, int ncy, int ncz) {
  if (ncx < 2 || ncy < 2 || ncz < 2) return -1;
  for (int t = 0; t < 30; ++t) {
    if ((ncx << t) == nx && (ncy << t) == ny && (ncz << t) == nz) return t;
    if ((ncx << t) > nx) break;
  }
  return -1;
}

/* node array of level dims (lx,ly,lz) sampled from the finest array at stride s */
static void sample_stride(int nx, int ny, int nz, const double *fine, int s, int mx, int my, int mz, double *out) {
  for (int k = 0; k <= mz; ++k)
    for (int j = 0; j <= my; ++j)
      for (int i = 0; i <= mx; ++i) {
        const size_t fi = NID(i * s, j * s, k * s);
        out[(((size_t)k) * (size_t)(my + 1) + (size_t)j) * (size_t)(mx + 1) + (size_t)i] = fine[fi];
      }
}

/* shared cascade; mode 0: b_l from (f, g); mode 1: b_l = G on the interior, zero Dirichlet data */
static int cascade(int mode, int guess, int stop_norm, int nx, int ny, int nz, double lx, double ly, double lz,
                   int ncx, int ncy, int ncz, const double *f, const double *g, double tol, double tol_order,
                   int max_iters, const int *fixed_iters, double *u, double *ut, double *w_out, int *iters,
                   double *relres, double *seconds) {
  if (!f || !u || !iters || !relres) return ORC_ERR_ARG;
  if (mode == 0 && !g) return ORC_ERR_ARG;
  if (!(lx > 0) || !(ly > 0) || !(lz > 0) || !(tol > 0) || max_iters < 0) return ORC_ERR_ARG;
  const int Lt = level_count(nx, ny, nz, ncx, ncy, ncz);
  if (Lt < 0) return ORC_ERR_SHAPE;
  if (Lt >= 2 && (ncx % 2 || ncy % 2 || ncz % 2)) return ORC_ERR_SHAPE;
  if (ut && Lt < 1) return ORC_ERR_SHAPE;
  if (w_out && Lt < 2) return ORC_ERR_SHAPE;
  const double t0 = now_s();
  double t_cg = 0.0;
  double *lev[32];
  memset(lev, 0, sizeof(lev));
  double *fl = NULL, *gl = NULL, *bl = NULL;
  int status = ORC_OK;
  const size_t nmax = node_count(nx, ny, nz);
  fl = (double *)malloc(nmax * sizeof(double));
  gl = (double *)malloc(nmax * sizeof(double));
  bl = (double *)malloc(nmax * sizeof(double));
  if (!fl || !gl || !bl) {
    status = ORC_ERR_NOMEM;
    goto done;
  }
  for (int l = 0; l <= Lt; ++l) {
    const int s = 1 << (Lt - l);
    const int mx = ncx << l, my = ncy << l, mz = ncz << l;
    const double hx = lx / mx, hy = ly / my, hz = lz / mz;
    const size_t nl = node_count(mx, my, mz);
    double *ul = (l == Lt) ? u : (double *)calloc(nl, sizeof(double));
    if (!ul) {
      status = ORC_ERR_NOMEM;
      goto done;
    }
    if (l != Lt) lev[l] = ul;
    /* level data by injection from the finest arrays */
    sample_stride(nx, ny, nz, f, s, mx, my, mz, fl);
    if (mode == 0) {
      sample_stride(nx, ny, nz, g, s, mx, my, mz, gl);
      orc_rhs(mx, my, mz, hx, hy, hz, fl, gl, bl);
    } else {
      memset(gl, 0, nl * sizeof(double));
      for (int k = 0; k <= mz; ++k)
        for (int j = 0; j <= my; ++j)
          for (int i = 0; i <= mx; ++i) {
            const size_t m = (((size_t)k) * (size_t)(my + 1) + (size_t)j) * (size_t)(mx + 1) + (size_t)i;
            bl[m] = is_bnd(mx, my, mz, i, j, k) ? 0.0 : fl[m];
          }
    }
    if (l <= 1) {
      /* DSOLVE on the two coarsest grids */
      memcpy(ul, gl, nl * sizeof(double));
      int e = orc_direct_solve(mx, my, mz, hx, hy, hz, bl, ul);
      if (e) {
        status = e;
        goto done;
      }
      iters[l] = 0;
      /* residual of the direct solve, for the record */
      double *tmp = (double *)malloc(nl * sizeof(double));
      double *rr = (double *)malloc(nl * sizeof(double));
      if (tmp && rr) {
        orc_apply_M(mx, my, mz, hx, hy, hz, ul, tmp);
        for (size_t m = 0; m < nl; ++m) rr[m] = bl[m] - tmp[m];
        const double bn = sqrt(dot_interior(mx, my, mz, bl, bl));
        const double rn = sqrt(dot_interior(mx, my, mz, rr, rr));
        relres[l] = bn > 0 ? rn / bn : 0.0;
      }
      free(tmp);
      free(rr);
    } else {
      /* w_h = EXP_finite(u_2h, u_4h) (or the compared initial guess), then CG from w_h */
      const double *u2 = lev[l - 1], *u4 = lev[l - 2];
      int e = orc_initial_guess(guess, mx, my, mz, u2, u4, gl, ul);
      if (e) {
        status = e;
        goto done;
      }
      if (l == Lt && w_out) memcpy(w_out, ul, nl * sizeof(double));
      const int fi = fixed_iters ? fixed_iters[l] : -1;
      /* the stopping test ||r|| <= tol ||f_h||: f_h = b (the eliminated right-hand side) or, with stop_norm 1, the
       * vector of R f on the interior nodes and g on the boundary nodes; with stop_norm 2, that vector on every level
       * below the finest and b on the finest; the CG's test is against ||b||, so the tolerance is rescaled by
       * ||f_h|| / ||b|| */
      /* the level's tolerance: tol on every level, or (a schedule the paper does not give, for its remark on the
       * extrapolated solution in Section 5.1) tol * 2^(tol_order (Lt - l)), capped at max(tol, 1e-2) */
      double tol_l = tol;
      if (tol_order > 0.0) {
        const double cap = tol > 1e-2 ? tol : 1e-2;
        tol_l = tol * pow(2.0, tol_order * (double)(Lt - l));
        if (tol_l > cap) tol_l = cap;
      }
      if (stop_norm == 1 || (stop_norm == 2 && l < Lt)) {
        double *rf = (double *)malloc(nl * sizeof(double));
        if (!rf) {
          status = ORC_ERR_NOMEM;
          goto done;
        }
        orc_apply_R(mx, my, mz, hx, hy, hz, fl, rf);
        double fg2 = dot_interior(mx, my, mz, rf, rf);
        for (int k = 0; k <= mz; ++k)
          for (int j = 0; j <= my; ++j)
            for (int i = 0; i <= mx; ++i)
              if (is_bnd(mx, my, mz, i, j, k)) {
                const double gv = gl[(((size_t)k) * (size_t)(my + 1) + (size_t)j) * (size_t)(mx + 1) + (size_t)i];
                fg2 += gv * gv;
              }
        free(rf);
        const double bn = sqrt(dot_interior(mx, my, mz, bl, bl));
        tol_l = bn > 0.0 ? tol_l * sqrt(fg2) / bn : tol_l;
      }
      const double tc = now_s();
      e = orc_cg(mx, my, mz, hx, hy, hz, bl, ul, tol_l, max_iters, fi, &iters[l], &relres[l], NULL);
      t_cg += now_s() - tc;
      if (e) status = e;
      if (e && e != ORC_ERR_NOCONV) goto done;
      /* only the two previous levels are needed from here on */
      if (l - 2 >= 0 && lev[l - 2]) {
        free(lev[l - 2]);
        lev[l - 2] = NULL;
      }
    }
    if (g_progress) {
      fprintf(stderr, "oracle: grid %d of %d (%d x %d x %d cells) done, %d iterations, %.1f s\n", l, Lt + 1, mx, my,
              mz, iters[l], now_s() - t0);
      fflush(stderr);
    }
  }
  if (ut) {
    int e = orc_exp_true(nx, ny, nz, u, lev[Lt - 1], ut);
    if (e) status = e;
  }
done:
  for (int l = 0; l < 32; ++l) free(lev[l]);
  free(fl);
  free(gl);
  free(bl);
  if (seconds) {
    seconds[0] = now_s() - t0;
    seconds[1] = t_cg;
  }
  return status;
}

int orc_excmg(int nx, int ny, int nz, double lx, double ly, double lz, int ncx, int ncy, int ncz,
              const double *f, const double *g, double tol, int max_iters, const int *fixed_iters, double *u,
              double *ut, double *w_out, int *iters, double *relres, double *seconds) {
  return cascade(0, ORC_GUESS_QUARTIC, 0, nx, ny, nz, lx, ly, lz, ncx, ncy, ncz, f, g, tol, 0.0, max_iters,
                 fixed_iters, u, ut, w_out, iters, relres, seconds);
}

int orc_excmg_variant(int guess, int stop_norm, int nx, int ny, int nz, double lx, double ly, double lz, int ncx,
                      int ncy, int ncz, const double *f, const double *g, double tol, double tol_order,
                      int max_iters, const int *fixed_iters, double *u, double *ut, double *w_out, int *iters,
                      double *relres) {
  if (guess != ORC_GUESS_QUARTIC && guess != ORC_GUESS_QUADRATIC && guess != ORC_GUESS_LINEAR) return ORC_ERR_ARG;
  if (stop_norm != 0 && stop_norm != 1 && stop_norm != 2) return ORC_ERR_ARG;
  if (!(tol_order >= 0.0) || tol_order > 16.0) return ORC_ERR_ARG;
  return cascade(0, guess, stop_norm, nx, ny, nz, lx, ly, lz, ncx, ncy, ncz, f, g, tol, tol_order, max_iters,
                 fixed_iters, u, ut, w_out, iters, relres, NULL);
}

/* ------------------------------------------------------------------------------------------------------------ */
/* adjoint                                                                                                      */
/* ------------------------------------------------------------------------------------------------------------ */

int orc_apply_RT(int nx, int ny, int nz, const double *lam, double *out) {
  if (bad_grid(nx, ny, nz) || !lam || !out) return ORC_ERR_ARG;
  memset(out, 0, node_count(nx, ny, nz) * sizeof(double));
  /* R has 3 on the diagonal and 1/2 for each face neighbour: scatter every interior row into its columns */
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        const double l = lam[NID(i, j, k)];
        out[NID(i, j, k)] += 3.0 * l;
        out[NID(i + 1, j, k)] += 0.5 * l;
        out[NID(i - 1, j, k)] += 0.5 * l;
        out[NID(i, j + 1, k)] += 0.5 * l;
        out[NID(i, j - 1, k)] += 0.5 * l;
        out[NID(i, j, k + 1)] += 0.5 * l;
        out[NID(i, j, k - 1)] += 0.5 * l;
      }
  return ORC_OK;
}

int orc_apply_LIBT(int nx, int ny, int nz, double hx, double hy, double hz, const double *lam, double *out) {
  if (bad_grid(nx, ny, nz) || !lam || !out) return ORC_ERR_ARG;
  const double a = 1.0 / (hx * hx), b = 1.0 / (hy * hy), c = 1.0 / (hz * hz);
  memset(out, 0, node_count(nx, ny, nz) * sizeof(double));
  /* L's coefficient for offset d is -M_coef(d); scatter each interior row into its boundary columns */
  for (int k = 1; k < nz; ++k)
    for (int j = 1; j < ny; ++j)
      for (int i = 1; i < nx; ++i) {
        const double l = lam[NID(i, j, k)];
        for (int dk = -1; dk <= 1; ++dk)
          for (int dj = -1; dj <= 1; ++dj)
            for (int di = -1; di <= 1; ++di) {
              const int ii = i + di, jj = j + dj, kk = k + dk;
              if (!is_bnd(nx, ny, nz, ii, jj, kk)) continue;
              const double v = -M_coef(a, b, c, di, dj, dk);
              if (v == 0.0) continue;
              out[NID(ii, jj, kk)] += v * l;
            }
      }
  return ORC_OK;
}

int orc_adjoint(int nx, int ny, int nz, double lx, double ly, double lz, int ncx, int ncy, int ncz,
                const double *G, double tol, int max_iters, const int *fixed_iters, double *dLdf, double *dLdg,
                double *lambda_out, int *iters, double *relres) {
  if (!G || !dLdf || !dLdg) return ORC_ERR_ARG;
  const size_t n = node_count(nx, ny, nz);
  double *lam = (double *)calloc(n, sizeof(double));
  if (!lam) return ORC_ERR_NOMEM;
  int status = cascade(1, ORC_GUESS_QUARTIC, 0, nx, ny, nz, lx, ly, lz, ncx, ncy, ncz, G, NULL, tol, 0.0, max_iters,
                       fixed_iters, lam, NULL, NULL, iters, relres, NULL);
  if (status && status != ORC_ERR_NOCONV) {
    free(lam);
    return status;
  }
  const double hx = lx / nx, hy = ly / ny, hz = lz / nz;
  orc_apply_RT(nx, ny, nz, lam, dLdf);
  for (size_t m = 0; m < n; ++m) dLdf[m] = -dLdf[m];
  orc_apply_LIBT(nx, ny, nz, hx, hy, hz, lam, dLdg);
  for (int k = 0; k <= nz; ++k)
    for (int j = 0; j <= ny; ++j)
      for (int i = 0; i <= nx; ++i)
        if (is_bnd(nx, ny, nz, i, j, k)) dLdg[NID(i, j, k)] += G[NID(i, j, k)];
  if (lambda_out) memcpy(lambda_out, lam, n * sizeof(double));
  free(lam);
  return status;
}
