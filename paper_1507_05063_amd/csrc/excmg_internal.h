// Internal declarations of the gfx950 EXCMG library: array layout, stencil coefficients, device scalar state and
// the launchers of every kernel.  Host code and kernels share this header; nothing here is part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/excmg.h"

namespace excmg {

// ------------------------------------------------------------------------------------------------------------
// Layout of a node array: element (i,j,k) at base + off + k*sz + j*sy + i.
// User arrays are dense (off = 0, sy = Nx+1, sz = (Nx+1)(Ny+1)).  The library's own arrays are pitched so that the
// first interior node of every row (i = 1) starts a 128-byte line: off = A-1 and sy a multiple of A, with
// A = 128 / sizeof(T).  Whole 64-lane row segments of interior nodes then map to whole cache lines.
// ------------------------------------------------------------------------------------------------------------
struct Grid {
  int nx, ny, nz;   // cells per axis; nodes 0..n
  long long sy, sz; // element strides of a row (j) and a plane (k)
  long long off;    // element offset of node (0,0,0)
  long long elems;  // elements to allocate (including the leading offset and a tail pad)

  __host__ __device__ long long at(int i, int j, int k) const {
    return off + (long long)k * sz + (long long)j * sy + (long long)i;
  }
  __host__ __device__ long long interior() const { return (long long)(nx - 1) * (ny - 1) * (nz - 1); }
  __host__ __device__ long long nodes() const { return (long long)(nx + 1) * (ny + 1) * (nz + 1); }
};

// DSOLVE (the exact solve of the two coarsest grids, Algorithm 1) by sine transforms in one workgroup: grids of at
// most kDstMax cells per axis.  Larger direct-solve grids are solved by CG to a relative residual of kDsolveTol (one
// workgroup up to kSmallCg unknowns, else the multi-workgroup sweeps), which reports EXCMG_ERR_NOCONV if its
// iteration cap is reached first.
constexpr int kDstMax = 64;
constexpr double kDsolveTol = 1e-15;
constexpr long long kSmallCg = 8000;

__host__ __device__ inline bool dst_fits(const Grid &g) {
  return g.nx <= kDstMax && g.ny <= kDstMax && g.nz <= kDstMax;
}

// Iteration cap of a direct solve by CG on a grid of n interior unknowns.
inline int dsolve_cap(long long n) {
  const long long c = 4 * n + 200;
  return c > 20000 ? 20000 : (int)c;
}

inline Grid dense_grid(int nx, int ny, int nz) {
  Grid g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.sy = nx + 1;
  g.sz = (long long)(nx + 1) * (ny + 1);
  g.off = 0;
  g.elems = g.sz * (nz + 1);
  return g;
}

template <typename T>
inline Grid pitched_grid(int nx, int ny, int nz) {
  const long long A = 128 / (long long)sizeof(T);
  Grid g;
  g.nx = nx; g.ny = ny; g.nz = nz;
  g.off = A - 1;
  g.sy = ((nx + A) + A - 1) / A * A;  // holds off + nx + 1 elements, a multiple of A
  g.sz = g.sy * (ny + 1);
  g.elems = ((g.off + g.sz * (nz + 1) + A) + A - 1) / A * A;
  return g;
}

// Coefficients of M = -A_h (eq. compact negated), a = 1/hx^2, b = 1/hy^2, c = 1/hz^2:
//   centre 8(a+b+c); x faces -(4a-b-c); y faces -(4b-a-c); z faces -(4c-a-b);
//   xy edges -(a+b)/2; xz edges -(a+c)/2; yz edges -(b+c)/2.
struct Stencil {
  double c0, cx, cy, cz, cxy, cxz, cyz;
};

inline Stencil make_stencil(double hx, double hy, double hz) {
  const double a = 1.0 / (hx * hx), b = 1.0 / (hy * hy), c = 1.0 / (hz * hz);
  Stencil s;
  s.c0 = 8.0 * (a + b + c);
  s.cx = -(4.0 * a - b - c);
  s.cy = -(4.0 * b - a - c);
  s.cz = -(4.0 * c - a - b);
  s.cxy = -0.5 * (a + b);
  s.cxz = -0.5 * (a + c);
  s.cyz = -0.5 * (b + c);
  return s;
}

// Level right-hand side at an interior node (i,j,k) of a grid with cells (nx,ny,nz), read from the finest dense
// arrays at stride s (level data by injection, Section 2: every coarse node is a fine node).
//   mode 0: b = -R f + A_IB g, R f = (6 f_c + sum of the 6 face neighbours)/2 and, for neighbours on the boundary,
//           A's coefficient times g: faces (4a-b-c), (4b-a-c), (4c-a-b); edges (a+b)/2, (a+c)/2, (b+c)/2
//           (eq. compact with the Dirichlet values moved to the right, negated so that M = -A_h is positive definite)
//   mode 1: b = f(i s, j s, k s) (the adjoint's data, zero Dirichlet values)
struct RhsSrc {
  Grid gf;          // layout of the finest dense arrays
  const double *f;  // f (mode 0) or the adjoint's G (mode 1)
  const double *g;  // Dirichlet data (mode 0), only boundary nodes read
  int s;            // stride into the finest arrays
  int mode;
  double a, b, c;   // 1/hx^2, 1/hy^2, 1/hz^2 of the level
  int fg;           // 1 (mode 0 only): the stopping test's norm is that of (R f inside, g on the boundary), so the
                    // residual sweeps sum (R f)^2 where they otherwise sum b^2 (EXCMG_STOP_F_G)
};

// A's couplings to the Dirichlet values of the boundary neighbours of (i,j,k) (only nodes next to the boundary have any)
__device__ __forceinline__ double rhs_boundary_terms_inl(const RhsSrc &rs, int nx, int ny, int nz, int i, int j,
                                                         int k) {
  const int s = rs.s;
  const double a = rs.a, b = rs.b, c = rs.c;
  const double fx = 4.0 * a - b - c, fy = 4.0 * b - a - c, fz = 4.0 * c - a - b;
  const double exy = 0.5 * (a + b), exz = 0.5 * (a + c), eyz = 0.5 * (b + c);
  double lg = 0.0;
  for (int dk = -1; dk <= 1; ++dk)
    for (int dj = -1; dj <= 1; ++dj)
      for (int di = -1; di <= 1; ++di) {
        const int ad = (di != 0) + (dj != 0) + (dk != 0);
        if (ad == 0 || ad == 3) continue;
        const int ii = i + di, jj = j + dj, kk = k + dk;
        if (!(ii == 0 || jj == 0 || kk == 0 || ii == nx || jj == ny || kk == nz)) continue;
        double w;
        if (ad == 1) w = di ? fx : (dj ? fy : fz);
        else w = (dk == 0) ? exy : ((dj == 0) ? exz : eyz);
        lg += w * rs.g[rs.gf.at(ii * s, jj * s, kk * s)];
      }
  return lg;
}

// The same as a call (kept out of line in the large sweep kernels, where it runs only for nodes next to the boundary).
__device__ __noinline__ inline double rhs_boundary_terms(const RhsSrc &rs, int nx, int ny, int nz, int i, int j,
                                                         int k) {
  return rhs_boundary_terms_inl(rs, nx, ny, nz, i, j, k);
}

// b at an interior node; rf (out): R f there (mode 0; the adjoint's G in mode 1)
template <bool kInline = false>
__device__ __forceinline__ double rhs_at(const RhsSrc &rs, int nx, int ny, int nz, int i, int j, int k, double &rf) {
  const int s = rs.s;
  auto F = [&](int di, int dj, int dk) { return rs.f[rs.gf.at((i + di) * s, (j + dj) * s, (k + dk) * s)]; };
  if (rs.mode == 1) {
    rf = F(0, 0, 0);
    return rf;
  }
  rf = 0.5 * (6.0 * F(0, 0, 0) + (F(1, 0, 0) + F(-1, 0, 0)) + (F(0, 1, 0) + F(0, -1, 0)) + (F(0, 0, 1) + F(0, 0, -1)));
  double lg = 0.0;
  if (i == 1 || j == 1 || k == 1 || i == nx - 1 || j == ny - 1 || k == nz - 1)
    lg = kInline ? rhs_boundary_terms_inl(rs, nx, ny, nz, i, j, k) : rhs_boundary_terms(rs, nx, ny, nz, i, j, k);
  return -rf + lg;
}
template <bool kInline = false>
__device__ __forceinline__ double rhs_at(const RhsSrc &rs, int nx, int ny, int nz, int i, int j, int k) {
  double rf;
  return rhs_at<kInline>(rs, nx, ny, nz, i, j, k, rf);
}
// the term a node adds to the squared norm of the stopping test: b^2, or (R f)^2 in the EXCMG_STOP_F_G reading
__device__ __forceinline__ double stop_norm_term(const RhsSrc &rs, double bv, double rf) {
  return rs.fg ? rf * rf : bv * bv;
}

// Device-resident CG state of one solve (one per problem in a batch).  Written only by the finalize kernels (and
// gbnd2 by boundary_g2_kernel).
struct CgState {
  double rho;      // r.r of the current residual
  double rho_old;  // r.r of the previous residual
  double pq;       // p.Mp of the current direction
  double alpha, beta;
  double bnorm2;   // ||b||^2 of the system being solved
  double stop2;    // stop when rho <= stop2 (= (tol ||b||)^2)
  double rho0;     // rho of the starting residual (the host predicts how many iterations remain from it)
  int iter;        // iterations completed
  int done;        // 1: converged or stopped; every CG kernel returns at once
  int status;      // 0 ok, EXCMG_ERR_NOCONV, EXCMG_ERR_BREAKDOWN
  int max_iters;
  int hist_on;     // record sqrt(rho / bnorm2) after each iteration into hist
  // Sweeps that finalize their own reductions (small and mid-size grids): pass A of iteration k reads iterA and
  // writes iterB = k, pass B reads iterB and writes iterA = k + 1, so no kernel writes a field its own workgroups
  // read; rhoA[k mod 2] holds r.r of iteration k; preset: iteration 0 takes rho and stop2 from this state (FP32
  // inner solves) instead of the residual's partial sums.
  int iterA, iterB;
  int preset;
  int pad_;
  double gbnd2;    // added to the squared norm of the stopping test: the sum of g^2 over the grid's boundary nodes
                   // under EXCMG_STOP_F_G, else 0 (set at setup and by boundary_g2_kernel)
  double rhoA[2];
  double alphaA[2];  // the single-reduction CG: alpha of iteration k in slot k mod 2
  double hist[EXCMG_MAX_HISTORY];
};

// ------------------------------------------------------------------------------------------------------------
// Launchers (defined in the .hip files).  All take the stream last.
// ------------------------------------------------------------------------------------------------------------

// A stencil sweep over one grid: layout, coefficients and the workgroup decomposition (64 x 4 column tiles, zc
// planes per workgroup; chosen by make_sweep).
struct Sweep {
  Grid g;
  Stencil st;
  int zc, ntx, nty, nzc;
  int depth;  // planes of loads in flight per thread in the z-march (2, 3, 4 or 6 in the CG passes; 2 or 3 in
              // the residual sweeps)
  int nt;     // 1: data read or written once per sweep uses non-temporal (streaming) loads and stores
  int ty;     // tile height in rows of 64 nodes (4, 8 or 16 in the CG passes; 4 in the residual sweeps)
};

// zc <= 0: default chunk; ty: 4 unless 8 or 16
Sweep make_sweep(const Grid &g, const Stencil &s, int zc, int depth = 2, int nt = 0, int ty = 4);
int sweep_blocks(const Sweep &sw);
// the same sweep with ty-row tiles, and with 4-row tiles (what the residual sweeps are built for)
Sweep with_height(const Sweep &sw, int ty);
Sweep default_height(const Sweep &sw);
// partial-sum buffer length needed by the CG and residual kernels for a grid
long long cg_partials_needed(const Grid &g);

// r = b - M u (interior of u only) on the level layout of sw, with b formed on the fly from the finest data (rs);
// initialises the CG state (rho, ||b||^2, stop test)
void launch_residual(const Sweep &sw, const double *u, const RhsSrc &rs, double *r, CgState *cs, double *partials,
                     double tol, int max_iters, int hist_on, hipStream_t st);
// FP32 inner step setup: r32 = (float)(b - M u), d32 = 0 (layout g32); sets the outer FP64 test and the inner state
// (bterm: FP64 scratch in the level layout for the boundary terms of b)
void launch_residual_cast(const Sweep &sw, const double *u, const RhsSrc &rs, double *bterm, const Grid &g32,
                          float *r32, float *d32, CgState *outer, CgState *inner, double *partials, double tol,
                          double eta, int outer_step, int max_outer, int max_inner, hipStream_t st);

// achievable-bandwidth probes over a caller buffer: copy of the first half into the second, and a read of the whole
void launch_probe_copy(const double *src, double *dst, long long n, hipStream_t st);
void launch_probe_read(const double *src, long long n, double *sink, hipStream_t st);
void launch_probe_copy_nt(const double *src, double *dst, long long n, hipStream_t st);
void launch_probe_read_nt(const double *src, long long n, double *sink, hipStream_t st);
void launch_probe_mix_nt(const double *a, double *b, double *c, long long n, hipStream_t st);
// the swept streaming kernels: mode 0 copy a -> b, 1 read a, 2 b += a/2 and c -= a/2, 3 write b; arrays of n doubles
void launch_probe_sweep(int mode, int u, bool nt, bool chunk, int wg_per_cu, const double *a, double *b, double *c,
                        long long n, double *sink, hipStream_t st);

// one CG iteration with the reductions finalized inside the sweeps: pass A reads nb_prev partial sums from partsB
// (the residual's [r.r | b.b] before iteration 0, pass B's r.r afterwards) and writes partsA; pass B reads nbA from
// partsA and writes partsB
template <typename T>
void launch_selfred_a(const Sweep &swA, T *r, T *p0, T *p1, CgState *cs, const double *partsB, int nb_prev,
                      double tol, double *partsA, hipStream_t st);
template <typename T>
void launch_selfred_b(const Sweep &swB, T *u, T *r, T *p0, T *p1, CgState *cs, const double *partsA,
                      int nbA, double *partsB, hipStream_t st);
// largest sweep (workgroups) that finalizes its own reductions
int selfred_max_blocks();
// the CG state before the first self-finalizing iteration (iterA = 0, not done, preset as given)
void launch_selfred_init(CgState *cs, int max_iters, int hist_on, int preset, hipStream_t st);
// cs->gbnd2 = the sum of g^2 over the boundary nodes of grid g (0 if rs.fg is 0 or rs.mode is 1); one workgroup
void launch_boundary_g2(const RhsSrc &rs, const Grid &g, CgState *cs, hipStream_t st);
// cs->gbnd2 = 0 for each state (at setup)
void launch_clear_gbnd2(CgState *a, CgState *b, hipStream_t st);
// residual sweep writing [r.r | b.b] partials without a finalize (for the self-finalizing iterations)
// The single-reduction CG of self-finalizing grids (kernels_cg.hip): the init sweep w = M r with the partial sums
// of r.r and w.r into parts, and iteration k (launch parity par) from r, w, s into ro, wo, so (u, p in place), from
// the partials of the previous launch (or the init's) and, at k = 0, the residual sweep's partsR (nbR workgroups);
// both use sweep sw (depth 2 or 3).
void launch_cg1_init(const Sweep &sw, const double *r, double *w, double *parts, hipStream_t st);
void launch_cg1_iteration(const Sweep &sw, double *u, double *p, const double *r, const double *w, const double *s,
                          double *ro, double *wo, double *so, CgState *cs, int par, const double *partsIn,
                          const double *partsR, int nbR, double tol, double *partsOut, hipStream_t st);
void launch_residual_partials(const Sweep &sw, const double *u, const RhsSrc &rs, double *r, double *parts,
                              hipStream_t st);

// one CG pass and its finalize kernel (a second, single-workgroup launch)
template <typename T>
void launch_cg_pass_a(const Sweep &sw, T *r, T *p0, T *p1, CgState *cs, double *partials, hipStream_t st);
template <typename T>
void launch_cg_pass_b(const Sweep &sw, T *u, T *r, T *p0, T *p1, CgState *cs, double *partials,
                      hipStream_t st);

// CG state for timing sweeps in isolation: iteration 0, alpha = beta = 0, never done
void launch_tune_state(CgState *cs, int iter, hipStream_t st);  // at iteration iter (0 or 1)
// the trial state of the self-finalizing passes in cs, and parts[0, n) = 1 (n <= the self-finalizing limit)
void launch_tune_selfred(CgState *cs, double *parts, int n, hipStream_t st);
// a single-wave kernel that returns after about `us` microseconds (bounded), to queue launches behind it
void launch_delay(double us, hipStream_t st);
// copy bytes (a multiple of 8) from device memory to host memory mapped for the device
void launch_publish(const void *src, void *dst, size_t bytes, hipStream_t st);

// u += (double) d32 on the interior
void launch_add_correction(const Grid &gu, double *u, const Grid &g32, const float *d32, hipStream_t st);

// single-workgroup CG on a small grid: exact = 1 to rounding (DSOLVE), exact = 0 to tol (relaxation); work arrays
// r, p, q on grid gw
void launch_small_cg(const Grid &gu, double *u, const RhsSrc &rs, const Grid &gw, double *r, double *p, double *q,
                     const Stencil &s, CgState *cs, double tol, int max_iters, int exact, int hist_on,
                     hipStream_t st);

// y = M x (interior of x only), y = 0 on the boundary
void launch_apply(const Grid &gx, const double *x, const Grid &gy, double *y, const Stencil &s, hipStream_t st);

// level data b (layout gb) on the interior, from rhs_at
void launch_rhs(const RhsSrc &rs, const Grid &gb, double *b, hipStream_t st);
// boundary nodes of u <- g (finest dense g sampled at stride s); interior set to 0 if zero_interior
void launch_set_boundary(const Grid &gg, const double *g, int stride, const Grid &gu, double *u, int zero_interior,
                         hipStream_t st);
// w on grid gw from u2 (grid g2, n/2) and u4 (grid g4, n/4); boundary from dense finest g at stride s
// Initial guess of a grid from the two coarser solutions: kGuessQuartic = EXP_finite (the paper's), kGuessQuadratic =
// the same extrapolation with tri-quadratic interpolation, kGuessLinear = trilinear interpolation of u2 alone.
enum GuessKind { kGuessQuartic = 0, kGuessQuadratic = 1, kGuessLinear = 2 };
void launch_initial_guess(int kind, const Grid &g2, const double *u2, const Grid &g4, const double *u4,
                          const Grid &gg, const double *g, int stride, const Grid &gw, double *w, hipStream_t st);
// ut (grid gt) = EXP_true(uh (grid gh), u2 (grid g2))
void launch_exp_true(const Grid &gh, const double *uh, const Grid &g2, const double *u2, const Grid &gt, double *ut,
                     double *ucopy, hipStream_t st);
// copy between layouts (same n)
void launch_copy(const Grid &gs, const double *src, const Grid &gd, double *dst, hipStream_t st);
// count of non-finite values in a dense array -> *flag (device int, must be zeroed by the caller)
void launch_check_finite(const double *a, long long n, int *flag, hipStream_t st);

// ------------------------------------------------------------------------------------------------------------
// Batched solves.  One table per cascade step holds an entry for every problem of the batch on that step.  Launches
// over several problems are flattened: launch kind K gives entry e the workgroups [pre[K][e], pre[K][e+1]) (zero
// for entries the launch does not concern) and a workgroup finds its entry by binary search on pre[K].  Launches with
// one workgroup per entry (reductions, small-grid CG) use blockIdx.x as the entry index.  Every problem keeps its own
// arrays, partial sums and CG states in its own workspace, so the problems of one launch share nothing.
// ------------------------------------------------------------------------------------------------------------
enum BatchKind { kBSmall = 0, kBCg64 = 1, kBIr = 2, kBNone = 3 };
enum BatchLaunch {
  kLA64 = 0, kLB64, kLR64,   // FP64 CG passes and residual (kind kBCg64)
  kLA32, kLB32, kLRC,        // FP32 inner passes and FP64 residual + cast (kind kBIr)
  kLExp,                     // EXP_finite (grids >= 2)
  kLSetB,                    // boundary values and zero interior (grids 0, 1)
  kLCopy,                    // copy of the finest grid to the caller's dense array
  kLCorr,                    // u += d (kind kBIr)
  kLBterm,                   // boundary terms of the right-hand side (kinds kBCg64 and kBIr)
  kLaunchKinds
};

struct BatchMirror {  // copy of one CG state's scalars, for the host
  int done, iter, status, pad;
  double rho, bnorm2, rho0, stop2;
};

struct BatchStatus {
  BatchMirror m[2];  // [0]: the FP64 CG (or, under refinement, the outer loop); [1]: the FP32 inner solve
  long long t_done;  // wall_clock64() when the problem's finest grid finished, 0 before
  long long pad;
};

struct BatchEntry {
  int kind;       // BatchKind
  int problem;    // index into the status array
  int finest;     // this grid is the problem's finest
  int exact;      // kBSmall: 1 = direct solve (grids 0, 1), 0 = relaxation to tol
  int level;      // grid index in the problem's cascade
  int cap;        // CG iteration cap (kBIr: per inner solve)
  int max_outer;  // kBIr: outer refinement steps allowed
  int pad;
  double tol, eta;
  Sweep swA, swB, swR, swA32, swB32;
  Grid g, g32, gd, g2, g4;  // this grid (FP64, FP32 layouts), the problem's dense node layout, grids l-1 and l-2
  Stencil st;
  RhsSrc rs;                // level data from the problem's finest f, g
  double *u, *r, *p0, *p1;  // u: this grid's solution; r, p0, p1: the problem's work vectors
  float *r32, *p32a, *p32b, *d32;
  CgState *cs, *cs2;
  double *parts;
  const double *u2, *u4;    // solutions of grids l-1 and l-2 (EXP_finite)
  const double *gb;         // the problem's finest g (boundary values)
  double *out;              // the caller's u (finest grid)
};

// ---- batched launches ----
// A list of entries for one launch: ent[0..n) point into the device tables; flattened launches give entry e the
// workgroups [pre[e], pre[e+1]) (total = pre[n] workgroups); aux[e] is a per-entry argument (the refinement's outer
// step for the residual-and-cast launch).  Launches with one workgroup per entry use n workgroups.
struct BatchList {
  const BatchEntry *const *ent;
  const int *pre;
  const int *aux;
  int n;
  int total;
};

void launch_b_init(BatchStatus *stat, int count, long long *t0, hipStream_t st);
void launch_b_set_boundary(const BatchList &L, hipStream_t st);
void launch_b_exp_finite(const BatchList &L, hipStream_t st);
void launch_b_small_cg(const BatchList &L, int lds_nodes, BatchStatus *stat, hipStream_t st);
int b_small_lds_nodes(const Grid &g);  // LDS (doubles) the small-grid CG of this grid uses, 0 if it does not fit
void launch_b_boundary_terms(const BatchList &L, hipStream_t st);
void launch_b_residual(const BatchList &L, BatchStatus *stat, hipStream_t st);       // + the reduction
void launch_b_residual_cast(const BatchList &L, BatchStatus *stat, hipStream_t st);  // + the reduction
// one CG iteration (pass A, its reduction, pass B, its reduction) of the entries of A and B (the same entries, with the
// workgroup prefixes of pass A and pass B); fp32: the inner FP32 solves of the refinement; ty: the tile height every
// entry's pass sweeps use; depth: their prefetch depth (2, 3, 4 or 6)
void launch_b_iteration(int fp32, int ty, int depth, const BatchList &A, const BatchList &B, BatchStatus *stat,
                        hipStream_t st);
void launch_b_add_correction(const BatchList &L, hipStream_t st);
// the autotuner's trial CG state in every entry of L, and the two passes alone (timed by the batched autotuner)
void launch_b_tune_state(const BatchList &L, hipStream_t st);
void launch_b_passes(int fp32, int ty, int depth, const BatchList &A, const BatchList &B, hipStream_t st);
void launch_b_copy(const BatchList &L, hipStream_t st);
// workgroup counts of the flattened launches for one grid
int b_blocks_exp_finite(const Grid &gw);
int b_blocks_nodes(const Grid &g);     // set_boundary and copy
int b_blocks_interior(const Grid &g);  // add_correction
int b_blocks_bterms(const Grid &g);    // boundary terms

// gradient of a grid function (layout gu) into dense outputs (layout gd); table: 1/m_i for N up to nmax
void launch_gradient(const Grid &gu, const double *u, const Grid &gd, double *ux, double *uy, double *uz, double hx,
                     double hy, double hz, const double *inv_m_x, const double *inv_m_y, const double *inv_m_z,
                     hipStream_t st);

// adjoint transposes: dLdf = -R^T lam (all nodes); dLdg = A_IB^T lam + G (boundary), 0 inside
void launch_adjoint_transposes(const Grid &gl, const double *lam, const Grid &gd, const double *G, double *dLdf,
                               double *dLdg, double hx, double hy, double hz, hipStream_t st);

}  // namespace excmg
