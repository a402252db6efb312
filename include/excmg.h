/*
 * excmg.h -- C ABI of the MI355X (gfx950) EXCMG solver for the 3D Dirichlet Poisson problem
 *
 *     u_xx + u_yy + u_zz = f in the box [0,Lx]x[0,Ly]x[0,Lz],   u = g on its boundary
 *
 * (Pan, He & Hu, arXiv 1507.05063: problem statement eq. (bvp), Section 1; grid and unequal meshsizes,
 * Section 2), discretised by the 19-point fourth-order compact scheme (eq. compact) and solved by the
 * extrapolation cascadic multigrid method of Algorithm 1: direct solves on the two coarsest grids, then on every
 * finer grid an initial guess from Richardson extrapolation plus tri-quartic Lagrange interpolation of the two
 * previous solutions (Sections 4.2-4.3), relaxed by conjugate gradients until the relative residual
 * ||A_h u_h - f_h||_2 <= tol ||f_h||_2 (Algorithm 1, loop over the levels).
 *
 * Conventions for every entry point
 *   - Node arrays: (Nz+1)*(Ny+1)*(Nx+1) contiguous doubles, x fastest: node (i,j,k) is at ((k*(Ny+1))+j)*(Nx+1)+i,
 *     coordinates (i*hx, j*hy, k*hz), hx = Lx/Nx (Section 2).  All array arguments are DEVICE pointers to memory on
 *     the device that was current at excmg_setup, unless a comment says "host".
 *   - Ownership: the caller owns every array and the workspace; the library allocates no device memory.  The handle
 *     owns only host-side state; excmg_destroy frees it.
 *   - Streams: all device work is enqueued on the stream given at setup.  Calls that report iteration counts wait
 *     for their own work on that stream before returning; their outputs are complete when they return.
 *   - Errors: every int-returning call returns EXCMG_OK (0) or a negative EXCMG_ERR_* code; excmg_strerror names it.
 *     No exception crosses the ABI.  On EXCMG_ERR_NOCONV the outputs hold the last iterate and the stats are filled.
 *   - Calls on one handle must not overlap (one stream, one workspace).  Different handles are independent.
 */
#ifndef EXCMG_H
#define EXCMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EXCMG_OK 0
#define EXCMG_ERR_ARG (-1)       /* null pointer, non-positive box edge or tolerance, bad precision or flags */
#define EXCMG_ERR_SHAPE (-2)     /* cell counts are not n_coarse * 2^L, odd coarsest counts, too many levels,
                                    fewer than 4 cells on an axis for the gradient */
#define EXCMG_ERR_NONFINITE (-3) /* f or g holds a NaN or an infinity */
#define EXCMG_ERR_NOCONV (-4)    /* a level reached max_iters before the tolerance */
#define EXCMG_ERR_BREAKDOWN (-5) /* CG met p.Ap <= 0 or a non-finite scalar */
#define EXCMG_ERR_HIP (-6)       /* a HIP runtime call failed */
#define EXCMG_ERR_WORKSPACE (-7) /* workspace null, too small or misaligned (256-byte alignment required) */
#define EXCMG_ERR_SCRATCH (-8)   /* excmg_solve_noalloc: the problem needs more than the library's fixed scratch
                                    array (EXCMG_NOALLOC_MAX_BYTES) */

#define EXCMG_FP64 0    /* CG in FP64 */
#define EXCMG_FP32_IR 1 /* CG sweeps in FP32 inside FP64 iterative refinement on every grid with at least 2^20
                           interior unknowns (smaller grids are latency-bound and relax in FP64) */

#define EXCMG_WANT_HISTORY 1u /* record the finest level's relative-residual history (stats.history) */
#define EXCMG_WANT_TIMING 2u  /* time every kernel of the finest grid with HIP events (stats.kernel_ms,
                                 kernel_calls); the coarser grids are not timed */
#define EXCMG_NO_GRAPHS 4u    /* launch every CG iteration directly instead of replaying graphs of iteration batches on
                                 the grids below the finest (same kernels in the same order: same results) */
/* The initial guesses the paper compares its own with (at most one of the two; neither = EXP_finite, Algorithm 1):
 * on every grid from the third on, the CG starts from */
#define EXCMG_GUESS_QUADRATIC 8u /* the extrapolation of EXP_finite at the 2h nodes, then tri-quadratic Lagrange
                                    interpolation on cells of 2x2x2 2h elements (the earlier EXCMG's interpolation,
                                    which the remark after eq. (inter) in Section 4.3 finds too weak here) */
#define EXCMG_GUESS_LINEAR 16u   /* trilinear interpolation of u_2h, no extrapolation (the CMG method, Section 3) */
/* The norm ||f_h|| of the stopping test (Algorithm 1).  Default: f_h is the right-hand side b of the eliminated
 * system, the vector the CG's residual is measured against.  With this flag f_h is the vector of the discrete
 * equations before elimination: R f at the interior nodes and the Dirichlet value g at the boundary nodes (the same
 * test with a larger ||f_h|| on fine grids, so more CG iterations; the finer-grid errors the paper prints for its
 * Tables 1-12 follow this reading, its iteration counts the default one). */
#define EXCMG_STOP_F_G 32u
/* A third reading of the same test: the norm of (R f inside, g on the boundary) on every grid below the finest, and of
 * the eliminated right-hand side b on the finest grid (so the grids that feed the extrapolation are relaxed to the
 * tighter test, and the finest grid stops after the few iterations the default reading needs).  With it, one cascade
 * reproduces both the paper's printed finest-grid errors (Tables 1-12, read as the grids of one run) and its printed
 * finest-grid iteration counts.  At most one of EXCMG_STOP_F_G and this flag. */
#define EXCMG_STOP_F_G_BELOW_FINEST 64u
/* CG form on the small grids below the finest (at most 2^18 unknowns, from the third grid on) whose iterations
 * finalize their own reductions.  Default:
 * the single-reduction form of Chronopoulos and Gear, the same Krylov iterates as Algorithm 1's CG in exact
 * arithmetic (so the same iteration counts up to rounding), with both inner products of an iteration from one
 * reduction, which makes an iteration one kernel launch instead of two; it keeps s = M p and w = M r and moves 80
 * bytes per unknown and iteration instead of 64.  With this flag every grid runs the two-pass CG as written. */
#define EXCMG_TWO_PASS_CG 256u

#define EXCMG_MAX_LEVELS 16
#define EXCMG_MAX_HISTORY 256

/* Kernel classes reported by EXCMG_WANT_TIMING. */
#define EXCMG_K_CG_A 0      /* p = r + beta p; partial sums of p.Mp                          (FP64) */
#define EXCMG_K_CG_B 1      /* u += alpha p; r -= alpha Mp; partial sums of r.r              (FP64) */
#define EXCMG_K_CG_A32 2    /* the same two passes in FP32 (inner solves of EXCMG_FP32_IR) */
#define EXCMG_K_CG_B32 3
#define EXCMG_K_RESID 4     /* r = b - M u (+ cast for the FP32 inner solve), partial sums */
#define EXCMG_K_FINALIZE 5  /* fixed-order reduction of block partials, CG scalars */
#define EXCMG_K_RHS 6       /* right-hand side assembly (excmg_op_rhs; the solver forms b inside its kernels) */
#define EXCMG_K_EXP_FINITE 7
#define EXCMG_K_EXP_TRUE 8
#define EXCMG_K_DSOLVE 9     /* single-workgroup kernels: the direct solves, and the CG of grids <= 8000 unknowns */
#define EXCMG_K_GRADIENT 10
#define EXCMG_K_OTHER 11
#define EXCMG_K_CG_A0 12     /* the FP64 passes of a grid's first CG iteration, where p = r: pass A reads r and */
#define EXCMG_K_CG_B0 13     /* writes no p, pass B reads r once for both operands (EXCMG_K_CG_A/B: the others) */
#define EXCMG_K_CLASSES 14

typedef struct excmg_handle excmg_handle;

/* Problem description (paper, Section 2 and Algorithm 1). */
typedef struct {
  double box[3];        /* Lx, Ly, Lz > 0 */
  int32_t n[3];         /* Nx, Ny, Nz: cells per axis on the finest grid */
  int32_t n_coarse[3];  /* cells per axis on the coarsest grid H; {0,0,0} = automatic: halve the finest counts
                           while the halves are all even and >= 2 and the largest half is >= 4 */
  double tol;           /* relative-residual tolerance epsilon of Algorithm 1, on every level (see tol_order), > 0 */
  int32_t precision;    /* EXCMG_FP64 or EXCMG_FP32_IR */
  double inner_tol;     /* FP32_IR: largest residual reduction asked of one inner FP32 solve (0 = 1e-5); an inner
                           solve also stops once its residual is half the outer target tol*||f_h|| */
  int32_t max_iters;    /* CG iterations allowed per level (FP32_IR: inner iterations per outer step); 0 = 10000 */
  uint32_t flags;       /* EXCMG_WANT_* */
  double tol_order;     /* level-dependent tolerance (not in the paper, which uses one tol on every grid and notes
                           that the extrapolated solution then loses its sixth order on fine grids, Section 5.1):
                           0 = tol on every grid; p > 0: grid l of L (coarsest 0) relaxes to
                           tol * 2^(p (L-1-l)), at most max(tol, 1e-2), so tol holds on the finest grid and each
                           coarser grid's algebraic error keeps the ratio to h^p of the finest's.  p = 6 with
                           EXCMG_STOP_F_G (whose ||f_h|| / sqrt(unknowns) does not grow as h falls) keeps the
                           algebraic error of every grid proportional to the sixth-order truncation error.  0 <= p
                           <= 16 */
  double tol_coarse;    /* 0 = as above; > 0 (and < 1, with tol_order 0): every grid below the finest relaxes to
                           tol_coarse and the finest to tol (the paper gives one epsilon for all grids; this reading
                           of Algorithm 1's stopping test, tol_coarse = tol / 100, reproduces the anisotropic example's
                           two finest meshes in Section 5).  Errors: EXCMG_ERR_ARG outside that range */
} excmg_problem;

/* Statistics of one call (host struct, filled by the library). */
typedef struct {
  int32_t levels;                            /* number of grids, coarsest first */
  int32_t n[EXCMG_MAX_LEVELS][3];            /* cells per axis of each grid */
  int32_t iters[EXCMG_MAX_LEVELS];           /* CG iterations per grid (FP32_IR: inner iterations summed);
                                                0 on the two directly solved grids */
  int32_t ir_outer[EXCMG_MAX_LEVELS];        /* FP32_IR: outer refinement steps per grid */
  int32_t dsolve_iters[2];                   /* the two coarsest grids are solved exactly: by sine transforms
                                                (0 here) up to 64 cells per axis, else by CG to a relative
                                                residual of 1e-15 (its iteration count here) */
  double relres[EXCMG_MAX_LEVELS];           /* relative residual at exit per grid (FP64: recursive CG residual;
                                                FP32_IR: the FP64 outer residual) */
  double ms_level[EXCMG_MAX_LEVELS];         /* wall time of each grid's work (transfer + relaxation), ms */
  double ms_total;                           /* wall time of the call, ms */
  double kernel_ms[EXCMG_K_CLASSES];         /* EXCMG_WANT_TIMING: summed kernel time per class on the finest
                                                grid, ms (CG launches made after it converged are not counted) */
  int32_t kernel_calls[EXCMG_K_CLASSES];     /* EXCMG_WANT_TIMING: launches per class */
  double kernel_ms_finest[EXCMG_K_CLASSES];  /* the same, finest grid only */
  int32_t kernel_calls_finest[EXCMG_K_CLASSES];
  int32_t history_len;                       /* EXCMG_WANT_HISTORY: entries in history */
  double history[EXCMG_MAX_HISTORY];         /* finest grid: relative residual before iteration 1, after 1, ... */
} excmg_stats;

/* Host only.  Bytes of device workspace excmg_setup needs for this problem. */
int excmg_workspace_bytes(const excmg_problem *p, size_t *bytes);

/* Host only.  The level plan: *levels grids, the coarsest with n_coarse_out[3] cells (rule of n_coarse). */
int excmg_plan(const excmg_problem *p, int32_t *levels, int32_t n_coarse_out[3]);

/* Bind a problem to a workspace (device memory of at least excmg_workspace_bytes, 256-byte aligned, owned by the
 * caller and not touched by anything else while the handle lives) and a HIP stream (hipStream_t, may be NULL for
 * the null stream).  Allocates only the host-side handle. */
int excmg_setup(const excmg_problem *p, void *workspace, size_t bytes, void *hip_stream, excmg_handle **h);

/* Algorithm 1.  f: node array (every node is read); g: node array (only boundary nodes are read).
 * u (out): node array, the finest-grid solution with its boundary equal to g.
 * u_ext (out, nullable): EXP_true(u_h, u_2h), the sixth-order extrapolated solution on the finest grid
 * (Algorithm 1, optional step; Sections 4.2.1 and 4.3); needs at least two grids.
 * stats (host, nullable). */
int excmg_solve(excmg_handle *h, const double *f, const double *g, double *u, double *u_ext, excmg_stats *stats);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): excmg_solve for the problem p without a handle or a caller workspace.  Its workspace is a
 * fixed device array inside the library, EXCMG_NOALLOC_MAX_BYTES bytes, one per GPU the library is loaded on, held
 * until the process ends; problems whose excmg_workspace_bytes exceeds it are rejected with EXCMG_ERR_SCRATCH before
 * any device work.  The call allocates no device or pinned host memory and creates no HIP event, stream or graph: it
 * launches kernels on hip_stream (hipStream_t, may be NULL) of the current device and reads the CG states back with
 * stream copies, waiting for the stream before it returns, as excmg_solve does.  f, g, u, u_ext, stats: as for
 * excmg_solve (same kernels and results as a handle set up for p without autotuning; EXCMG_WANT_TIMING is ignored
 * and every iteration is launched directly).  All calls on one GPU share the array, which keeps the last call's
 * contents: calls that overlap on one GPU (other host threads, other streams) race and must be serialised by the
 * caller.  Errors: as excmg_solve, plus EXCMG_ERR_ARG for a null p, f, g or u, EXCMG_ERR_SHAPE for a bad plan, and
 * EXCMG_ERR_HIP if the array's device address cannot be looked up. */
#define EXCMG_NOALLOC_MAX_BYTES ((size_t)128 << 20)
int excmg_solve_noalloc(const excmg_problem *p, const double *f, const double *g, double *u, double *u_ext,
                        void *hip_stream, excmg_stats *stats);

/* Fourth-order compact gradient of a finest-grid node array u (Section 5.1): one-sided fourth-order formulas at both
 * ends of every grid line, tridiagonal (1,4,1)/6 systems inside solved by the Thomas algorithm.  ux, uy, uz (out):
 * node arrays.  Needs at least 4 cells per axis. */
int excmg_gradient(excmg_handle *h, const double *u, double *ux, double *uy, double *uz);

/* Adjoint of the discrete solution map (f, g) -> u (interior: the compact-scheme solution; boundary: g) for an
 * upstream gradient G = dL/du (node array).  Solves M lambda = G_I (M = -A_h restricted to the interior, the same
 * symmetric operator) by the same cascade with the level data taken from G, then
 *   dLdf = -R^T lambda on every node (R f = (6 f_c + sum of the 6 face neighbours)/2, eq. compact),
 *   dLdg = A_IB^T lambda + G on boundary nodes, 0 inside.
 * lambda_out (nullable): lambda as a node array with zero boundary.  Uses the handle's tolerance and precision. */
int excmg_adjoint(excmg_handle *h, const double *G, double *dLdf, double *dLdg, double *lambda_out,
                  excmg_stats *stats);

/* Host only.  Bytes of device workspace excmg_solve_batched needs for a batch of count problems (the per-step
 * problem tables and the per-problem status words; about 20 KB per problem). */
int excmg_batch_workspace_bytes(int32_t count, size_t *bytes);

/* Many independent problems at once (Algorithm 1 for each): handles hs[0..count-1], each with its own workspace,
 * all set up on the same device; problem b reads f[b], g[b] and writes u[b] (node arrays of its own shape, as for
 * excmg_solve).  All work is enqueued on the stream of hs[0]; work the caller has queued for the other handles on
 * other streams must be complete.  The cascades run in step, grid s of every problem in step s: each kernel launch
 * covers every problem it concerns (the workgroups of one launch are split among the problems), so a batch costs
 * about as many launches as its largest problem.  Each problem keeps its own precision, tolerance and iteration
 * limits; the history and timing flags are ignored.  Handles set up with an EXCMG_GUESS_* flag, EXCMG_STOP_F_G or
 * EXCMG_STOP_F_G_BELOW_FINEST are rejected (EXCMG_ERR_ARG): batched solves start every grid from EXP_finite and take
 * the default stopping norm.
 * batch_ws: device memory of at least excmg_batch_workspace_bytes(count), 256-byte aligned, owned by the caller.
 * stats (host, nullable): count entries (ms_total = the host time of the whole call).  ms_per_problem (host,
 * nullable): count entries, the device time from the start of the batch until problem b's finest grid converged.
 * Returns the first error met (the batch stops), else EXCMG_ERR_NOCONV if a problem hit its iteration limit, else
 * EXCMG_OK. */
int excmg_solve_batched(excmg_handle *const *hs, int32_t count, const double *const *f, const double *const *g,
                        double *const *u, void *batch_ws, size_t batch_bytes, excmg_stats *stats,
                        double *ms_per_problem);

/* Host only.  Batched solves run the CG iterations of each round as a graph: replayed from a cache on the batch's
 * first handle when a round has the launch shape of an earlier one (the same batch workspace, iteration counts and,
 * per launch, numbers of problems and workgroups; which problems a launch covers is read from the workspace when it
 * runs), else captured and instantiated (1024 are kept, the least recently used dropped first; EXCMG_NO_GRAPHS on
 * that handle launches them directly).  replays, captures (host): the graphs replayed and captured on h so far. */
int excmg_batch_graph_counts(const excmg_handle *h, int64_t *replays, int64_t *captures);

/* Autotuner of excmg_solve_batched for a batch of handles (host call, device work on the stream of hs[0]; the same
 * conditions on the handles as excmg_solve_batched).  In a batched launch the workgroups of all the problems concerned
 * run together, so the z chunk a problem prefers alone is not the one the batch prefers.  For each grid counted from
 * the problems' finest (t = 0 each problem's finest grid, t = 1 the next coarser, ...) and each precision, every z
 * chunk in {2, 4, ..., 128} planes is timed as one flattened launch of the two CG passes over all problems whose grid
 * t relaxes in that precision, at each tile height (4, 8, 16 rows) and prefetch depth (2, 3, 4, 6 planes); a batched
 * launch holds all the batch's grids, so one height and depth are chosen per precision (those whose fastest chunks
 * sum to the least time), and the chunks, height and depth are kept in those problems' handles (replacing what
 * excmg_autotune chose there; results do not depend on them; excmg_get_sweep and excmg_get_batch_shape read them).
 * Trial launches touch only the handles' work buffers and CG states.
 * batch_ws: as for excmg_solve_batched.  zc_out (host, nullable, 2 * EXCMG_MAX_LEVELS entries): zc_out[2 t + p] the
 * chunk chosen for grid t in precision p (0 FP64, 1 FP32), 0 where no problem relaxes that grid that way. */
int excmg_autotune_batched(excmg_handle *const *hs, int32_t count, void *batch_ws, size_t batch_bytes,
                           int32_t *zc_out);

/* Autotuner (host call, device work on the handle's stream): times the two CG sweep kernels of every relaxed grid
 * (FP64, and FP32 where EXCMG_FP32_IR relaxes in FP32) for each z-chunk length in {2, 4, ..., 512} planes per
 * workgroup, each tile height (4, 8 or 16 rows of 64 nodes per workgroup), each prefetch depth (2, 3, 4 or 6 planes
 * of loads in flight per thread) and each cache policy (ordinary or non-temporal loads and stores of the data a
 * sweep touches once), on the handle's own work buffers (no caller array is read or written), and keeps the fastest
 * per grid and kernel for every later call on this handle.  Grids below the finest, whose iterations run as graphs
 * of self-finalizing passes, are timed on those kernels, with the shapes that keep them self-finalizing; on those
 * that run the single-reduction CG (see EXCMG_TWO_PASS_CG) the pass-B shape, which that CG uses, is timed on its
 * iterations.
 * zc_out, depth_out (host, nullable, 4 * levels entries each): per grid, pass A and pass B in FP64, then in FP32 (0
 * where the grid is not relaxed that way): the chunk, and depth + 10 (if the non-temporal policy won) + 100 * tile
 * height.  Batched solves (excmg_solve_batched) keep the chunk and use the handle's batch shape
 * (excmg_get_batch_shape; excmg_autotune_batched chooses it).
 * Optional: without it the handle uses a fixed default (16 planes, fewer on small grids; 4 rows; depth 2;
 * ordinary). */
int excmg_autotune(excmg_handle *h, int32_t *zc_out, int32_t *depth_out);

/* Sweep shapes (host calls).  A sweep of grid `level` (0 = coarsest) of kind EXCMG_SWEEP_*: the CG passes A and B in
 * FP64, in FP32 (EXCMG_FP32_IR), and the FP64 passes of a grid's first iteration (used on grids whose passes do not
 * finalize their own reductions).  shape[4] (host) = {z chunk in planes (even, 2..4096), prefetch depth (2, 3, 4 or
 * 6), non-temporal policy (0 or 1), tile height in rows of 64 nodes (4, 8 or 16)}.  excmg_get_sweep reads the shape
 * in use (the setup's default or the autotuner's choice); excmg_set_sweep replaces it for every later call on this
 * handle (so that a shape found by excmg_autotune can be saved and restored without tuning again, or a shape
 * forced), after waiting for the handle's stream, and drops the handle's captured iteration graphs.  Results depend
 * on the shape only through the order of the partial sums (rounding).  Errors: EXCMG_ERR_ARG for a null handle or
 * shape, a level or kind out of range, a value outside the sets above, or a shape with more workgroups than the
 * handle's partial-sum buffer holds (chunks of 2 planes at 4 rows always fit); EXCMG_ERR_HIP. */
#define EXCMG_SWEEP_A 0
#define EXCMG_SWEEP_B 1
#define EXCMG_SWEEP_A32 2
#define EXCMG_SWEEP_B32 3
#define EXCMG_SWEEP_A_FIRST 4
#define EXCMG_SWEEP_B_FIRST 5
int excmg_get_sweep(excmg_handle *h, int32_t level, int32_t kind, int32_t shape[4]);
int excmg_set_sweep(excmg_handle *h, int32_t level, int32_t kind, const int32_t shape[4]);

/* Shape of the batched CG passes of the batches this handle leads (hs[0] of excmg_solve_batched), shape[4] (host) =
 * {tile height of the FP64 passes, of the FP32 passes (4, 8 or 16 rows), prefetch depth of the FP64 passes, of the
 * FP32 passes (2, 3, 4 or 6 planes)}; {4, 4, 2, 2} until excmg_autotune_batched chooses.  Every grid of a batched launch
 * uses it; a grid's z chunk comes from its own handle.  Set waits for the handle's stream and drops its captured
 * graphs.  Errors: EXCMG_ERR_ARG for a null handle or array or a value outside those sets. */
int excmg_get_batch_shape(excmg_handle *h, int32_t shape[4]);
int excmg_set_batch_shape(excmg_handle *h, const int32_t shape[4]);

/* Host call.  Turns the kernel timing of EXCMG_WANT_TIMING on (on != 0) or off for later calls on this handle, as
 * if the flag had been given at setup (the timing events are created the first time it is turned on).  The solver's
 * results do not depend on it; the timing only adds event records between the finest grid's launches.  Waits for the
 * handle's stream first.  Errors: EXCMG_ERR_ARG for a null handle, EXCMG_ERR_HIP if the events cannot be created. */
int excmg_set_timing(excmg_handle *h, int32_t on);

void excmg_destroy(excmg_handle *h);
const char *excmg_strerror(int code);

/* Kinds of the bandwidth probe, in the order of its rates. */
enum {
  EXCMG_PROBE_COPY = 0,    /* first half of buf into the second half, ordinary loads and stores */
  EXCMG_PROBE_READ = 1,    /* all of buf read, ordinary loads */
  EXCMG_PROBE_COPY_NT = 2, /* the copy with non-temporal loads and stores */
  EXCMG_PROBE_READ_NT = 3, /* the read with non-temporal loads */
  EXCMG_PROBE_MIX_NT = 4,  /* buf as three arrays a, b, c: b += a/2, c -= a/2, non-temporal (pass B's 3 reads, 2 writes) */
  EXCMG_PROBE_MIX = 5,     /* the same mix with ordinary loads and stores */
  EXCMG_PROBE_WRITE = 6,   /* all of buf written, ordinary stores */
  EXCMG_PROBE_WRITE_NT = 7, /* the write with non-temporal stores */
  EXCMG_PROBE_KINDS = 8
};

/* Same-run bandwidth ceilings for the roofline: for each kind above, the best rate over a sweep of launch shapes --
 * 2 to 64 workgroups of 256 threads per compute unit, 2, 4 or 8 independent 16-byte accesses in flight per lane, and
 * two patterns (grid-stride loops; or each workgroup streaming through one contiguous range, as a stencil sweep's
 * workgroup does) -- each run reps times after one warm-up pass, plus, for kinds 0-4, one fixed-shape kernel (8 or 32
 * workgroups per CU, 4 accesses per lane, grid-stride; the copy of this one calibrates the hardware traffic
 * counters).  GBs[kind] = bytes read plus bytes written / the fastest launch, in GB/s.  buf: device, at least 4096
 * bytes, 16-byte aligned; its contents are overwritten.  GBs: host, EXCMG_PROBE_KINDS entries.  shapes (host,
 * nullable, 3 * EXCMG_PROBE_KINDS entries): per kind, the fastest launch's workgroups per CU, accesses in flight per
 * lane and pattern (1 = contiguous ranges).  Errors: EXCMG_ERR_ARG for a null or misaligned pointer, too few bytes
 * or reps <= 0. */
int excmg_bandwidth_probe(void *buf, size_t bytes, int32_t reps, void *hip_stream, double *GBs, int32_t *shapes);

/* ---- single steps of the path, on one grid of cells n = (Nx,Ny,Nz) and box (node arrays as above) ---- */

/* y = M x with M = -A_h on the interior (eq. compact, left-hand side, negated; boundary entries of x are read as 0);
 * y is 0 on boundary nodes. */
int excmg_op_apply(const int32_t n[3], const double box[3], const double *x, double *y, void *hip_stream);

/* b = -R f + A_IB g on interior nodes (eq. compact with the Dirichlet values moved to the right), 0 on boundary. */
int excmg_op_rhs(const int32_t n[3], const double box[3], const double *f, const double *g, double *b,
                 void *hip_stream);

/* EXP_finite(u_2h, u_4h) (Sections 4.2.2 and 4.3): w on the grid n (multiples of 8) from u2h (n/2) and u4h (n/4);
 * boundary nodes of w are g. */
int excmg_op_exp_finite(const int32_t n[3], const double *u2h, const double *u4h, const double *g, double *w,
                        void *hip_stream);

/* The initial guess of a kind: 0 = EXP_finite (as excmg_op_exp_finite), 1 = tri-quadratic after the same
 * extrapolation, 2 = trilinear interpolation of u2h (u4h not read, may be NULL); see EXCMG_GUESS_*.  n: multiples of 8
 * for kinds 0 and 1, even for kind 2.  Errors: EXCMG_ERR_ARG for an unknown kind or a null pointer,
 * EXCMG_ERR_SHAPE for counts that do not fit. */
int excmg_op_initial_guess(int32_t kind, const int32_t n[3], const double *u2h, const double *u4h, const double *g,
                           double *w, void *hip_stream);

/* EXP_true(u_h, u_2h) (eqs. t1, chenlin; Section 4.3) on the grid n (even counts). */
int excmg_op_exp_true(const int32_t n[3], const double *uh, const double *u2h, double *ut, void *hip_stream);

#ifdef __cplusplus
}
#endif
#endif
