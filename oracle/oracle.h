/*
 * Plain FP64 CPU oracle for the EXCMG method with the 19-point fourth-order compact scheme
 * (Pan, He & Hu, "An extrapolation cascadic multigrid method combined with a fourth-order compact scheme
 * for 3D Poisson equation", arXiv 1507.05063).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the correctness reference for the GPU solver.  Only the test suite,
 * the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no code, header, table or
 * constant with the GPU library, and the GPU library never calls it.
 *
 * Conventions (paper, Section 2): box [0,Lx]x[0,Ly]x[0,Lz]; nx, ny, nz uniform intervals; hx = Lx/nx, ...
 * A node array holds (nz+1)(ny+1)(nx+1) doubles, x fastest: index ((k*(ny+1)) + j)*(nx+1) + i.
 * Interior nodes are 1 <= i <= nx-1 (likewise j, k); the rest are boundary nodes.
 *
 * The interior system.  The compact scheme (eq. compact) reads L u = R f at interior nodes, where L is the
 * 19-point left-hand side and R f = (6 f_c + sum of the 6 face neighbours of f)/2.  Splitting L u into the
 * interior part and the boundary part gives L_II u_I = R f - L_IB g.  The oracle solves the negated system
 * M u_I = b with M = -L_II (symmetric positive definite) and b = -R f + L_IB g.  The relative residual
 * ||b - M u|| / ||b|| equals the paper's ||A_h u_h - f_h|| / ||f_h|| (the norm does not see the sign).
 *
 * All functions return 0 on success or a negative ORC_ERR_* code.
 */
#ifndef EXCMG_ORACLE_H
#define EXCMG_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_ERR_ARG (-1)
#define ORC_ERR_SHAPE (-2)
#define ORC_ERR_NOCONV (-4)
#define ORC_ERR_BREAKDOWN (-5)
#define ORC_ERR_NOMEM (-7)

/* Thread control for the OpenMP loops (plane-parallel sweeps; reductions are summed plane by plane in order). */
void orc_set_threads(int n);
void orc_set_progress(int on);
int orc_get_threads(void);

/* Left-hand side of eq. (compact) at interior nodes of the full node array u; out is 0 on boundary nodes. */
int orc_apply_L(int nx, int ny, int nz, double hx, double hy, double hz, const double *u, double *out);

/* Right-hand side operator of eq. (compact): out = (6 f_c + sum of 6 face neighbours)/2 at interior nodes. */
int orc_apply_R(int nx, int ny, int nz, double hx, double hy, double hz, const double *f, double *out);

/* y = M x = -L_II x.  x is a node array whose boundary entries are ignored (taken as zero). */
int orc_apply_M(int nx, int ny, int nz, double hx, double hy, double hz, const double *x, double *y);

/* b = -R f + L_IB g at interior nodes (eq. FD with the Dirichlet values eliminated); b is 0 on the boundary.
 * Only the boundary entries of g are read. */
int orc_rhs(int nx, int ny, int nz, double hx, double hy, double hz, const double *f, const double *g,
            double *b);

/* Conjugate gradients on M u = b from the interior of u (Algorithm 1, the relaxation loop).  The stopping test
 * ||r|| <= tol ||b|| is checked before every iteration on the recursively updated residual.  If fixed_iters >= 0
 * exactly that many iterations are taken instead.  hist (nullable, max_iters+1 entries) receives the recursive
 * relative residual after each iteration (entry 0: initial).  relres_out receives the true relative residual
 * ||b - M u|| / ||b|| at exit.  Boundary entries of u are left as they are. */
int orc_cg(int nx, int ny, int nz, double hx, double hy, double hz, const double *b, double *u, double tol,
           int max_iters, int fixed_iters, int *iters_out, double *relres_out, double *hist);

/* Direct solve of M u = b by banded Cholesky (DSOLVE of Algorithm 1 on the two coarsest grids).  Interior of u is
 * written. */
int orc_direct_solve(int nx, int ny, int nz, double hx, double hy, double hz, const double *b, double *u);

/* Banded matrix-vector product with the assembled M used by orc_direct_solve (cross-check of the assembly). */
int orc_banded_M_apply(int nx, int ny, int nz, double hx, double hy, double hz, const double *x, double *y);

/* Lagrange fundamental polynomial of degree 4 on the nodes 0,1,2,3,4, evaluated at t (eq. inter). */
double orc_lagrange4(int a, double t);

/* EXP_finite (Section 4.2.2 and 4.3): the initial guess w on the fine grid (nx,ny,nz) from the solutions on the
 * 2h grid (nx/2,...) and the 4h grid (nx/4,...).  nx, ny, nz must be multiples of 8.  Extrapolation at the 2h
 * nodes by eqs. (jiedian)/(zhongdian) and the diagonal means, tri-quartic Lagrange interpolation (eq. inter) on
 * every interpolation cell of 2x2x2 elements of the 4h grid, then boundary nodes set to g. */
int orc_exp_finite(int nx, int ny, int nz, const double *u2h, const double *u4h, const double *g, double *w);

/* The initial guesses the paper compares: its own (ORC_GUESS_QUARTIC, = orc_exp_finite), the same extrapolation at
 * the 2h nodes followed by tri-quadratic Lagrange interpolation on every cell of 2x2x2 elements of the 2h grid
 * (ORC_GUESS_QUADRATIC: the interpolation of the earlier EXCMG for linear elements, which the remark in Section 4.3
 * finds too inaccurate for a fourth-order solution), and trilinear interpolation of u_2h without extrapolation
 * (ORC_GUESS_LINEAR: the CMG prolongation of Section 3).  Shapes: multiples of 8, 4 and 2.  u4h is not read by
 * ORC_GUESS_LINEAR (may be NULL).  Boundary nodes of w are g. */
#define ORC_GUESS_QUARTIC 0
#define ORC_GUESS_QUADRATIC 1
#define ORC_GUESS_LINEAR 2
double orc_lagrange2(int a, double t);
int orc_initial_guess(int kind, int nx, int ny, int nz, const double *u2h, const double *u4h, const double *g,
                      double *w);

/* EXP_true (Sections 4.2.1 and 4.3): sixth-order extrapolated solution on the fine grid from u_h (fine) and
 * u_2h (nx/2,...): eq. (t1) at coarse nodes, eq. (chenlin) and its diagonal means elsewhere.  nx, ny, nz even. */
int orc_exp_true(int nx, int ny, int nz, const double *uh, const double *u2h, double *ut);

/* Compact fourth-order gradient (Section 5.1): one-sided fourth-order formulas at both ends of every grid line,
 * tridiagonal system (1/6, 4/6, 1/6) inside, solved by the Thomas algorithm.  Every axis needs >= 4 intervals. */
int orc_gradient(int nx, int ny, int nz, double hx, double hy, double hz, const double *u, double *ux,
                 double *uy, double *uz);

/* The EXCMG driver (Algorithm 1).  Levels nc * 2^l, l = 0..Lt, with nc * 2^Lt = n on every axis; the data of
 * level l is the finest f and g sampled at stride 2^(Lt-l).  Levels 0 and 1 are solved directly; every finer
 * level starts CG from EXP_finite of the two previous solutions.
 *   fixed_iters (nullable, Lt+1 entries): per level, >= 0 forces that CG iteration count, < 0 uses tol.
 *   u (out): finest solution, full node array with the boundary set to g.
 *   ut (nullable out): EXP_true(u_h, u_2h) on the finest grid (needs Lt >= 1).
 *   w_out (nullable out): the finest level's initial guess EXP_finite(u_2h, u_4h) (needs Lt >= 2).
 *   iters, relres (Lt+1 entries each): CG iterations and the true relative residual at exit per level.
 *   seconds (nullable, 2 entries): wall time of the whole solve and of the CG loops alone. */
int orc_excmg(int nx, int ny, int nz, double lx, double ly, double lz, int ncx, int ncy, int ncz,
              const double *f, const double *g, double tol, int max_iters, const int *fixed_iters, double *u,
              double *ut, double *w_out, int *iters, double *relres, double *seconds);

/* orc_excmg with the initial guess of kind guess (ORC_GUESS_*) on every level from 2 on, and the norm of the
 * stopping test ||A_h u_h - f_h|| <= eps ||f_h|| (Algorithm 1) read as stop_norm says: 0 = f_h is the eliminated
 * right-hand side b (the reading of orc_excmg), 1 = f_h is R f on the interior nodes and g on the boundary nodes
 * (the boundary values kept as identity rows), 2 = reading 1 on every level below the finest and reading 0 on the
 * finest.  tol_order = p > 0: level l of the finest Lt relaxes to
 * eps_l = tol * 2^(p (Lt - l)), capped at max(tol, 1e-2) (0: tol on every level).  No timing. */
int orc_excmg_variant(int guess, int stop_norm, int nx, int ny, int nz, double lx, double ly, double lz, int ncx,
                      int ncy, int ncz, const double *f, const double *g, double tol, double tol_order,
                      int max_iters, const int *fixed_iters, double *u, double *ut, double *w_out, int *iters,
                      double *relres);

/* Adjoint of the exact discrete map u = (interior: M^-1 b(f, g); boundary: g) for an upstream gradient G
 * (node array, dL/du).  lambda solves M lambda = G_I by the same cascade (level data: G sampled on the interior),
 * then dLdf = -R^T lambda on every node, and dLdg = L_IB^T lambda + G on boundary nodes (0 inside).
 * lambda_out (nullable) receives lambda as a node array with zero boundary. */
int orc_adjoint(int nx, int ny, int nz, double lx, double ly, double lz, int ncx, int ncy, int ncz,
                const double *G, double tol, int max_iters, const int *fixed_iters, double *dLdf, double *dLdg,
                double *lambda_out, int *iters, double *relres);

/* Plain transposes used by orc_adjoint, exposed for the transpose (dot-product) tests.
 * orc_apply_RT: out (all nodes) = R^T lam, lam read on interior nodes.
 * orc_apply_LIBT: out (boundary nodes) = L_IB^T lam, 0 inside. */
int orc_apply_RT(int nx, int ny, int nz, const double *lam, double *out);
int orc_apply_LIBT(int nx, int ny, int nz, double hx, double hy, double hz, const double *lam, double *out);

#ifdef __cplusplus
}
#endif
#endif
