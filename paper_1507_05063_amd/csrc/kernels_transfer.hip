// Level-transition and post-processing kernels of EXCMG for gfx950:
//   rhs            level right-hand side b = -R f + A_IB g (eq. compact with the Dirichlet values eliminated)
//   exp_finite     initial guess w_h = EXP_finite(u_2h, u_4h) (Sections 4.2.2 and 4.3)
//   exp_true       sixth-order u~_h = EXP_true(u_h, u_2h) (eqs. t1 and chenlin, Section 4.3)
//   set_boundary, copy: layout and boundary helpers
#include <math.h>

#include "excmg_internal.h"

namespace excmg {

namespace {

__device__ __forceinline__ bool on_boundary(int i, int j, int k, int nx, int ny, int nz) {
  return i == 0 || j == 0 || k == 0 || i == nx || j == ny || k == nz;
}

// ------------------------------------------------------------------------------------------------------------ rhs
// One thread per interior node of the level grid gb (rhs_at: eq. compact with the Dirichlet values eliminated).
__global__ void rhs_kernel(RhsSrc rs, Grid gb, double *__restrict__ b) {
  const int i = 1 + blockIdx.x * blockDim.x + threadIdx.x;
  const int j = 1 + blockIdx.y;
  const int k = 1 + blockIdx.z;
  if (i >= gb.nx) return;
  b[gb.at(i, j, k)] = rhs_at(rs, gb.nx, gb.ny, gb.nz, i, j, k);
}

// Node-wise kernels run 256 threads per workgroup over (x segment, y, z) = (bx, j, k).
__device__ __forceinline__ void set_boundary_block(const Grid &gg, const double *__restrict__ g, int s, const Grid &gu,
                                                   double *__restrict__ u, int zero_interior, int bx, int j, int k) {
  const int i = bx * 256 + threadIdx.x;
  if (i > gu.nx) return;
  if (on_boundary(i, j, k, gu.nx, gu.ny, gu.nz)) {
    u[gu.at(i, j, k)] = g ? g[gg.at(i * s, j * s, k * s)] : 0.0;
  } else if (zero_interior) {
    u[gu.at(i, j, k)] = 0.0;
  }
}

__global__ __launch_bounds__(256) void set_boundary_kernel(Grid gg, const double *__restrict__ g, int s, Grid gu,
                                                           double *__restrict__ u, int zero_interior) {
  set_boundary_block(gg, g, s, gu, u, zero_interior, blockIdx.x, blockIdx.y, blockIdx.z);
}

__device__ __forceinline__ void copy_block(const Grid &gs, const double *__restrict__ src, const Grid &gd,
                                           double *__restrict__ dst, int bx, int j, int k) {
  const int i = bx * 256 + threadIdx.x;
  if (i > gs.nx) return;
  __builtin_nontemporal_store(__builtin_nontemporal_load(&src[gs.at(i, j, k)]), &dst[gd.at(i, j, k)]);
}

__global__ __launch_bounds__(256) void copy_kernel(Grid gs, const double *__restrict__ src, Grid gd,
                                                   double *__restrict__ dst) {
  copy_block(gs, src, gd, dst, blockIdx.x, blockIdx.y, blockIdx.z);
}

__global__ void check_finite_kernel(const double *__restrict__ a, long long n, int *flag) {
  long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long stride = (long long)gridDim.x * blockDim.x;
  bool bad = false;
  for (; q < n; q += stride) bad |= !isfinite(a[q]);
  if (bad) *flag = 1;
}

// ----------------------------------------------------------------------------------------------------- exp_finite
// Quartic Lagrange weights (x128) at the odd fine offsets t = 1, 3, 5, 7 inside an interpolation cell whose known
// values sit at the even offsets 0, 2, 4, 6, 8 (the cell is 2x2x2 elements of the 4h grid = 8 fine elements per
// axis).  They are the Lagrange basis polynomials on the nodes 0..4 evaluated at t/2 = 0.5, 1.5, 2.5, 3.5.
constexpr double kQw[4][5] = {
    {35.0 / 128, 140.0 / 128, -70.0 / 128, 28.0 / 128, -5.0 / 128},
    {-5.0 / 128, 60.0 / 128, 90.0 / 128, -20.0 / 128, 3.0 / 128},
    {3.0 / 128, -20.0 / 128, 90.0 / 128, 60.0 / 128, -5.0 / 128},
    {-5.0 / 128, 28.0 / 128, -70.0 / 128, 140.0 / 128, 35.0 / 128},
};

constexpr int CXN = 8;               // interpolation cells per workgroup along x
constexpr int EX2 = 4 * CXN + 1;     // 2h nodes along x in the workgroup's slab
constexpr int EX4 = 2 * CXN + 1;     // 4h nodes along x
constexpr int EXF = 8 * CXN + 1;     // fine nodes along x
constexpr int ET = 256;

// quartic interpolation of five values at the odd offset T (0..3 for offsets 1, 3, 5, 7): the weights are
// compile-time constants
template <int T>
__device__ __forceinline__ double quartic(double a0, double a1, double a2, double a3, double a4) {
  return kQw[T][0] * a0 + kQw[T][1] * a1 + kQw[T][2] * a2 + kQw[T][3] * a3 + kQw[T][4] * a4;
}
// the same with a run-time offset t, from a copy of the weights in LDS
__device__ __forceinline__ double quartic(const double (*q)[5], int t, double a0, double a1, double a2, double a3,
                                          double a4) {
  return q[t][0] * a0 + q[t][1] * a1 + q[t][2] * a2 + q[t][3] * a3 + q[t][4] * a4;
}

// Quadratic Lagrange weights on the nodes 0, 1, 2 at 1/2 (T = 0) and 3/2 (T = 1): the odd fine offsets of a cell of
// two 2h elements (the tri-quadratic initial guess the paper compares its own with).
template <int T>
__device__ __forceinline__ double quadratic(double a0, double a1, double a2) {
  return T == 0 ? 0.375 * a0 + 0.75 * a1 - 0.125 * a2 : -0.125 * a0 + 0.75 * a1 + 0.375 * a2;
}

// The nine values at fine offsets 0..8 along one axis of a staged block, from the five known values at the even
// offsets: one tri-quartic cell (the paper's), or two tri-quadratic cells of two 2h elements each.
template <bool QUAD>
__device__ __forceinline__ void axis9(double a0, double a1, double a2, double a3, double a4, double (&o)[9]) {
  o[0] = a0;
  o[2] = a1;
  o[4] = a2;
  o[6] = a3;
  o[8] = a4;
  if constexpr (QUAD) {
    o[1] = quadratic<0>(a0, a1, a2);
    o[3] = quadratic<1>(a0, a1, a2);
    o[5] = quadratic<0>(a2, a3, a4);
    o[7] = quadratic<1>(a2, a3, a4);
  } else {
    o[1] = quartic<0>(a0, a1, a2, a3, a4);
    o[3] = quartic<1>(a0, a1, a2, a3, a4);
    o[5] = quartic<2>(a0, a1, a2, a3, a4);
    o[7] = quartic<3>(a0, a1, a2, a3, a4);
  }
}

// One workgroup per CXN x 1 x 1 interpolation cells.
//  1. stage u_2h on the 5x5x(4CXN+1) 2h nodes and delta = u_2h - u_4h on the 3x3x(2CXN+1) 4h nodes in LDS;
//  2. W = u_2h + delta_avg / 16 at every 2h node, where delta_avg is the mean of delta over the corners of the 4h
//     element face/edge the node is the centre of.  At 4h nodes this is eq. (jiedian), at edge midpoints eq.
//     (zhongdian), at face and element centres the mean over the 2 face / 4 space diagonals of eq. (zhongdian): all
//     four rules are the same tri-linear interpolation of delta with the factor 1/16;
//  3. tri-quartic interpolation (eq. inter) applied separably, x then y then z (the 604x125 cell matrix is the
//     tensor product of the 1D quartic weights): the x pass through LDS (one thread per cell, row and layer, so
//     that the four odd offsets have constant weights), then one thread per (x, y) column that interpolates its five
//     z layers in y from the x-pass values and then produces its nine z outputs;
//  4. boundary nodes get g.
// QUAD: the tri-quadratic variant of step 3 (cells of 2x2x2 elements of the 2h grid, two per axis of the block), the
// initial guess of the earlier EXCMG that the remark after eq. (inter) compares with; steps 1, 2 and 4 are the same.
template <bool QUAD>
__device__ void exp_finite_block(const Grid &g2, const double *__restrict__ u2, const Grid &g4,
                                 const double *__restrict__ u4, const Grid &gg, const double *__restrict__ gdat, int s,
                                 const Grid &gw, double *__restrict__ w, int bx, int cj, int ck, bool nt) {
  __shared__ double W[5][5][EX2];
  __shared__ double Wx[5][5][EXF];
  // D lives in Wx's space: it is dead (after the extrapolation) before the x pass writes Wx.  That keeps the
  // workgroup under 20 KB of LDS, so the LDS does not cap the occupancy below what the registers allow.
  static_assert(9 * EX4 <= 25 * EXF, "D fits in Wx");
  double(*D)[3][EX4] = reinterpret_cast<double(*)[3][EX4]>(&Wx[0][0][0]);
  __shared__ double Q[4][5];
  if (threadIdx.x < 20) Q[threadIdx.x / 5][threadIdx.x % 5] = kQw[threadIdx.x / 5][threadIdx.x % 5];
  const int ncx = gw.nx / 8, ncy = gw.ny / 8, ncz = gw.nz / 8;
  const int cx0 = bx * CXN;
  const int nc = min(CXN, ncx - cx0);  // cells in this workgroup (fewer in the last one along x)
  const int n2x = 4 * nc + 1, n4x = 2 * nc + 1;
  const int tid = threadIdx.x;
  const int I0 = 4 * cx0, J0 = 4 * cj, K0 = 4 * ck;  // 2h-grid origin of the slab
  // Index decompositions use the full-slab extents (compile-time divisors); entries past a short slab are skipped.
  // 1. stage
  // Every staging load of the thread is issued before any is waited for (a load per loop trip, stored to LDS in the
  // same trip, made the trips wait one memory latency each): addresses are clamped into the slab's 2h and 4h nodes,
  // and only the entries of the slab are stored.
  {
    constexpr int NW = (25 * EX2 + ET - 1) / ET, ND = (9 * EX4 + ET - 1) / ET;
    double wv[NW], dv[ND];
#pragma unroll
    for (int m = 0; m < NW; ++m) {
      const int e = min(tid + m * ET, 25 * EX2 - 1);
      const int a = min(e % EX2, n2x - 1), bc = e / EX2, b = bc % 5, c = bc / 5;
      wv[m] = u2[g2.at(I0 + a, J0 + b, K0 + c)];
    }
#pragma unroll
    for (int m = 0; m < ND; ++m) {
      const int e = min(tid + m * ET, 9 * EX4 - 1);
      const int a = min(e % EX4, n4x - 1), bc = e / EX4, b = bc % 3, c = bc / 3;
      dv[m] = u4[g4.at(I0 / 2 + a, J0 / 2 + b, K0 / 2 + c)];
    }
#pragma unroll
    for (int m = 0; m < NW; ++m) {
      const int e = tid + m * ET;
      const int a = e % EX2, bc = e / EX2, b = bc % 5, c = bc / 5;
      if (e < 25 * EX2 && a < n2x) W[c][b][a] = wv[m];
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < ND; ++m) {
      const int e = tid + m * ET;
      const int a = e % EX4, bc = e / EX4, b = bc % 3, c = bc / 3;
      if (e < 9 * EX4 && a < n4x) D[c][b][a] = W[2 * c][2 * b][2 * a] - dv[m];
    }
  }
  __syncthreads();
  // 2. extrapolate at the 2h nodes
  for (int e = tid; e < 25 * EX2; e += ET) {
    const int a = e % EX2, bc = e / EX2, b = bc % 5, c = bc / 5;
    if (a >= n2x) continue;
    const int al = a >> 1, ah = (a + 1) >> 1, bl = b >> 1, bh = (b + 1) >> 1, cl = c >> 1, ch = (c + 1) >> 1;
    const double d = ((D[cl][bl][al] + D[cl][bl][ah]) + (D[cl][bh][al] + D[cl][bh][ah])) +
                     ((D[ch][bl][al] + D[ch][bl][ah]) + (D[ch][bh][al] + D[ch][bh][ah]));
    W[c][b][a] += d * (1.0 / 128.0);  // (1/16) * (1/8) * sum over the 8 corner slots
  }
  __syncthreads();
  // 3a. x: one thread per (cell, row b, layer c) writes the cell's fine offsets 0..7 (the last cell also 8)
  static_assert(CXN * 25 <= ET, "one x-pass item per thread");
  if (tid < 25 * CXN) {
    const int cx = tid % CXN, bc = tid / CXN, b = bc % 5, c = bc / 5;
    if (cx < nc) {
      const double *wr = &W[c][b][4 * cx];
      double v9[9];
      axis9<QUAD>(wr[0], wr[1], wr[2], wr[3], wr[4], v9);
      double *o = &Wx[c][b][8 * cx];
#pragma unroll
      for (int q = 0; q < 8; ++q) o[q] = v9[q];
      if (cx == nc - 1) o[8] = v9[8];
    }
  }
  __syncthreads();
  // 3c. z and 4. write, one thread per (xf, yf) column.  Along x a workgroup writes offsets 1..8nc of its slab (the
  // slab's first node, offset 0, is the previous workgroup's last), so that with the grid's interior aligned to
  // 128-byte lines every row segment it stores is whole lines: 64 consecutive lanes take offsets 1..64.  The first
  // workgroup also writes offset 0 (the boundary).  Along y and z it owns offsets [0, 8), plus offset 8 at the far
  // faces.
  const bool lasty = (cj == ncy - 1), lastz = (ck == ncz - 1);
  const int oy = lasty ? 9 : 8, oz = lastz ? 9 : 8;
  const int gi0 = 8 * cx0, gj0 = 8 * cj, gk0 = 8 * ck;
  const int xhi = 8 * nc;
  auto column = [&](int xf, int yf) {
    const int gi = gi0 + xf, gj = gj0 + yf;
    // y: the five z layers of this column, from the x-interpolated values (known at even yf, quartic at odd yf)
    double a[5];
    if constexpr (QUAD) {
      const int q2 = 2 * (yf >> 2);  // first 2h node of the y cell
      const bool hi = (yf >> 1) & 1;  // offset 3/2 rather than 1/2
      const double w0 = hi ? -0.125 : 0.375, w2 = hi ? 0.375 : -0.125;
#pragma unroll
      for (int c = 0; c < 5; ++c)
        a[c] = (yf & 1) ? w0 * Wx[c][q2][xf] + 0.75 * Wx[c][q2 + 1][xf] + w2 * Wx[c][q2 + 2][xf]
                        : Wx[c][yf >> 1][xf];
    } else {
#pragma unroll
      for (int c = 0; c < 5; ++c)
        a[c] = (yf & 1) ? quartic(Q, yf >> 1, Wx[c][0][xf], Wx[c][1][xf], Wx[c][2][xf], Wx[c][3][xf], Wx[c][4][xf])
                        : Wx[c][yf >> 1][xf];
    }
    const bool side = (gi == 0 || gj == 0 || gi == gw.nx || gj == gw.ny);
    double zv[9];
    axis9<QUAD>(a[0], a[1], a[2], a[3], a[4], zv);
#pragma unroll
    for (int zf = 0; zf < 9; ++zf) {
      if (zf < oz) {
        const int gk = gk0 + zf;
        double v = zv[zf];
        if (side || gk == 0 || gk == gw.nz) v = gdat ? gdat[gg.at(gi * s, gj * s, gk * s)] : 0.0;
        if (nt) __builtin_nontemporal_store(v, &w[gw.at(gi, gj, gk)]);
        else w[gw.at(gi, gj, gk)] = v;
      }
    }
  };
  for (int e = tid; e < 64 * 9; e += ET) {
    const int xf = 1 + (e & 63), yf = e >> 6;
    if (xf <= xhi && yf < oy) column(xf, yf);
  }
  if (gi0 == 0)
    for (int yf = tid; yf < oy; yf += ET) column(0, yf);
}

// 7 waves per SIMD: the compiler's own choice (6, at 78 VGPRs) left too few workgroups in flight to cover the
// staging loads (0.455 -> 0.42 ms at 512^3; 8 waves spills registers and is slower)
template <bool QUAD>
__global__ __launch_bounds__(ET) __attribute__((amdgpu_waves_per_eu(7, 7))) void exp_finite_kernel(Grid g2, const double *__restrict__ u2, Grid g4,
                                                        const double *__restrict__ u4, Grid gg,
                                                        const double *__restrict__ gdat, int s, Grid gw,
                                                        double *__restrict__ w) {
  // w is read again right away by the residual sweep: streaming stores only where it cannot stay in the caches
  exp_finite_block<QUAD>(g2, u2, g4, u4, gg, gdat, s, gw, w, blockIdx.x, blockIdx.y, blockIdx.z,
                         gw.interior() >= (1LL << 23));
}

// The CMG initial guess the paper compares with (Section 3): u_2h interpolated trilinearly, without extrapolation
// (the mean of the 1, 2, 4 or 8 nearest 2h nodes), and g on the boundary.  One thread per node.
__global__ __launch_bounds__(256) void prolong_linear_kernel(Grid g2, const double *__restrict__ u2, Grid gg,
                                                             const double *__restrict__ gdat, int s, Grid gw,
                                                             double *__restrict__ w) {
  const int i = blockIdx.x * 256 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
  if (i > gw.nx) return;
  double v;
  if (on_boundary(i, j, k, gw.nx, gw.ny, gw.nz)) {
    v = gdat ? gdat[gg.at(i * s, j * s, k * s)] : 0.0;
  } else {
    const int I = i >> 1, J = j >> 1, K = k >> 1, di = i & 1, dj = j & 1, dk = k & 1;
    double acc = 0.0;
    for (int c = 0; c <= dk; ++c)
      for (int b = 0; b <= dj; ++b)
        for (int a = 0; a <= di; ++a) acc += u2[g2.at(I + a, J + b, K + c)];
    v = acc * (1.0 / (double)(1 << (di + dj + dk)));
  }
  w[gw.at(i, j, k)] = v;
}

// ------------------------------------------------------------------------------------------------------- exp_true
// u~ = u_h + delta_avg / 15 where delta = u_h - u_2h at the 2h nodes and delta_avg its mean over the corners of the
// 2h edge/face/element the node is the midpoint of: eq. (t1) at 2h nodes, eq. (chenlin) at edge midpoints, and its
// mean over the 2 face / 4 space diagonals at face / element centres.
// A workgroup owns the fine nodes x0+1 .. x0+64, y0+1 .. y0+4, z0+1 .. z0+2 (x0, y0, z0 multiples of the block
// size; the first block along an axis also takes node 0): it first forms delta on the 33 x 3 x 2 even nodes
// x0 .. x0+64, ... in LDS, then every thread writes the 2 (or 3) nodes of its (x, y) column.  Starting the blocks at
// offset 1 keeps the row segments of u_h on whole 128-byte lines and leaves no block with a single node along an
// axis.  Thin blocks measured fastest at 512^3: 2 planes 0.72 ms, 4 planes 0.79 ms, 8 planes 0.88 ms, 16 planes
// 0.92 ms (more workgroups in flight, each with a short chain of loads and stores).
constexpr int TTX = 64, TTY = 4, TTZ = 2;
constexpr int DTX = TTX / 2 + 1, DTY = TTY / 2 + 1, DTZ = TTZ / 2 + 1;

// ucopy (nullable): u_h itself is also written there, in the layout gt (the solution's copy to the caller's array,
// made from the same read of u_h).
__global__ __launch_bounds__(TTX *TTY) void exp_true_kernel(Grid gh, const double *__restrict__ uh, Grid g2,
                                                           const double *__restrict__ u2, Grid gt,
                                                           double *__restrict__ ut, double *__restrict__ ucopy) {
  __shared__ double D[DTZ][DTY][DTX];
  // blockIdx.x runs along y: consecutive workgroups (which the hardware deals out to the XCDs in turn) take
  // different rows, so all the blocks of one row segment run on one XCD and no cache line is written from two
  const int bx = blockIdx.y, by = blockIdx.x;
  const int x0 = bx * TTX, y0 = by * TTY, z0 = blockIdx.z * TTZ;
  const int tid = threadIdx.x;
  for (int e = tid; e < DTX * DTY * DTZ; e += TTX * TTY) {
    const int a = e % DTX, bc = e / DTX, b = bc % DTY, c = bc / DTY;
    const int I = x0 / 2 + a, J = y0 / 2 + b, K = z0 / 2 + c;  // 2h-grid node
    double d = 0.0;
    if (2 * I <= gh.nx && 2 * J <= gh.ny && 2 * K <= gh.nz) d = uh[gh.at(2 * I, 2 * J, 2 * K)] - u2[g2.at(I, J, K)];
    D[c][b][a] = d;
  }
  __syncthreads();
  const int lx = tid % TTX, ly = tid / TTX;
  const bool z_first = (blockIdx.z == 0);
  // column (x0 + ox, y0 + oy), local offsets ox in 0..64, oy in 0..4
  auto column = [&](int ox, int oy) {
    const int i = x0 + ox, j = y0 + oy;
    if (i > gh.nx || j > gh.ny) return;
    const int al = ox >> 1, ah = (ox + 1) >> 1, bl = oy >> 1, bh = (oy + 1) >> 1;
    double dxy[DTZ];  // the four corner slots in x and y of every even z layer of the block
#pragma unroll
    for (int c = 0; c < DTZ; ++c) dxy[c] = (D[c][bl][al] + D[c][bl][ah]) + (D[c][bh][al] + D[c][bh][ah]);
    auto put = [&](int q, double v) {  // z offset q in 0..8, u_h there
      const int k = z0 + q;
      const double d = dxy[q >> 1] + dxy[(q + 1) >> 1];
      // the outputs are the caller's: streaming stores
      __builtin_nontemporal_store(v + d * (1.0 / 120.0), &ut[gt.at(i, j, k)]);  // (1/15) (1/8) sum of the 8 slots
      if (ucopy) __builtin_nontemporal_store(v, &ucopy[gt.at(i, j, k)]);
    };
    if (z_first) put(0, uh[gh.at(i, j, z0)]);
    double v[TTZ];  // all of the column's loads first (planes past the grid read its last plane and are not stored)
#pragma unroll
    for (int q = 1; q <= TTZ; ++q) v[q - 1] = uh[gh.at(i, j, min(z0 + q, gh.nz))];
#pragma unroll
    for (int q = 1; q <= TTZ; ++q)
      if (z0 + q <= gh.nz) put(q, v[q - 1]);
  };
  column(1 + lx, 1 + ly);
  if (bx == 0 && lx == 0) column(0, 1 + ly);
  if (by == 0 && ly == 0) column(1 + lx, 0);
  if (bx == 0 && by == 0 && tid == 0) column(0, 0);
}

// ------------------------------------------------------------------------------------------------------- adjoint
// Gather form of the transposes, one thread per node of the finest grid (dense outputs):
//   dLdf(n) = -(3 lam_n [n interior] + 1/2 * sum of lam over the interior face neighbours of n)
//   dLdg(n) = sum over interior neighbours m of A's coefficient for the offset m - n, times lam_m, plus G(n),
//             on boundary nodes; 0 inside.
__global__ void adjoint_kernel(Grid gl, const double *__restrict__ lam, Grid gd, const double *__restrict__ G,
                               double *__restrict__ dLdf, double *__restrict__ dLdg, double a, double bb, double c) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  const int k = blockIdx.z;
  const int nx = gl.nx, ny = gl.ny, nz = gl.nz;
  if (i > nx) return;
  auto L = [&](int ii, int jj, int kk) -> double {
    if (ii <= 0 || jj <= 0 || kk <= 0 || ii >= nx || jj >= ny || kk >= nz) return 0.0;
    return lam[gl.at(ii, jj, kk)];
  };
  const double rt = 3.0 * L(i, j, k) +
                    0.5 * ((L(i + 1, j, k) + L(i - 1, j, k)) + (L(i, j + 1, k) + L(i, j - 1, k)) +
                           (L(i, j, k + 1) + L(i, j, k - 1)));
  const long long q = gd.at(i, j, k);
  dLdf[q] = -rt;
  if (!on_boundary(i, j, k, nx, ny, nz)) {
    dLdg[q] = 0.0;
    return;
  }
  const double fx = 4.0 * a - bb - c, fy = 4.0 * bb - a - c, fz = 4.0 * c - a - bb;
  const double exy = 0.5 * (a + bb), exz = 0.5 * (a + c), eyz = 0.5 * (bb + c);
  double s = fx * (L(i + 1, j, k) + L(i - 1, j, k)) + fy * (L(i, j + 1, k) + L(i, j - 1, k)) +
             fz * (L(i, j, k + 1) + L(i, j, k - 1));
  s += exy * ((L(i + 1, j + 1, k) + L(i - 1, j + 1, k)) + (L(i + 1, j - 1, k) + L(i - 1, j - 1, k)));
  s += exz * ((L(i + 1, j, k + 1) + L(i - 1, j, k + 1)) + (L(i + 1, j, k - 1) + L(i - 1, j, k - 1)));
  s += eyz * ((L(i, j + 1, k + 1) + L(i, j - 1, k + 1)) + (L(i, j + 1, k - 1) + L(i, j - 1, k - 1)));
  dLdg[q] = s + G[q];
}

// ---------------------------------------------------------------------------------------------------- batched form
// Flattened over a table of problems (see BatchEntry): workgroup b belongs to the entry e with
// pre[e] <= b < pre[e+1] and takes the local index b - pre[e] in that entry's launch.
__device__ __forceinline__ int find_entry_t(const int *pre, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// boundary values and zero interior on grids 0 and 1
__global__ __launch_bounds__(256) void b_set_boundary_kernel(BatchList L) {
  const int e = find_entry_t(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const int gx = (E.g.nx + 1 + 255) / 256, gy = E.g.ny + 1;
  const int lb = blockIdx.x - L.pre[e];
  set_boundary_block(E.gd, E.gb, E.rs.s, E.g, E.u, 1, lb % gx, (lb / gx) % gy, lb / (gx * gy));
}

__global__ __launch_bounds__(256) void b_copy_kernel(BatchList L) {
  const int e = find_entry_t(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const int gx = (E.g.nx + 1 + 255) / 256, gy = E.g.ny + 1;
  const int lb = blockIdx.x - L.pre[e];
  copy_block(E.g, E.u, E.gd, E.out, lb % gx, (lb / gx) % gy, lb / (gx * gy));
}

__global__ __launch_bounds__(ET) void b_exp_finite_kernel(BatchList L) {
  const int e = find_entry_t(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const int ncx = E.g.nx / 8, ncy = E.g.ny / 8;
  const int gx = (ncx + CXN - 1) / CXN;
  const int lb = blockIdx.x - L.pre[e];
  exp_finite_block<false>(E.g2, E.u2, E.g4, E.u4, E.gd, E.gb, E.rs.s, E.g, E.u, lb % gx, (lb / gx) % ncy, lb / (gx * ncy),
                   false);
}

inline dim3 node_grid(const Grid &g, int bx) { return dim3((g.nx + 1 + bx - 1) / bx, g.ny + 1, g.nz + 1); }
inline dim3 interior_grid(const Grid &g, int bx) { return dim3((g.nx - 1 + bx - 1) / bx, g.ny - 1, g.nz - 1); }

}  // namespace

void launch_rhs(const RhsSrc &rs, const Grid &gb, double *b, hipStream_t st) {
  rhs_kernel<<<interior_grid(gb, 256), 256, 0, st>>>(rs, gb, b);
}

void launch_set_boundary(const Grid &gg, const double *g, int stride, const Grid &gu, double *u, int zero_interior,
                         hipStream_t st) {
  set_boundary_kernel<<<node_grid(gu, 256), 256, 0, st>>>(gg, g, stride, gu, u, zero_interior);
}

void launch_initial_guess(int kind, const Grid &g2, const double *u2, const Grid &g4, const double *u4,
                          const Grid &gg, const double *g, int stride, const Grid &gw, double *w, hipStream_t st) {
  if (kind == kGuessLinear) {
    prolong_linear_kernel<<<node_grid(gw, 256), 256, 0, st>>>(g2, u2, gg, g, stride, gw, w);
    return;
  }
  const int ncx = gw.nx / 8, ncy = gw.ny / 8, ncz = gw.nz / 8;
  dim3 grid((ncx + CXN - 1) / CXN, ncy, ncz);
  if (kind == kGuessQuadratic) exp_finite_kernel<true><<<grid, ET, 0, st>>>(g2, u2, g4, u4, gg, g, stride, gw, w);
  else exp_finite_kernel<false><<<grid, ET, 0, st>>>(g2, u2, g4, u4, gg, g, stride, gw, w);
}

void launch_exp_true(const Grid &gh, const double *uh, const Grid &g2, const double *u2, const Grid &gt, double *ut,
                     double *ucopy, hipStream_t st) {
  dim3 grid((gh.ny + TTY - 1) / TTY, (gh.nx + TTX - 1) / TTX, (gh.nz + TTZ - 1) / TTZ);
  exp_true_kernel<<<grid, TTX * TTY, 0, st>>>(gh, uh, g2, u2, gt, ut, ucopy);
}

void launch_copy(const Grid &gs, const double *src, const Grid &gd, double *dst, hipStream_t st) {
  copy_kernel<<<node_grid(gs, 256), 256, 0, st>>>(gs, src, gd, dst);
}

void launch_check_finite(const double *a, long long n, int *flag, hipStream_t st) {
  long long blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  check_finite_kernel<<<(int)blocks, 256, 0, st>>>(a, n, flag);
}

void launch_adjoint_transposes(const Grid &gl, const double *lam, const Grid &gd, const double *G, double *dLdf,
                               double *dLdg, double hx, double hy, double hz, hipStream_t st) {
  adjoint_kernel<<<node_grid(gl, 256), 256, 0, st>>>(gl, lam, gd, G, dLdf, dLdg, 1.0 / (hx * hx), 1.0 / (hy * hy),
                                                     1.0 / (hz * hz));
}

int b_blocks_nodes(const Grid &g) { return ((g.nx + 1 + 255) / 256) * (g.ny + 1) * (g.nz + 1); }

int b_blocks_exp_finite(const Grid &gw) {
  const int ncx = gw.nx / 8, ncy = gw.ny / 8, ncz = gw.nz / 8;
  return ((ncx + CXN - 1) / CXN) * ncy * ncz;
}

void launch_b_set_boundary(const BatchList &L, hipStream_t st) {
  if (L.total > 0) b_set_boundary_kernel<<<L.total, 256, 0, st>>>(L);
}

void launch_b_exp_finite(const BatchList &L, hipStream_t st) {
  if (L.total > 0) b_exp_finite_kernel<<<L.total, ET, 0, st>>>(L);
}

void launch_b_copy(const BatchList &L, hipStream_t st) {
  if (L.total > 0) b_copy_kernel<<<L.total, 256, 0, st>>>(L);
}

}  // namespace excmg
