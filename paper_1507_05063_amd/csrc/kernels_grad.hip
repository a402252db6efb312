// Fourth-order compact gradient (Section 5.1) for gfx950.
//
// Along every grid line (including lines on the boundary) of length N cells, with v = du/dx (or y, z):
//   v_0 = (-25 u_0 + 48 u_1 - 36 u_2 + 16 u_3 - 3 u_4) / (12 h),  v_N the mirror image with the opposite sign,
//   v_{i-1} + 4 v_i + v_{i+1} = 3 (u_{i+1} - u_{i-1}) / h,  i = 1..N-1
// (the paper's (1/6, 4/6, 1/6) system times 6).  The constant-coefficient Thomas factors m_1 = 4,
// m_i = 4 - 1/m_{i-1} are shared by all lines; the host passes 1/m_i per axis.
#include "excmg_internal.h"

namespace excmg {

namespace {

__device__ __forceinline__ double end0(double u0, double u1, double u2, double u3, double u4, double h) {
  return (-25.0 * u0 + 48.0 * u1 - 36.0 * u2 + 16.0 * u3 - 3.0 * u4) / (12.0 * h);
}

// One line per thread: u[idx0 + t*su] and out[odx0 + t*so], t = 0..N.  The Thomas sweeps run chunk by chunk, GC
// unknowns at a time, with the forward-eliminated values d of two chunks in registers: once the forward sweep has
// finished chunk c+1, the back substitution starts at the top of chunk c+1 with v = d there (as if the unknown above
// were 0) and runs down through chunk c, whose values are then final and stored.  The starting error is damped by
// 1/m_t < 2 - sqrt(3) per step, so after the GC = 32 steps of chunk c+1 it is below 0.268^32 = 5e-19 of |v|: the
// result is the exact Thomas solution to rounding, while u is read once and each output written once.
constexpr int GC = 32;

__device__ __forceinline__ void line_solve(const double *__restrict__ u, long long idx0, long long su, double *out,
                                           long long odx0, long long so, int N, double h,
                                           const double *__restrict__ inv_m) {
  auto U = [&](int t) { return u[idx0 + (long long)t * su]; };
  const double v0 = end0(U(0), U(1), U(2), U(3), U(4), h);
  const double vN = -end0(U(N), U(N - 1), U(N - 2), U(N - 3), U(N - 4), h);
  out[odx0] = v0;
  out[odx0 + (long long)N * so] = vN;
  const double s3 = 3.0 / h;
  const int M = N - 1;  // interior unknowns t = 1..M
  double um = U(0), uc = U(1), dprev = 0.0;
  // forward elimination of the chunk starting at t0 into d[]
  auto forward = [&](double (&d)[GC], int t0) {
    constexpr int G = 8;  // loads issued ahead of the dependent elimination chain
#pragma unroll
    for (int q0 = 0; q0 < GC; q0 += G) {
      double up[G];
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int t = t0 + q0 + q;
        up[q] = (t <= M) ? U(t + 1) : 0.0;
      }
#pragma unroll
      for (int q = 0; q < G; ++q) {
        const int t = t0 + q0 + q;
        if (t <= M) {
          double rhs = s3 * (up[q] - um);
          if (t == 1) rhs -= v0;
          if (t == M) rhs -= vN;
          const double dd = (rhs - dprev) * inv_m[t];
          d[q0 + q] = dd;
          dprev = dd;
          um = uc;
          uc = up[q];
        }
      }
    }
  };
  double dA[GC], dB[GC];
  forward(dA, 1);
  for (int t0 = 1; t0 <= M; t0 += GC) {
    const int t1 = t0 + GC;  // first unknown of the next chunk
    double v = 0.0;          // v_{t+1} during the back substitution
    if (t1 <= M) {
      forward(dB, t1);
#pragma unroll
      for (int q = GC - 1; q >= 0; --q) {
        const int t = t1 + q;
        if (t <= M) v = (t == M) ? dB[q] : dB[q] - inv_m[t] * v;
      }
    }
#pragma unroll
    for (int q = GC - 1; q >= 0; --q) {
      const int t = t0 + q;
      if (t <= M) {
        v = (t == M) ? dA[q] : dA[q] - inv_m[t] * v;
        __builtin_nontemporal_store(v, &out[odx0 + (long long)t * so]);  // the caller's output
      }
    }
#pragma unroll
    for (int q = 0; q < GC; ++q) dA[q] = dB[q];
  }
}

// x lines: one thread per line, 64 lines per workgroup.  The rows are contiguous in memory, so the chunk of GC values
// every line needs next is staged through an LDS tile with coalesced loads (each 32-value row segment read by 32
// consecutive threads), and the finished chunk goes back out through the same tile with coalesced stores.  The
// Thomas sweeps are those of line_solve, with u taken from the tile.
constexpr int XW = 64;

__global__ __launch_bounds__(XW) void grad_x_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *ux,
                                                    double hx, const double *__restrict__ inv_m) {
  __shared__ double tile[XW][GC + 1];
  __shared__ long long rb[XW], ob[XW];  // row starts of the workgroup's lines in u and in ux
  const int nlines = (gu.ny + 1) * (gu.nz + 1);
  const int L0 = blockIdx.x * XW;
  const int tid = threadIdx.x;
  const int nl = min(XW, nlines - L0);
  const int N = gu.nx, M = N - 1;
  {
    const int L = L0 + (tid < nl ? tid : 0);
    const int j = L % (gu.ny + 1), k = L / (gu.ny + 1);
    rb[tid] = gu.at(0, j, k);
    ob[tid] = gd.at(0, j, k);
  }
  __syncthreads();
  const bool act = tid < nl;
  const long long b = rb[tid];
  double v0 = 0.0, vN = 0.0, um = 0.0, uc = 0.0;
  if (act) {
    v0 = end0(u[b], u[b + 1], u[b + 2], u[b + 3], u[b + 4], hx);
    vN = -end0(u[b + N], u[b + N - 1], u[b + N - 2], u[b + N - 3], u[b + N - 4], hx);
    ux[ob[tid]] = v0;
    ux[ob[tid] + N] = vN;
    um = u[b];
    uc = u[b + 1];
  }
  const double s3 = 3.0 / hx;
  double dprev = 0.0;
  // tile <- u at x = t0+1 .. t0+GC of every line (the values the forward sweep over t0 .. t0+GC-1 needs)
  auto load = [&](int t0) {
#pragma unroll 8
    for (int m = 0; m < GC; ++m) {
      const int e = tid + m * XW;
      const int ln = e / GC, xx = e % GC, x = t0 + 1 + xx;
      tile[ln][xx] = (ln < nl && x <= N) ? u[rb[ln] + x] : 0.0;
    }
  };
  auto forward = [&](double (&d)[GC], int t0) {
#pragma unroll
    for (int q = 0; q < GC; ++q) {
      const int t = t0 + q;
      if (t <= M) {
        const double up = tile[tid][q];
        double rhs = s3 * (up - um);
        if (t == 1) rhs -= v0;
        if (t == M) rhs -= vN;
        const double dd = (rhs - dprev) * inv_m[t];
        d[q] = dd;
        dprev = dd;
        um = uc;
        uc = up;
      }
    }
  };
  double dA[GC], dB[GC];
  load(1);
  __syncthreads();
  forward(dA, 1);
  __syncthreads();
  for (int t0 = 1; t0 <= M; t0 += GC) {
    const int t1 = t0 + GC;
    double v = 0.0;
    if (t1 <= M) {
      load(t1);
      __syncthreads();
      forward(dB, t1);
      __syncthreads();  // every line has consumed the tile
#pragma unroll
      for (int q = GC - 1; q >= 0; --q) {
        const int t = t1 + q;
        if (t <= M) v = (t == M) ? dB[q] : dB[q] - inv_m[t] * v;
      }
    }
#pragma unroll
    for (int q = GC - 1; q >= 0; --q) {
      const int t = t0 + q;
      if (t <= M) {
        v = (t == M) ? dA[q] : dA[q] - inv_m[t] * v;
        tile[tid][q] = v;
      }
    }
    __syncthreads();
#pragma unroll 8
    for (int m = 0; m < GC; ++m) {
      const int e = tid + m * XW;
      const int ln = e / GC, xx = e % GC, t = t0 + xx;
      if (ln < nl && t <= M) __builtin_nontemporal_store(tile[ln][xx], &ux[ob[ln] + t]);
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < GC; ++q) dA[q] = dB[q];
  }
}

// x lines, one wavefront per line (grids of at most kXWaveMax cells along x): the line is read into LDS with
// contiguous loads, and lane l produces the XS unknowns t0 = 1 + XS l (+ 64 XS per pass) from its own windows: the
// forward elimination starts XWIN unknowns before t0 with d = 0 in place of the true d there, the back substitution
// starts XWIN unknowns after the lane's last one with v = d there; both starting errors are damped below
// 0.268^32 = 5e-19 of the values by the time they reach the lane's unknowns, so the result is the Thomas solution to
// rounding (as in line_solve).  The factors 1/m_t reach their limit 1/(2 + sqrt 3) to the last bit by t = 14, so the
// first kInvM of them sit in LDS and the rest equal the last of those.  The results go back through LDS and out with
// contiguous stores.
constexpr int XS = 8, XWIN = 32, kInvM = 32;
constexpr int kXWaveMax = 4095;

__global__ __launch_bounds__(64) void grad_x_wave_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *ux,
                                                         double hx, const double *__restrict__ inv_m) {
  extern __shared__ double lds[];
  __shared__ double im[kInvM + 1];
  const int N = gu.nx, M = N - 1;
  // LDS position of unknown t: one pad word per XS, so that the lanes (XS apart) hit different banks
  auto P = [](int t) { return t + (t >> 3); };
  double *lu = lds, *lo = lds + P(N) + 1;
  const int L = blockIdx.x;
  const int j = L % (gu.ny + 1), k = L / (gu.ny + 1);
  const long long b = gu.at(0, j, k), ob = gd.at(0, j, k);
  for (int t = threadIdx.x; t <= N; t += 64) lu[P(t)] = u[b + t];
  for (int t = threadIdx.x; t <= kInvM; t += 64) im[t] = (t >= 1 && t <= M) ? inv_m[t] : (t > M ? inv_m[M] : 0.0);
  __syncthreads();
  const double v0 = end0(lu[P(0)], lu[P(1)], lu[P(2)], lu[P(3)], lu[P(4)], hx);
  const double vN = -end0(lu[P(N)], lu[P(N - 1)], lu[P(N - 2)], lu[P(N - 3)], lu[P(N - 4)], hx);
  const double s3 = 3.0 / hx;
  auto rhs = [&](int t) {
    double r = s3 * (lu[P(t + 1)] - lu[P(t - 1)]);
    if (t == 1) r -= v0;
    if (t == M) r -= vN;
    return r;
  };
  auto invm = [&](int t) { return im[t < kInvM ? t : kInvM]; };
  if (threadIdx.x == 0) {
    lo[P(0)] = v0;
    lo[P(N)] = vN;
  }
  for (int base = 1; base <= M; base += 64 * XS) {
    const int t0 = base + threadIdx.x * XS;
    if (t0 <= M) {
      const int te = t0 + XS - 1 + XWIN > M ? M : t0 + XS - 1 + XWIN;
      double d = 0.0;
#pragma unroll
      for (int q = -XWIN; q < 0; ++q) {
        const int t = t0 + q;
        if (t >= 1) d = (rhs(t) - d) * invm(t);
      }
      double dk[XS + XWIN];
#pragma unroll
      for (int q = 0; q < XS + XWIN; ++q) {
        const int t = t0 + q;
        if (t <= te) {
          d = (rhs(t) - d) * invm(t);
          dk[q] = d;
        }
      }
      double v = 0.0;
#pragma unroll
      for (int q = XS + XWIN - 1; q >= 0; --q) {
        const int t = t0 + q;
        if (t <= te) {
          v = (t == M) ? dk[q] : dk[q] - invm(t) * v;
          if (q < XS) lo[P(t)] = v;
        }
      }
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t <= N; t += 64) __builtin_nontemporal_store(lo[P(t)], &ux[ob + t]);
}

// y and z lines: one thread per line, consecutive threads on consecutive x, so every step of the sweeps is a
// coalesced row access.
__global__ __launch_bounds__(64) void grad_y_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *uy,
                                                    double hy, const double *__restrict__ inv_m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i > gu.nx) return;
  line_solve(u, gu.at(i, 0, k), gu.sy, uy, gd.at(i, 0, k), gd.sy, gu.ny, hy, inv_m);
}

__global__ __launch_bounds__(64) void grad_z_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *uz,
                                                    double hz, const double *__restrict__ inv_m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i > gu.nx) return;
  line_solve(u, gu.at(i, j, 0), gu.sz, uz, gd.at(i, j, 0), gd.sz, gu.nz, hz, inv_m);
}

}  // namespace

void launch_gradient(const Grid &gu, const double *u, const Grid &gd, double *ux, double *uy, double *uz, double hx,
                     double hy, double hz, const double *inv_m_x, const double *inv_m_y, const double *inv_m_z,
                     hipStream_t st) {
  const int nlines = (gu.ny + 1) * (gu.nz + 1);
  if (gu.nx <= kXWaveMax)
    grad_x_wave_kernel<<<nlines, 64, 2 * (size_t)(gu.nx + gu.nx / 8 + 2) * sizeof(double), st>>>(gu, u, gd, ux, hx,
                                                                                                inv_m_x);
  else
    grad_x_kernel<<<(nlines + XW - 1) / XW, XW, 0, st>>>(gu, u, gd, ux, hx, inv_m_x);
  grad_y_kernel<<<dim3((gu.nx + 1 + 63) / 64, gu.nz + 1), 64, 0, st>>>(gu, u, gd, uy, hy, inv_m_y);
  grad_z_kernel<<<dim3((gu.nx + 1 + 63) / 64, gu.ny + 1), 64, 0, st>>>(gu, u, gd, uz, hz, inv_m_z);
}

}  // namespace excmg
