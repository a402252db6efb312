// Fourth-order compact gradient (Section 5.1) for gfx950.
//
// Along every grid line (including lines on the boundary) of length N cells, with v = du/dx (or y, z):
//   v_0 = (-25 u_0 + 48 u_1 - 36 u_2 + 16 u_3 - 3 u_4) / (12 h),  v_N the mirror image with the opposite sign,
//   v_{i-1} + 4 v_i + v_{i+1} = 3 (u_{i+1} - u_{i-1}) / h,  i = 1..N-1
// (the paper's (1/6, 4/6, 1/6) system times 6).  The constant-coefficient Thomas factors m_1 = 4,
// m_i = 4 - 1/m_{i-1} are shared by all lines; the host passes 1/m_i per axis.  Forward elimination stores the
// modified right-hand sides in the output array, back substitution overwrites them with v.
//
// y and z lines: one thread per line, consecutive threads on consecutive x, so every step of the sweep is a
// coalesced row access.  x lines: a workgroup of 256 threads takes 256 lines and walks x in chunks of 8 staged
// through LDS (loads and stores run along x; each thread then sweeps its own row of the chunk).
#include "excmg_internal.h"

namespace excmg {

namespace {

__device__ __forceinline__ double end0(double u0, double u1, double u2, double u3, double u4, double h) {
  return (-25.0 * u0 + 48.0 * u1 - 36.0 * u2 + 16.0 * u3 - 3.0 * u4) / (12.0 * h);
}

// one line: u[idx0 + t*su], out[odx0 + t*so], t = 0..N
__device__ __forceinline__ void line_solve(const double *__restrict__ u, long long idx0, long long su, double *out,
                                           long long odx0, long long so, int N, double h,
                                           const double *__restrict__ inv_m) {
  auto U = [&](int t) { return u[idx0 + (long long)t * su]; };
  const double v0 = end0(U(0), U(1), U(2), U(3), U(4), h);
  const double vN = -end0(U(N), U(N - 1), U(N - 2), U(N - 3), U(N - 4), h);
  out[odx0] = v0;
  out[odx0 + (long long)N * so] = vN;
  const double s3 = 3.0 / h;
  double um = U(0), uc = U(1);
  double dprev = 0.0;
  constexpr int UN = 8;  // loads issued ahead of the dependent elimination chain
  int t = 1;
  for (; t + UN - 1 <= N - 1; t += UN) {
    double up[UN];
#pragma unroll
    for (int q = 0; q < UN; ++q) up[q] = U(t + q + 1);
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      const int tt = t + q;
      double rhs = s3 * (up[q] - um);
      if (tt == 1) rhs -= v0;
      if (tt == N - 1) rhs -= vN;
      const double d = (rhs - dprev) * inv_m[tt];
      out[odx0 + (long long)tt * so] = d;
      dprev = d;
      um = uc;
      uc = up[q];
    }
  }
  for (; t <= N - 1; ++t) {
    const double up = U(t + 1);
    double rhs = s3 * (up - um);
    if (t == 1) rhs -= v0;
    if (t == N - 1) rhs -= vN;
    const double d = (rhs - dprev) * inv_m[t];
    out[odx0 + (long long)t * so] = d;
    dprev = d;
    um = uc;
    uc = up;
  }
  double vnext = out[odx0 + (long long)(N - 1) * so];
  int tb = N - 2;
  for (; tb - UN + 1 >= 1; tb -= UN) {
    double dd[UN];
#pragma unroll
    for (int q = 0; q < UN; ++q) dd[q] = out[odx0 + (long long)(tb - q) * so];
#pragma unroll
    for (int q = 0; q < UN; ++q) {
      const double v = dd[q] - inv_m[tb - q] * vnext;
      out[odx0 + (long long)(tb - q) * so] = v;
      vnext = v;
    }
  }
  for (; tb >= 1; --tb) {
    const double v = out[odx0 + (long long)tb * so] - inv_m[tb] * vnext;
    out[odx0 + (long long)tb * so] = v;
    vnext = v;
  }
}

__global__ void grad_y_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *uy, double hy,
                              const double *__restrict__ inv_m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  if (i > gu.nx) return;
  line_solve(u, gu.at(i, 0, k), gu.sy, uy, gd.at(i, 0, k), gd.sy, gu.ny, hy, inv_m);
}

__global__ void grad_z_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *uz, double hz,
                              const double *__restrict__ inv_m) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (i > gu.nx) return;
  line_solve(u, gu.at(i, j, 0), gu.sz, uz, gd.at(i, j, 0), gd.sz, gu.nz, hz, inv_m);
}

constexpr int XL = 256;     // x lines per workgroup (one thread per line)
constexpr int XC = 8;       // chunk length along x
constexpr int XP = XC + 3;  // LDS row pitch of the u tile (odd in 8-byte words: no bank conflicts on row sweeps)
constexpr int XQ = XC + 1;  // LDS row pitch of the output tile

__global__ __launch_bounds__(XL) void grad_x_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *ux,
                                                    double hx, const double *__restrict__ inv_m) {
  __shared__ double tu[XL][XP];
  __shared__ double to[XL][XQ];
  __shared__ long long ub[XL], ob[XL];  // row start of each line in u and in ux
  const int nlines = (gu.ny + 1) * (gu.nz + 1);
  const int L0 = blockIdx.x * XL;
  const int t = threadIdx.x;
  const int N = gu.nx;
  const int nl = min(XL, nlines - L0);  // lines in this workgroup
  const bool act = t < nl;
  {
    const int L = L0 + (act ? t : 0);
    const int j = L % (gu.ny + 1), k = L / (gu.ny + 1);
    ub[t] = gu.at(0, j, k);
    ob[t] = gd.at(0, j, k);
  }
  double v0 = 0.0, vN = 0.0;
  if (act) {
    const long long b = ub[t];
    v0 = end0(u[b], u[b + 1], u[b + 2], u[b + 3], u[b + 4], hx);
    vN = -end0(u[b + N], u[b + N - 1], u[b + N - 2], u[b + N - 3], u[b + N - 4], hx);
    ux[ob[t]] = v0;
    ux[ob[t] + N] = vN;
  }
  __syncthreads();
  const double s3 = 3.0 / hx;
  double dprev = 0.0;
  // forward elimination, chunk by chunk over the interior x = 1..N-1; the next chunk's u is loaded into registers
  // while the current chunk is swept
  constexpr int PER = (XL * (XC + 2) + XL - 1) / XL;  // staged values per thread and chunk
  double nxt[PER];
  auto load_chunk = [&](int x0) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = t + m * XL;
      const int ln = e / (XC + 2), xx = e % (XC + 2);
      double v = 0.0;
      if (e < XL * (XC + 2) && ln < nl && x0 - 1 + xx <= N) v = u[ub[ln] + x0 - 1 + xx];
      nxt[m] = v;
    }
  };
  load_chunk(1);
  for (int x0 = 1; x0 <= N - 1; x0 += XC) {
    const int wn = min(XC, N - x0);  // interior values in this chunk
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int e = t + m * XL;
      if (e < XL * (XC + 2)) tu[e / (XC + 2)][e % (XC + 2)] = nxt[m];
    }
    __syncthreads();
    if (x0 + XC <= N - 1) load_chunk(x0 + XC);
    if (act) {
      for (int q = 0; q < wn; ++q) {
        const int x = x0 + q;
        double rhs = s3 * (tu[t][q + 2] - tu[t][q]);
        if (x == 1) rhs -= v0;
        if (x == N - 1) rhs -= vN;
        const double d = (rhs - dprev) * inv_m[x];
        to[t][q] = d;
        dprev = d;
      }
    }
    __syncthreads();
    for (int e = t; e < XL * XC; e += XL) {
      const int ln = e / XC, xx = e % XC;
      if (ln < nl && xx < wn) ux[ob[ln] + x0 + xx] = to[ln][xx];
    }
    __syncthreads();
  }
  // back substitution over the same chunks in reverse order
  const int nchunks = (N - 1 + XC - 1) / XC;
  double vnext = 0.0;
  for (int c = nchunks - 1; c >= 0; --c) {
    const int x0 = 1 + c * XC;
    const int wn = min(XC, N - x0);
    for (int e = t; e < XL * XC; e += XL) {
      const int ln = e / XC, xx = e % XC;
      to[ln][xx] = (ln < nl && xx < wn) ? ux[ob[ln] + x0 + xx] : 0.0;
    }
    __syncthreads();
    if (act) {
      for (int q = wn - 1; q >= 0; --q) {
        const int x = x0 + q;
        const double d = to[t][q];
        const double v = (x == N - 1) ? d : d - inv_m[x] * vnext;
        to[t][q] = v;
        vnext = v;
      }
    }
    __syncthreads();
    for (int e = t; e < XL * XC; e += XL) {
      const int ln = e / XC, xx = e % XC;
      if (ln < nl && xx < wn) ux[ob[ln] + x0 + xx] = to[ln][xx];
    }
    __syncthreads();
  }
}

}  // namespace

void launch_gradient(const Grid &gu, const double *u, const Grid &gd, double *ux, double *uy, double *uz, double hx,
                     double hy, double hz, const double *inv_m_x, const double *inv_m_y, const double *inv_m_z,
                     hipStream_t st) {
  const int nlines = (gu.ny + 1) * (gu.nz + 1);
  grad_x_kernel<<<(nlines + XL - 1) / XL, XL, 0, st>>>(gu, u, gd, ux, hx, inv_m_x);
  grad_y_kernel<<<dim3((gu.nx + 1 + 63) / 64, gu.nz + 1), 64, 0, st>>>(gu, u, gd, uy, hy, inv_m_y);
  grad_z_kernel<<<dim3((gu.nx + 1 + 63) / 64, gu.ny + 1), 64, 0, st>>>(gu, u, gd, uz, hz, inv_m_z);
}

}  // namespace excmg
