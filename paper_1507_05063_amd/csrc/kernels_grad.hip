// Fourth-order compact gradient (Section 5.1) for gfx950.
//
// Along every grid line (including lines on the boundary) of length N cells, with v = du/dx (or y, z):
//   v_0 = (-25 u_0 + 48 u_1 - 36 u_2 + 16 u_3 - 3 u_4) / (12 h),  v_N the mirror image with the opposite sign,
//   v_{i-1} + 4 v_i + v_{i+1} = 3 (u_{i+1} - u_{i-1}) / h,  i = 1..N-1
// (the paper's (1/6, 4/6, 1/6) system times 6).  The constant-coefficient Thomas factors m_1 = 4,
// m_i = 4 - 1/m_{i-1} are shared by all lines; the host passes 1/m_i per axis.
#include <algorithm>

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

// x lines, one wavefront per line, by prefix scans.  Both Thomas recursions are first-order linear recurrences,
//   forward  d_t = w_t rhs_t - w_t d_{t-1}   (d_0 = 0),        back  v_t = d_t - w_t v_{t+1}   (v_{M+1} = 0),
// with w_t = 1/m_t, i.e. compositions of affine maps x -> A + B x.  The line is cut into segments of 64 XL unknowns
// and lane l of the wavefront owns unknowns t = 1 + 64 XL s + XL l + q (q < XL) of segment s: it composes the maps of
// its XL steps (running them from 0 gives A, the product of the B's gives B), a Kogge-Stone scan over the 64 lanes
// (shuffles, in lane order for the forward sweep and in reverse for the back substitution) composes the lanes' maps,
// and each lane then has the exact value entering its first step; its XL results follow as A_q + B_q x_in.  Segments
// are chained through the value leaving the last (forward) or first (back) lane.  The back substitution runs over
// the segments from the last to the first and redoes the forward sweep of every segment but the last (whose d stay
// in registers) from its stored entering value.  This is the Thomas solution, summed in another order.
// Past the last unknown the maps are x -> 0, which makes d and v vanish there.  A segment of u goes into LDS with
// contiguous loads and the lanes read their XL + 2 values from there; the results go out the same way.  LDS slots
// are padded by 2 words per 8 so that the lanes' blocks (XL apart) start on different banks.
constexpr int XL = 8;
constexpr int XSEG = 64 * XL;
constexpr int kInvM = 32;  // 1/m_t has reached its limit 1/(2 + sqrt 3) to the last bit well before t = 32

__device__ __forceinline__ void scan_lanes_up(double &A, double &B, int lane) {  // maps of lanes 0..lane
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double Ap = __shfl_up(A, off, 64), Bp = __shfl_up(B, off, 64);
    const bool take = lane >= off;
    A = take ? A + B * Ap : A;
    B = take ? B * Bp : B;
  }
}

__device__ __forceinline__ void scan_lanes_down(double &A, double &B, int lane) {  // maps of lanes lane..63
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const double An = __shfl_down(A, off, 64), Bn = __shfl_down(B, off, 64);
    const bool take = lane + off < 64;
    A = take ? A + B * An : A;
    B = take ? B * Bn : B;
  }
}

__device__ __forceinline__ int xslot(int e) { return e + 2 * (e >> 3); }
constexpr int kXBuf = XSEG + 2 + 2 * ((XSEG + 2) >> 3) + 2;  // slots of u at t0-1 .. t0+XSEG

__global__ __launch_bounds__(64) void grad_x_scan_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *ux,
                                                         double hx, const double *__restrict__ inv_m) {
  __shared__ double buf[kXBuf];
  __shared__ double wt[kInvM + 1];
  extern __shared__ double seg_in[];  // d entering each segment
  const int N = gu.nx, M = N - 1;
  const int lane = threadIdx.x;
  const int L = blockIdx.x;
  const int j = L % (gu.ny + 1), k = L / (gu.ny + 1);
  const long long b = gu.at(0, j, k), ob = gd.at(0, j, k);
  const int wlast = min(M, kInvM);
  if (lane <= kInvM) wt[lane] = inv_m[min(max(lane, 1), wlast)];
  const double v0 = end0(u[b], u[b + 1], u[b + 2], u[b + 3], u[b + 4], hx);
  const double vN = -end0(u[b + N], u[b + N - 1], u[b + N - 2], u[b + N - 3], u[b + N - 4], hx);
  if (lane == 0) {
    ux[ob] = v0;
    ux[ob + N] = vN;
  }
  const double s3 = 3.0 / hx;
  const int nseg = (M + XSEG - 1) / XSEG;
  auto W = [&](int t) { return wt[min(t, kInvM)]; };  // 1/m_t (t >= 1; entries past wlast repeat it)

  // u of segment s into buf (slot e: x = 64 XL s + e), then the lane's composite forward map (A, B)
  auto forward_map = [&](int s, double &A, double &B) {
    const int base = s * XSEG;
    __syncthreads();  // earlier reads of buf are done
#pragma unroll
    for (int m = 0; m < (XSEG + 2 + 63) / 64; ++m) {
      const int e = lane + 64 * m;
      if (e < XSEG + 2) buf[xslot(e)] = u[b + min(base + e, N)];
    }
    __syncthreads();
    const int tb = 1 + base + lane * XL;
    double d = 0.0, pr = 1.0, um = buf[xslot(lane * XL)], uc = buf[xslot(lane * XL + 1)];
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int t = tb + q;
      const double up = buf[xslot(lane * XL + q + 2)];
      double rhs = s3 * (up - um);
      rhs = (t == 1) ? rhs - v0 : rhs;
      rhs = (t == M) ? rhs - vN : rhs;
      const double w = W(t);
      const bool ok = t <= M;
      d = ok ? w * (rhs - d) : 0.0;
      pr = ok ? -w * pr : 0.0;
      um = uc;
      uc = up;
    }
    A = d;
    B = pr;
  };
  // the exact d of the lane's unknowns (replayed from the scanned entering value); returns d leaving the segment
  double dd[XL];
  auto forward_fix = [&](int s, double A, double B, double din_seg) {
    scan_lanes_up(A, B, lane);
    const double dend = A + B * din_seg;
    double d = __shfl_up(dend, 1, 64);
    d = lane == 0 ? din_seg : d;
    const int tb = 1 + s * XSEG + lane * XL;
    double um = buf[xslot(lane * XL)], uc = buf[xslot(lane * XL + 1)];
#pragma unroll
    for (int q = 0; q < XL; ++q) {
      const int t = tb + q;
      const double up = buf[xslot(lane * XL + q + 2)];
      double rhs = s3 * (up - um);
      rhs = (t == 1) ? rhs - v0 : rhs;
      rhs = (t == M) ? rhs - vN : rhs;
      d = (t <= M) ? W(t) * (rhs - d) : 0.0;
      dd[q] = d;
      um = uc;
      uc = up;
    }
    return __shfl(dend, 63, 64);
  };

  double carry = 0.0;
  for (int s = 0; s < nseg; ++s) {
    if (lane == 0) seg_in[s] = carry;
    double A, B;
    forward_map(s, A, B);
    carry = forward_fix(s, A, B, carry);
  }
  double vcarry = 0.0;  // v just past the segment
  for (int s = nseg - 1; s >= 0; --s) {
    if (s < nseg - 1) {
      double A, B;
      forward_map(s, A, B);
      forward_fix(s, A, B, seg_in[s]);
    }
    const int tb = 1 + s * XSEG + lane * XL;
    double v = 0.0, pr = 1.0;
#pragma unroll
    for (int q = XL - 1; q >= 0; --q) {
      const int t = tb + q;
      const bool ok = t <= M;
      const double w = W(t);
      v = ok ? dd[q] - w * v : 0.0;
      pr = ok ? -w * pr : 0.0;
    }
    double A = v, B = pr;
    scan_lanes_down(A, B, lane);
    const double vfirst = A + B * vcarry;
    v = __shfl_down(vfirst, 1, 64);
    v = lane == 63 ? vcarry : v;
    __syncthreads();  // the lanes' reads of buf are done
#pragma unroll
    for (int q = XL - 1; q >= 0; --q) {
      const int t = tb + q;
      v = (t <= M) ? dd[q] - W(t) * v : 0.0;
      buf[xslot(lane * XL + q)] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < XL; ++m) {
      const int e = lane + 64 * m, t = 1 + s * XSEG + e;
      if (t <= M) __builtin_nontemporal_store(buf[xslot(e)], &ux[ob + t]);
    }
    vcarry = __shfl(vfirst, 0, 64);
  }
}

// x lines of at most 64 XL unknowns (one segment), several lines per wavefront: the lanes load the next line's u
// into registers while the current line is solved, so the read latency of one line overlaps the work of the last.
// Every global access is unconditional (clamped indices; lanes past the last unknown store its value again), which
// lets the compiler wait for just the loads it needs instead of draining all of them.
constexpr int kXFetch = (XSEG + 2 + 63) / 64;  // u values per lane and line

__global__ __launch_bounds__(64) void grad_x_short_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *ux,
                                                          double hx, const double *__restrict__ inv_m) {
  __shared__ double buf[kXBuf];
  __shared__ double wt[kInvM + 1];
  const int N = gu.nx, M = N - 1;
  const int lane = threadIdx.x;
  const int nlines = (gu.ny + 1) * (gu.nz + 1);
  const int wlast = min(M, kInvM);
  if (lane <= kInvM) wt[lane] = inv_m[min(max(lane, 1), wlast)];
  const double s3 = 3.0 / hx;
  auto W = [&](int t) { return wt[min(t, kInvM)]; };
  double pf[kXFetch];
  auto fetch = [&](int L) {  // u of line L (clamped to the last line) at x = min(lane + 64 m, N)
    L = min(L, nlines - 1);
    const long long bb = gu.at(0, L % (gu.ny + 1), L / (gu.ny + 1));
#pragma unroll
    for (int m = 0; m < kXFetch; ++m) pf[m] = u[bb + min(lane + 64 * m, N)];
  };
  fetch(blockIdx.x);
  for (int L = blockIdx.x; L < nlines; L += gridDim.x) {
    const long long ob = gd.at(0, L % (gu.ny + 1), L / (gu.ny + 1));
    __syncthreads();  // the previous line's reads of buf are done
#pragma unroll
    for (int m = 0; m < kXFetch; ++m) buf[xslot(min(lane + 64 * m, XSEG + 1))] = pf[m];  // slot x: u at min(x, N)
    fetch(L + gridDim.x);
    __syncthreads();
    const double v0 = end0(buf[xslot(0)], buf[xslot(1)], buf[xslot(2)], buf[xslot(3)], buf[xslot(4)], hx);
    const double vN = -end0(buf[xslot(N)], buf[xslot(N - 1)], buf[xslot(N - 2)], buf[xslot(N - 3)],
                            buf[xslot(N - 4)], hx);
    const int tb = 1 + lane * XL;
    // forward: the lane's composite map, the scan, then the replay from the exact entering d
    double d = 0.0, pr = 1.0;
    {
      double um = buf[xslot(lane * XL)], uc = buf[xslot(lane * XL + 1)];
#pragma unroll
      for (int q = 0; q < XL; ++q) {
        const int t = tb + q;
        const double up = buf[xslot(lane * XL + q + 2)];
        double rhs = s3 * (up - um);
        rhs = (t == 1) ? rhs - v0 : rhs;
        rhs = (t == M) ? rhs - vN : rhs;
        const double w = W(t);
        const bool ok = t <= M;
        d = ok ? w * (rhs - d) : 0.0;
        pr = ok ? -w * pr : 0.0;
        um = uc;
        uc = up;
      }
    }
    double A = d, B = pr;
    scan_lanes_up(A, B, lane);
    d = __shfl_up(A, 1, 64);  // d entering the lane (the segment starts from d_0 = 0)
    d = lane == 0 ? 0.0 : d;
    double dd[XL];
    {
      double um = buf[xslot(lane * XL)], uc = buf[xslot(lane * XL + 1)];
#pragma unroll
      for (int q = 0; q < XL; ++q) {
        const int t = tb + q;
        const double up = buf[xslot(lane * XL + q + 2)];
        double rhs = s3 * (up - um);
        rhs = (t == 1) ? rhs - v0 : rhs;
        rhs = (t == M) ? rhs - vN : rhs;
        d = (t <= M) ? W(t) * (rhs - d) : 0.0;
        dd[q] = d;
        um = uc;
        uc = up;
      }
    }
    // back substitution: the same with the maps of v_t = d_t - w_t v_{t+1}, lanes in reverse
    double v = 0.0;
    pr = 1.0;
#pragma unroll
    for (int q = XL - 1; q >= 0; --q) {
      const int t = tb + q;
      const bool ok = t <= M;
      const double w = W(t);
      v = ok ? dd[q] - w * v : 0.0;
      pr = ok ? -w * pr : 0.0;
    }
    A = v;
    B = pr;
    scan_lanes_down(A, B, lane);
    v = __shfl_down(A, 1, 64);  // v entering the lane from above (v_{M+1} = 0)
    v = lane == 63 ? 0.0 : v;
    __syncthreads();  // the lanes' reads of buf are done
#pragma unroll
    for (int q = XL - 1; q >= 0; --q) {
      const int t = tb + q;
      v = (t <= M) ? dd[q] - W(t) * v : 0.0;
      buf[xslot(lane * XL + q)] = v;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < XL; ++m) {
      const int t = min(1 + lane + 64 * m, M);
      __builtin_nontemporal_store(buf[xslot(t - 1)], &ux[ob + t]);
    }
    __builtin_nontemporal_store(v0, &ux[ob]);
    __builtin_nontemporal_store(vN, &ux[ob + N]);
  }
}

// y and z lines: one thread per line, consecutive threads on consecutive x, so every step of the sweeps is a
// coalesced row access.  The lines are numbered x fastest, then the other cross axis (k for y lines, j for z lines),
// and a wavefront takes 64 consecutive numbers (at a row end the rest of the wavefront goes on with the next row), so
// that no wavefront is left with the one or few lines past the last full 64 of a row: every wavefront runs a whole
// line's length whatever its lines.  Wavefront numbers are dealt XCD by XCD (the hardware hands consecutive
// workgroups to the 8 XCDs in turn), so that neighbouring wavefronts, whose row segments meet inside cache lines of
// the caller's unpadded rows, write them from one XCD's L2.
constexpr int kXcd = 8;
constexpr int kLineWg = 64;

// logical wavefront of workgroup b of nb: consecutive logical numbers on one XCD
__device__ __forceinline__ int xcd_wave(int b, int nb) {
  const int per = nb / kXcd, rem = nb % kXcd;
  const int x = b % kXcd, l = b / kXcd;
  return ((x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + l;
}

__global__ __launch_bounds__(kLineWg) void grad_y_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *uy,
                                                         double hy, const double *__restrict__ inv_m) {
  const long long line = (long long)xcd_wave(blockIdx.x, gridDim.x) * kLineWg + threadIdx.x;
  const int nxl = gu.nx + 1;
  if (line >= (long long)nxl * (gu.nz + 1)) return;
  const int i = (int)(line % nxl), k = (int)(line / nxl);
  line_solve(u, gu.at(i, 0, k), gu.sy, uy, gd.at(i, 0, k), gd.sy, gu.ny, hy, inv_m);
}

__global__ __launch_bounds__(kLineWg) void grad_z_kernel(Grid gu, const double *__restrict__ u, Grid gd, double *uz,
                                                         double hz, const double *__restrict__ inv_m) {
  const long long line = (long long)xcd_wave(blockIdx.x, gridDim.x) * kLineWg + threadIdx.x;
  const int nxl = gu.nx + 1;
  if (line >= (long long)nxl * (gu.ny + 1)) return;
  const int i = (int)(line % nxl), j = (int)(line / nxl);
  line_solve(u, gu.at(i, j, 0), gu.sz, uz, gd.at(i, j, 0), gd.sz, gu.nz, hz, inv_m);
}

}  // namespace

void launch_gradient(const Grid &gu, const double *u, const Grid &gd, double *ux, double *uy, double *uz, double hx,
                     double hy, double hz, const double *inv_m_x, const double *inv_m_y, const double *inv_m_z,
                     hipStream_t st) {
  const int nlines = (gu.ny + 1) * (gu.nz + 1);
  const int nseg = (gu.nx - 1 + XSEG - 1) / XSEG;
  if (nseg == 1)  // about 8 lines per wavefront, 32 wavefronts per CU at most
    grad_x_short_kernel<<<std::min(nlines, 8192), 64, 0, st>>>(gu, u, gd, ux, hx, inv_m_x);
  else
    grad_x_scan_kernel<<<nlines, 64, (size_t)nseg * sizeof(double), st>>>(gu, u, gd, ux, hx, inv_m_x);
  const long long ylines = (long long)(gu.nx + 1) * (gu.nz + 1), zlines = (long long)(gu.nx + 1) * (gu.ny + 1);
  grad_y_kernel<<<(int)((ylines + kLineWg - 1) / kLineWg), kLineWg, 0, st>>>(gu, u, gd, uy, hy, inv_m_y);
  grad_z_kernel<<<(int)((zlines + kLineWg - 1) / kLineWg), kLineWg, 0, st>>>(gu, u, gd, uz, hz, inv_m_z);
}

}  // namespace excmg
