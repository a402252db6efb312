// Conjugate-gradient kernels of the EXCMG relaxation (Algorithm 1, the CG loop on each grid) for gfx950.
//
// One CG iteration is two bandwidth-bound sweeps separated by the two global reductions CG needs:
//   pass A:  p = r + beta p_old (beta = 0 on the first iteration), partial sums of p.Mp       reads r, p_old; writes p
//   pass B:  u += alpha p, r -= alpha Mp, partial sums of r.r                                 reads p, r, u;  writes r, u
// Mp is evaluated in both passes from p staged in LDS, so no q vector is stored: 64 B per unknown and iteration in
// FP64 (32 B in FP32) instead of the 80 B of the textbook q-storing form.  The direction vector is double-buffered,
// because pass A reads p_old with halos while it writes p.  On the first iteration p = r is not written out: pass A
// reads r only (8 B) and pass B takes both operands from r's buffer and writes the new r into another (32 B); the
// buffers then rotate as cg_bufs describes.
//
// Stencil sweep ("z-march"): a workgroup owns a TX x TY column tile (64 x 4, 8 or 16 nodes, one thread per node; the
// CG passes take the height per grid from the autotuner, the other sweeps use 4) and a chunk of z planes.  For each plane it loads
// the (TX+2) x (TY+2) tile with its halo into LDS (double-buffered, one barrier per plane) and every thread forms the
// plane sums of its column: centre C, x-pair X, y-pair Y, xy-diagonals D.  The 19-point result at plane k is
//   c0 C_k + cx X_k + cy Y_k + cxy D_k + cz (C_{k-1} + C_{k+1}) + cxz (X_{k-1} + X_{k+1}) + cyz (Y_{k-1} + Y_{k+1}),
// so each plane's global data is read once per workgroup and the z-neighbours come from registers.  The next plane
// is fetched into registers before the current one is reduced, to keep loads in flight.
//
// Workgroups are numbered so that consecutive tiles of one z chunk run on the same XCD (dispatch is round-robin over
// the 8 XCDs), which keeps the y-halo rows shared by neighbouring tiles in that XCD's L2.
//
// Reductions: wavefront butterfly (xor shuffles), then one value per wave through LDS, one partial per workgroup;
// a single-workgroup finalize kernel sums the partials in a fixed order and updates the CG scalars (alpha, beta, the
// stopping test) on the device.  Results are bitwise reproducible.
#include <math.h>

#include <type_traits>
#include <utility>

#include "excmg_internal.h"

namespace excmg {

namespace {

constexpr int kXcds = 8;

// Bijection from the hardware workgroup id to a logical tile id such that logical ids [x*per, (x+1)*per) run on XCD x.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int per = nb / kXcds, rem = nb % kXcds;
  const int x = b % kXcds, l = b / kXcds;
  const int start = (x < rem) ? x * (per + 1) : rem * (per + 1) + (x - rem) * per;
  return start + l;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum over the workgroup, deterministic; the result is valid in thread 0.
template <int NT>
__device__ __forceinline__ double block_sum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < (NT + 63) / 64; ++q) t += sh[q];
  }
  return t;
}

// Tile shape of the stencil sweeps (x is the fast axis: one wavefront covers one 64-node row segment).
constexpr int TX = 64;
// Threads of a workgroup with tile height TY, and the rows of one LDS plane buffer: the (TX+2) x (TY+2) tile with its
// halo, padded so that every fetch slot of the workgroup (a whole number of slots per thread) has an entry and the
// staging stores need no bounds test.  A taller tile re-reads fewer halo rows per node (2 per TY rows); a shorter one
// gives small grids more workgroups.
template <int TY>
struct Tile {
  static constexpr int NT = TX * TY;
  static constexpr int Rows = ((TX + 2) * (TY + 2) + NT - 1) / NT * NT / (TX + 2) + 1;
};
template <int TY>
constexpr bool height_ok() { return TY == 4 || TY == 8 || TY == 16; }
// the height of every sweep but the CG passes of a single problem (residuals, batched launches, operator apply)
constexpr int kTy = 4;
constexpr int NT = Tile<kTy>::NT;
constexpr int kTileRows = Tile<kTy>::Rows;

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Loads and stores of data a sweep touches once: non-temporal (streaming) when NTP, so that they do not displace the
// operand's halo lines, which neighbouring tiles read again, from the caches.
template <bool NTP, typename T>
__device__ __forceinline__ T ld1(const T *p) {
  if constexpr (NTP) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NTP, typename T>
__device__ __forceinline__ void st1(T v, T *p) {
  if constexpr (NTP) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// f(integral_constant<int, 0>), ..., f(integral_constant<int, N - 1>), in that order
template <typename F, int... Q>
__device__ __forceinline__ void static_for_impl(F &&f, std::integer_sequence<int, Q...>) {
  (f(std::integral_constant<int, Q>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F &&f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

// Prefetch depths the z-march is built for.  Deeper prefetch keeps more bytes in flight per thread, which the FP32
// sweeps need (half the bytes per load of FP64 at the same latency); it costs registers.
constexpr int kMaxDepth = 6;
template <int D>
constexpr bool depth_ok() { return D == 2 || D == 3 || D == 4 || D == 6; }

// The z-march.  P supplies operand(idx) (the raw loads of the stencil operand at an interior node, idx in grid g, of
// type P::Raw) and value(raw) (the operand formed from them when the plane is staged in LDS, so that no arithmetic
// waits on a load while later planes are being fetched),
// center<S>(i,j,k,idx) (load of the thread's own data for output plane k into slot S) and
// consume<S>(i,j,k,idx,C,out,cf,rf,acc0,acc1) (output plane k, data in slot S).  Both the stencil planes and the centre
// data are requested D planes ahead of their use, so D planes' worth of loads are in flight per thread while a
// plane is reduced.  The steps are unrolled in rounds of lcm(2, D) so that the LDS buffer (step parity), the
// register set and the centre slot (step mod D) of every step are compile-time constants.
// If P::kRhs, a second array (the finest f at the level's stride) is staged the same way in tileF and the 7-point
// average R f = (6 f_c + sum of the 6 face neighbours)/2 of the output plane is handed to consume as rf (with the
// centre value cf), so the right-hand side is formed with f read once.
// bid, nb: this workgroup's index among the nb workgroups of the sweep (the grid of a single-problem launch, or one
// problem's range of a batched launch); remap: number the tiles XCD by XCD (single-problem launches only, where the
// hardware's round-robin dispatch over the XCDs follows bid).
template <typename T, int D = 2, int TY = kTy, typename P>
__device__ __forceinline__ void zmarch(const Sweep &sw, P &pol, double &acc0, double &acc1,
                                       T (*tile)[Tile<TY>::Rows][TX + 2], double (*tileF)[Tile<TY>::Rows][TX + 2],
                                       int bid, int nb, bool remap) {
  static_assert(depth_ok<D>(), "prefetch depth");
  static_assert(height_ok<TY>(), "tile height");
  constexpr int NT = Tile<TY>::NT;
  constexpr int W = TX + 2, H = TY + 2, E = W * H, NL = (E + NT - 1) / NT;
  static_assert(NL * NT <= Tile<TY>::Rows * W, "every fetch slot has an LDS entry");
  constexpr int U = D % 2 == 0 ? D : 2 * D;  // steps per unrolled round: a multiple of both 2 (LDS buffers) and D
  constexpr bool R = P::kRhs;
  const Grid &g = sw.g;
  const int t = remap ? xcd_remap(bid, nb) : bid;
  const int bx = t % sw.ntx;
  const int rest = t / sw.ntx;
  const int by = rest % sw.nty;
  const int bz = rest / sw.nty;
  const int i0 = 1 + bx * TX, j0 = 1 + by * TY, k0 = 1 + bz * sw.zc;
  const int k1 = min(k0 + sw.zc, g.nz);  // output planes [k0, k1)
  const int tid = threadIdx.x;
  const int lx = tid % TX, ly = tid / TX;
  const int i = i0 + lx, j = j0 + ly;
  const bool active = (i < g.nx) && (j < g.ny);

  // Every load is issued unconditionally, from an address clamped into the interior (or, for f, into the grid), and
  // what lies outside is zeroed by a select when the plane is staged: with no branch around a load the compiler can
  // wait for each plane's loads alone instead of draining all of them.  Per fetch slot: column offset of its
  // (clamped) node and whether the node is interior in x and y; for f, any node of the grid.
  long long col[NL], colF[NL];
  bool cin[NL], fin[NL];
#pragma unroll
  for (int m = 0; m < NL; ++m) {
    const int e = tid + m * NT;
    const int ee = e < E ? e : E - 1;
    const int gi = i0 - 1 + ee % W, gj = j0 - 1 + ee / W;
    cin[m] = e < E && gi >= 1 && gi < g.nx && gj >= 1 && gj < g.ny;
    col[m] = g.off + (long long)clampi(gj, 1, g.ny - 1) * g.sy + clampi(gi, 1, g.nx - 1);
    fin[m] = e < E && gi <= g.nx && gj <= g.ny;
    colF[m] = R ? pol.fcol(min(gi, g.nx), min(gj, g.ny)) : 0;
  }
  const long long fstride = R ? pol.fplane() : 0;
  using Raw = typename P::Raw;
  Raw reg[D][NL];
  double fre[D][NL];
  auto fetch = [&](Raw(&rg)[NL], double(&fr)[NL], int kk) {  // planes past the chunk load a clamped, unused plane
    const long long pk = (long long)clampi(kk, 1, g.nz - 1) * g.sz;
#pragma unroll
    for (int m = 0; m < NL; ++m) rg[m] = pol.operand(col[m] + pk);
    if constexpr (R) {
      const long long pf = (long long)min(kk, g.nz) * fstride;
#pragma unroll
      for (int m = 0; m < NL; ++m) fr[m] = pol.fval(colF[m] + pf);
    }
  };

  const Stencil &st = sw.st;
  const T c0 = (T)st.c0, cx = (T)st.cx, cy = (T)st.cy, cz = (T)st.cz;
  const T cxy = (T)st.cxy, cxz = (T)st.cxz, cyz = (T)st.cyz;
  T Cm = 0, Xm = 0, Ym = 0, Cc = 0, Xc = 0, Yc = 0, Pc = 0;
  double Fm = 0.0, Fc = 0.0, Gc = 0.0;  // f: centre of the previous and current plane, in-plane face sum
  // the thread's own column, clamped into the interior (inactive threads load but never consume)
  const long long own = g.off + (long long)min(j, g.ny - 1) * g.sy + min(i, g.nx - 1);
  const int np = k1 - k0 + 2;  // planes k0-1 .. k1
  auto center_at = [&](auto sc, int k) {  // centre data of output plane k (clamped to the chunk) into slot sc
    pol.template center<decltype(sc)::value>(i, j, k, own + (long long)min(k, k1 - 1) * g.sz);
  };

  // Step s (plane kk = k0-1+s) takes the operand from register set s%D, stages it in LDS buffer s%2, refills the set
  // with plane kk+D, and (s >= 2) produces output plane kk-1 from the centre data in slot s%D, which it then refills
  // for output plane kk-1+D.
#pragma unroll
  for (int d = 0; d < D; ++d) fetch(reg[d], fre[d], k0 - 1 + d);
  // output plane k0 + m is produced at step m + 2, from centre slot (m + 2) mod D
  static_for<D>([&](auto mc) {
    constexpr int m = decltype(mc)::value;
    center_at(std::integral_constant<int, (m + 2) % D>{}, k0 + m);
  });

  // produce: compile-time step >= 2 (false only in the first round)
  auto body = [&](auto pb, auto pr, auto produce, int step) {
    constexpr int PB = decltype(pb)::value;  // LDS buffer of the step: step % 2
    constexpr int PR = decltype(pr)::value;  // register set and centre slot of the step: step % D
    T(*tb)[TX + 2] = tile[PB];
    T *tl = &tile[PB][0][0];
    const int kk = k0 - 1 + step;
    const bool kin = (kk >= 1) && (kk < g.nz);
#pragma unroll
    for (int m = 0; m < NL; ++m) tl[tid + m * NT] = (kin && cin[m]) ? pol.value(reg[PR][m]) : T(0);
    if constexpr (R) {
      double *tfl = &tileF[PB][0][0];
#pragma unroll
      for (int m = 0; m < NL; ++m) tfl[tid + m * NT] = fin[m] ? fre[PR][m] : 0.0;
    }
    __syncthreads();
    fetch(reg[PR], fre[PR], kk + D);
    const T c = tb[ly + 1][lx + 1];
    const T x = tb[ly + 1][lx] + tb[ly + 1][lx + 2];
    const T y = tb[ly][lx + 1] + tb[ly + 2][lx + 1];
    const T d = (tb[ly][lx] + tb[ly][lx + 2]) + (tb[ly + 2][lx] + tb[ly + 2][lx + 2]);
    double fc = 0.0, fg = 0.0;
    if constexpr (R) {
      double(*tf)[TX + 2] = tileF[PB];
      fc = tf[ly + 1][lx + 1];
      fg = (tf[ly + 1][lx] + tf[ly + 1][lx + 2]) + (tf[ly][lx + 1] + tf[ly + 2][lx + 1]);
    }
    if constexpr (decltype(produce)::value) {
      if (active) {
        const T out = Pc + cz * (Cm + c) + cxz * (Xm + x) + cyz * (Ym + y);
        const double rf = 0.5 * (6.0 * Fc + (Gc + (Fm + fc)));
        pol.template consume<PR>(i, j, kk - 1, own + (long long)(kk - 1) * g.sz, Cc, out, Fc, rf, acc0, acc1);
      }
      center_at(pr, kk - 1 + D);  // past the chunk: a clamped, unused load
    }
    Cm = Cc; Xm = Xc; Ym = Yc;
    Cc = c; Xc = x; Yc = y;
    Pc = c0 * c + cx * x + cy * y + cxy * d;
    Fm = Fc; Fc = fc; Gc = fg;
  };
  // First round (steps 0 and 1 only stage), whole rounds without bounds tests, then the tail.
  static_for<U>([&](auto sc) {
    constexpr int q = decltype(sc)::value;
    if (q < np) body(std::integral_constant<int, q % 2>{}, std::integral_constant<int, q % D>{}, std::bool_constant<(q >= 2)>{}, q);
  });
  int step = U;
  for (; step + U <= np; step += U) {
    static_for<U>([&](auto sc) {
      constexpr int q = decltype(sc)::value;
      body(std::integral_constant<int, q % 2>{}, std::integral_constant<int, q % D>{}, std::true_type{}, step + q);
    });
  }
  static_for<U>([&](auto sc) {
    constexpr int q = decltype(sc)::value;
    if (step + q < np) body(std::integral_constant<int, q % 2>{}, std::integral_constant<int, q % D>{}, std::true_type{}, step + q);
  });
}

// ---------------------------------------------------------------------------------------- grid-wide reductions
//
// Every workgroup writes its K partial sums to partials[k * nblocks + block]; a single-workgroup finalize kernel that
// runs next on the stream sums them in block order and updates the CG state.  The kernel boundary orders the two;
// no workgroup of a sweep fences or synchronises with another (on this GPU an agent-scope fence writes back and
// invalidates the XCD's L2, far too costly to issue from every workgroup).
template <int K, int NTB = NT>
__device__ __forceinline__ void write_partials(const double (&v)[K], double *partials, double *sh, int bid, int nb) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = block_sum<NTB>(v[k], sh);
    if (threadIdx.x == 0) partials[(long long)k * nb + bid] = s;
    __syncthreads();
  }
}

constexpr int FT = 1024;

// Strided part of a fixed-order sum: thread t adds a[t], a[t + W], a[t + 2W], ... in that order.  Eight loads are
// issued before their adds so that the loop is not one memory latency per element; the order of the adds, and so
// the result, is that of the plain loop.
template <int W>
__device__ __forceinline__ double strided_sum(const double *a, int n) {
  double v = 0.0;
  int q = threadIdx.x;
  for (; q + 7 * W < n; q += 8 * W) {
    double x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) x[u] = a[q + u * W];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += x[u];
  }
  for (; q < n; q += W) v += a[q];
  return v;
}

// fixed-order sum of n partials by one workgroup of FT threads; the result is valid in every thread
__device__ double fixed_sum(const double *a, int n, double *sh) {
  const double t = block_sum<FT>(strided_sum<FT>(a, n), sh);
  if (threadIdx.x == 0) sh[FT / 64] = t;
  __syncthreads();
  const double s = sh[FT / 64];
  __syncthreads();
  return s;
}

// ------------------------------------------------------------------------------------------------ state updates

__device__ void state_init(CgState *cs, double rho, double bb, double tol, int max_iters, int hist_on) {
  cs->rho = rho;
  cs->rho_old = rho;
  cs->rho0 = rho;
  cs->bnorm2 = bb;
  cs->stop2 = tol * tol * bb;
  cs->alpha = 0.0;
  cs->beta = 0.0;
  cs->pq = 0.0;
  cs->iter = 0;
  cs->status = 0;
  cs->max_iters = max_iters;
  cs->hist_on = hist_on;
  const bool finite = isfinite(rho) && isfinite(bb);
  cs->done = (!finite || rho <= cs->stop2) ? 1 : 0;
  if (!finite) cs->status = EXCMG_ERR_BREAKDOWN;
  if (hist_on) cs->hist[0] = bb > 0.0 ? sqrt(rho / bb) : 0.0;
}

// pass A: alpha = rho / p.Mp
__device__ void state_after_a(CgState *cs, double pq) {
  cs->pq = pq;
  if (!(pq > 0.0) || !isfinite(pq)) {
    cs->status = EXCMG_ERR_BREAKDOWN;
    cs->done = 1;
  } else {
    cs->alpha = cs->rho / pq;
  }
}

// pass B: beta = rho_new / rho, stopping test ||r|| <= tol ||b|| (Algorithm 1, the while condition)
__device__ void state_after_b(CgState *cs, double rho) {
  cs->rho_old = cs->rho;
  cs->rho = rho;
  cs->beta = rho / cs->rho_old;
  const int it = cs->iter + 1;
  cs->iter = it;
  if (cs->hist_on && it < EXCMG_MAX_HISTORY) cs->hist[it] = cs->bnorm2 > 0.0 ? sqrt(rho / cs->bnorm2) : 0.0;
  if (!isfinite(rho)) {
    cs->status = EXCMG_ERR_BREAKDOWN;
    cs->done = 1;
  } else if (rho <= cs->stop2) {
    cs->done = 1;
  } else if (it >= cs->max_iters) {
    cs->status = EXCMG_ERR_NOCONV;
    cs->done = 1;
  }
}

// Start of an outer step of FP32-in-FP64 iterative refinement.  outer: the FP64 residual test ||r|| <= tol ||b||;
// inner: the FP32 CG on M d = r32 from d = 0, which stops at ||r_inner|| <= max(eta ||r32||, theta tol ||b||): it
// reduces the residual no further than the outer test needs (with margin theta = 1/2), and no further than eta, the
// reduction one FP32 solve is asked for.
__device__ void state_ir(CgState *outer, CgState *inner, double r64, double bb, double r32, double tol, double eta,
                         int outer_step, int max_outer, int max_inner) {
  outer->rho = r64;
  outer->bnorm2 = bb;
  outer->stop2 = tol * tol * bb;
  outer->iter = outer_step;
  outer->status = 0;
  outer->done = 0;
  if (!isfinite(r64) || !isfinite(bb)) {
    outer->status = EXCMG_ERR_BREAKDOWN;
    outer->done = 1;
  } else if (r64 <= outer->stop2) {
    outer->done = 1;
  } else if (outer_step >= max_outer) {
    outer->status = EXCMG_ERR_NOCONV;
    outer->done = 1;
  }
  inner->rho = r32;
  inner->rho_old = r32;
  inner->rho0 = r32;
  inner->bnorm2 = r32;
  const double theta = 0.5;
  inner->stop2 = fmax(eta * eta * r32, theta * theta * outer->stop2);
  inner->alpha = 0.0;
  inner->beta = 0.0;
  inner->pq = 0.0;
  inner->iter = 0;
  inner->status = 0;
  inner->max_iters = max_inner;
  inner->hist_on = 0;
  inner->done = (outer->done || !(r32 > 0.0)) ? 1 : 0;
  inner->iterA = 0;
  inner->iterB = 0;
  inner->preset = 1;  // a self-finalizing inner solve takes rho and stop2 from here
}

// ---------------------------------------------------------------------------------------------------------- passes

// Buffers of CG iteration k, given r's buffer R and two more, P0 and P1.  Iteration 0 has p = r (beta = 0): pass A
// writes no p (it only forms p.Mp from r), and pass B takes p from R and writes the new residual into P0, which holds
// r from then on.  Later directions alternate between P1 (odd k) and R (even k), so pass A of iteration k reads
// p_{k-1} from the buffer it does not write.  The iterates are those of p_0 = r_0 written out; one vector write and
// one vector read less on every grid.
template <typename T>
struct CgBufs {
  T *r_in;   // r_k (read by both passes)
  T *r_out;  // r_{k+1} (written by pass B)
  T *p_old;  // p_{k-1} (pass A; R at k = 0, where it is not used)
  T *p;      // p_k (written by pass A unless k = 0, read by pass B)
};

template <typename T>
__device__ __forceinline__ CgBufs<T> cg_bufs(int k, T *R, T *P0, T *P1) {
  CgBufs<T> b;
  b.r_in = (k == 0) ? R : P0;
  b.r_out = P0;
  b.p_old = (k == 0 || (k & 1)) ? R : P1;
  b.p = (k == 0) ? R : ((k & 1) ? P1 : R);
  return b;
}

// FIRST: iteration 0, where p = r: the operand is r alone (one load per node) and p is not stored.
template <typename T, bool NTP = false, bool FIRST = false>
struct PolA {
  static constexpr bool kRhs = false;
  const T *r;
  const T *pold;
  T *pnew;
  T beta;
  struct Pair {
    T r, p;
  };
  using Raw = std::conditional_t<FIRST, T, Pair>;
  __device__ __forceinline__ Raw operand(long long idx) const {
    if constexpr (FIRST) {
      return r[idx];
    } else {
      Pair v;
      v.r = r[idx];
      v.p = pold[idx];
      return v;
    }
  }
  __device__ __forceinline__ T value(const Raw &v) const {
    if constexpr (FIRST) return v;
    else return v.r + beta * v.p;
  }
  __device__ __forceinline__ long long fcol(int, int) const { return -1; }
  __device__ __forceinline__ long long fplane() const { return 0; }
  __device__ __forceinline__ double fval(long long) const { return 0.0; }
  template <int S>
  __device__ __forceinline__ void center(int, int, int, long long) {}
  template <int S>
  __device__ __forceinline__ void consume(int, int, int, long long idx, T c, T out, double, double, double &acc0,
                                          double &) {
    if constexpr (!FIRST) st1<NTP>(c, &pnew[idx]);
    acc0 += (double)c * (double)out;
  }
};

// pass A's z-march of iteration it: the first iteration's form (r alone) or the general one
template <typename T, int D, bool NTP, int TY = kTy>
__device__ __forceinline__ void pass_a_march(const Sweep &sw, int it, const CgBufs<T> &bf, T beta, double &a0,
                                             T (*tile)[Tile<TY>::Rows][TX + 2], int bid, int nb, bool remap) {
  double a1 = 0.0;
  if (it == 0) {
    PolA<T, NTP, true> pol;
    pol.r = bf.r_in;
    pol.pold = bf.r_in;
    pol.pnew = bf.p;
    pol.beta = T(0);
    zmarch<T, D, TY>(sw, pol, a0, a1, tile, nullptr, bid, nb, remap);
  } else {
    PolA<T, NTP, false> pol;
    pol.r = bf.r_in;
    pol.pold = bf.p_old;
    pol.pnew = bf.p;
    pol.beta = beta;
    zmarch<T, D, TY>(sw, pol, a0, a1, tile, nullptr, bid, nb, remap);
  }
}

template <typename T, int D, bool NTP, int TY>
__global__ __launch_bounds__(Tile<TY>::NT) void cg_pass_a_kernel(Sweep sw, T *r, T *p0, T *p1,
                                                                 const CgState *cs, double *partials) {
  __shared__ T tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[Tile<TY>::NT / 64];
  if (cs->done) return;
  const int it = cs->iter;
  const CgBufs<T> bf = cg_bufs(it, r, p0, p1);
  double a0 = 0.0;
  pass_a_march<T, D, NTP, TY>(sw, it, bf, (T)cs->beta, a0, tile, blockIdx.x, gridDim.x, true);
  const double v[1] = {a0};
  write_partials<1, Tile<TY>::NT>(v, partials, sh, blockIdx.x, gridDim.x);
}

// FIRST: iteration 0, where p and r are the same array: r at the node is the staged operand's centre, not loaded again.
template <typename T, bool NTP = false, bool FIRST = false>
struct PolB {
  static constexpr bool kRhs = false;
  const T *p;
  T *u;
  const T *rin;
  T *rout;
  T alpha;
  T pr[kMaxDepth], pu[kMaxDepth];
  using Raw = T;
  __device__ __forceinline__ T operand(long long idx) const { return p[idx]; }
  __device__ __forceinline__ T value(T v) const { return v; }
  __device__ __forceinline__ long long fcol(int, int) const { return -1; }
  __device__ __forceinline__ long long fplane() const { return 0; }
  __device__ __forceinline__ double fval(long long) const { return 0.0; }
  template <int S>
  __device__ __forceinline__ void center(int, int, int, long long idx) {
    static_assert(S < kMaxDepth, "centre slot");
    if constexpr (!FIRST) pr[S] = ld1<NTP>(&rin[idx]);
    pu[S] = ld1<NTP>(&u[idx]);
  }
  template <int S>
  __device__ __forceinline__ void consume(int, int, int, long long idx, T c, T out, double, double, double &acc0,
                                          double &) {
    const T rn = (FIRST ? c : pr[S]) - alpha * out;
    st1<NTP>(rn, &rout[idx]);
    st1<NTP>(pu[S] + alpha * c, &u[idx]);
    acc0 += (double)rn * (double)rn;
  }
};

// pass B's z-march of iteration it (u: the solution, or the correction of an inner FP32 solve)
template <typename T, int D, bool NTP, int TY = kTy>
__device__ __forceinline__ void pass_b_march(const Sweep &sw, int it, const CgBufs<T> &bf, T *u, T alpha, double &a0,
                                             T (*tile)[Tile<TY>::Rows][TX + 2], int bid, int nb, bool remap) {
  double a1 = 0.0;
  auto go = [&](auto first) {
    PolB<T, NTP, decltype(first)::value> pol;
    pol.p = bf.p;
    pol.u = u;
    pol.rin = bf.r_in;
    pol.rout = bf.r_out;
    pol.alpha = alpha;
    for (int q = 0; q < kMaxDepth; ++q) pol.pr[q] = pol.pu[q] = 0;
    zmarch<T, D, TY>(sw, pol, a0, a1, tile, nullptr, bid, nb, remap);
  };
  if (it == 0) go(std::true_type{});
  else go(std::false_type{});
}

template <typename T, int D, bool NTP, int TY>
__global__ __launch_bounds__(Tile<TY>::NT) void cg_pass_b_kernel(Sweep sw, T *u, T *r, T *p0, T *p1,
                                                                 const CgState *cs, double *partials) {
  __shared__ T tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[Tile<TY>::NT / 64];
  if (cs->done) return;
  const int it = cs->iter;
  const CgBufs<T> bf = cg_bufs(it, r, p0, p1);
  double a0 = 0.0;
  pass_b_march<T, D, NTP, TY>(sw, it, bf, u, (T)cs->alpha, a0, tile, blockIdx.x, gridDim.x, true);
  const double v[1] = {a0};
  write_partials<1, Tile<TY>::NT>(v, partials, sh, blockIdx.x, gridDim.x);
}

// The right-hand side inside the residual sweeps: f (or the adjoint's G) staged by the z-march (R f from LDS and
// registers), plus A's couplings to the Dirichlet values for nodes next to the boundary, which a small kernel over
// the six boundary-adjacent layers (boundary_terms_kernel) has written into r beforehand.
struct RhsPart {
  RhsSrc rs;
  int nx, ny, nz;
  const double *bterm;  // the boundary terms (in r's layout, read before r is overwritten at the same node)
  double bt[3];         // boundary terms of the planes in flight
  __device__ __forceinline__ long long fcol(int gi, int gj) const { return rs.gf.at(gi * rs.s, gj * rs.s, 0); }
  __device__ __forceinline__ long long fplane() const { return (long long)rs.s * rs.gf.sz; }
  __device__ __forceinline__ double fval(long long idx) const { return rs.f[idx]; }
  template <int S>
  __device__ __forceinline__ void boundary(int i, int j, int k, long long idx) {
    static_assert(S < 3, "residual sweeps prefetch at most 3 planes");
    const bool near = (i == 1 || j == 1 || k == 1 || i == nx - 1 || j == ny - 1 || k == nz - 1);
    bt[S] = (rs.mode == 0 && near) ? bterm[idx] : 0.0;
  }
  template <int S>
  __device__ __forceinline__ double b(double cf, double rf) const {
    return rs.mode == 1 ? cf : -rf + bt[S];
  }
};

// ------------------------------------------------------------------------------ self-finalizing CG iterations
//
// For grids whose sweeps have few workgroups, every workgroup of a pass sums the previous pass's partial sums itself
// (in the same fixed order, so all agree bit for bit) instead of waiting for a separate finalize launch: an
// iteration is two launches.  Workgroup 0 records the scalars in the CG state for the host and for the next pass.

constexpr int kSelfRedMaxBlocks = 2048;

// fixed-order sum by a whole workgroup of NTB threads of the threads' strided parts v (strided_sum<NTB>); valid in
// every thread
template <int NTB>
__device__ double block_fixed_finish(double v, double *sh) {
  const double t = block_sum<NTB>(v, sh);
  if (threadIdx.x == 0) sh[NTB / 64] = t;
  __syncthreads();
  const double s = sh[NTB / 64];
  __syncthreads();
  return s;
}

// Makes v be computed here, before what follows (an empty statement that takes it as an input), so that loads
// feeding it are not moved past a branch that does not use it.
__device__ __forceinline__ void keep(double v) { __asm__ volatile("" ::"v"(v)); }

// Pass A of iteration k = iterA: the stopping test on rho_k (Algorithm 1, the while condition), then
// p = r + beta p with beta = rho_k / rho_{k-1}, partial sums of p.Mp into partsA.
template <typename T, int D, bool NTP, int TY>
__global__ __launch_bounds__(Tile<TY>::NT) void cg_selfred_a_kernel(Sweep sw, T *r, T *p0, T *p1,
                                                                    CgState *cs, const double *partsB, int nbB,
                                                                    double tol, double *partsA) {
  constexpr int NTB = Tile<TY>::NT;
  __shared__ T tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[NTB / 64];
  __shared__ double shf[NTB];
  // The state and the partial sums are loaded together, so that they cost one memory latency: the second half of
  // the partials (the residual sweep's b.b) is used at k = 0 only and read at every k (it lies inside the buffer).
  const int done = cs->done;
  const int k = cs->iterA;
  const double s1 = strided_sum<NTB>(partsB, nbB), s2 = strided_sum<NTB>(partsB + nbB, nbB);
  keep(s1);
  keep(s2);
  if (done) return;
  double rho, bb, stop2;
  if (k == 0 && cs->preset) {
    rho = cs->rho;
    bb = cs->bnorm2;
    stop2 = cs->stop2;
  } else if (k == 0) {
    rho = block_fixed_finish<NTB>(s1, shf);
    bb = block_fixed_finish<NTB>(s2, shf) + cs->gbnd2;
    stop2 = tol * tol * bb;
  } else {
    rho = block_fixed_finish<NTB>(s1, shf);
    bb = cs->bnorm2;
    stop2 = cs->stop2;
  }
  const bool finite = isfinite(rho) && isfinite(bb);
  const bool conv = finite && rho <= stop2;
  const bool cap = finite && !conv && k >= cs->max_iters;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) {
      cs->bnorm2 = bb;
      cs->stop2 = stop2;
      cs->rho0 = rho;
    }
    if (cs->hist_on && k < EXCMG_MAX_HISTORY) cs->hist[k] = bb > 0.0 ? sqrt(rho / bb) : 0.0;
    cs->rhoA[k & 1] = rho;
    cs->rho = rho;
    cs->iter = k;
    cs->iterB = k;
    if (!finite) cs->status = EXCMG_ERR_BREAKDOWN;
    if (cap) cs->status = EXCMG_ERR_NOCONV;
    if (!finite || conv || cap) cs->done = 1;
  }
  if (!finite || conv || cap) return;
  const CgBufs<T> bf = cg_bufs(k, r, p0, p1);
  double a0 = 0.0;
  pass_a_march<T, D, NTP, TY>(sw, k, bf, (k == 0) ? T(0) : (T)(rho / cs->rhoA[(k - 1) & 1]), a0, tile, blockIdx.x,
                              gridDim.x, true);
  const double v[1] = {a0};
  write_partials<1, NTB>(v, partsA, sh, blockIdx.x, gridDim.x);
}

// Pass B of iteration k = iterB: alpha = rho_k / p.Mp (from partsA), u += alpha p, r -= alpha Mp, partial sums of
// r.r into partsB.
template <typename T, int D, bool NTP, int TY>
__global__ __launch_bounds__(Tile<TY>::NT) void cg_selfred_b_kernel(Sweep sw, T *u, T *r, T *p0, T *p1,
                                                                    CgState *cs, const double *partsA, int nbA,
                                                                    double *partsB) {
  constexpr int NTB = Tile<TY>::NT;
  __shared__ T tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[NTB / 64];
  __shared__ double shf[NTB];
  const int done = cs->done;  // loaded together with the partials, as in pass A
  const int k = cs->iterB;
  const double s1 = strided_sum<NTB>(partsA, nbA);
  keep(s1);
  if (done) return;
  const double pq = block_fixed_finish<NTB>(s1, shf);
  const bool bad = !(pq > 0.0) || !isfinite(pq);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cs->pq = pq;
    if (bad) {
      cs->status = EXCMG_ERR_BREAKDOWN;
      cs->done = 1;
    }
    cs->iterA = k + 1;
  }
  if (bad) return;
  const CgBufs<T> bf = cg_bufs(k, r, p0, p1);
  double a0 = 0.0;
  pass_b_march<T, D, NTP, TY>(sw, k, bf, u, (T)(cs->rhoA[k & 1] / pq), a0, tile, blockIdx.x, gridDim.x, true);
  const double v[1] = {a0};
  write_partials<1, NTB>(v, partsB, sh, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------- single-reduction CG on self-finalizing grids
//
// The Krylov iterates of Algorithm 1's CG (equal in exact arithmetic; the rounding differs), with both inner products
// of an iteration taken in one reduction (Chronopoulos and Gear's form): with s = M p and w = M r kept as vectors,
//   p = r + beta p,  s = w + beta s,  u += alpha p,  r -= alpha s,  w = M r,  gamma = r.r,  delta = w.r,
//   beta = gamma / gamma_old,  alpha = gamma / (delta - beta gamma / alpha_old)   (p = r, s = w, alpha = gamma / delta
// at k = 0).  An iteration is one launch: the new r is formed at staging on the tile and its halo (r - alpha (w +
// beta s) from the three old vectors, the same bits in every workgroup that stages a node), so w = M r needs no
// other pass, and each launch sums the previous launch's partials itself.

// w = M r and the partial sums of r.r and w.r: the start of the single-reduction CG
struct PolCg1Init {
  static constexpr bool kRhs = false;
  const double *r;
  double *w;
  using Raw = double;
  __device__ __forceinline__ double operand(long long idx) const { return r[idx]; }
  __device__ __forceinline__ double value(double v) const { return v; }
  __device__ __forceinline__ long long fcol(int, int) const { return -1; }
  __device__ __forceinline__ long long fplane() const { return 0; }
  __device__ __forceinline__ double fval(long long) const { return 0.0; }
  template <int S>
  __device__ __forceinline__ void center(int, int, int, long long) {}
  template <int S>
  __device__ __forceinline__ void consume(int, int, int, long long idx, double rc, double out, double, double,
                                          double &acc0, double &acc1) {
    w[idx] = out;
    acc0 += rc * rc;
    acc1 += out * rc;
  }
};

struct Cg1Raw {
  double r, w, s;
};

// one iteration of the single-reduction CG (first: k = 0, where p and s start as r and w).  r, w and s are read
// with halos, so the new ones go to another set of arrays (ro, wo, so); u and p are read and written at the node only.
template <int D>
struct PolCg1 {
  static constexpr bool kRhs = false;
  double *u, *p;
  const double *r, *w, *s;
  double *ro, *wo, *so;
  double alpha, beta;
  bool first;
  double cu[D], cp[D], cr[D], cw[D], cs[D];  // centre data of the output planes in flight
  using Raw = Cg1Raw;
  __device__ __forceinline__ Cg1Raw operand(long long idx) const { return Cg1Raw{r[idx], w[idx], s[idx]}; }
  __device__ __forceinline__ double dir(double a, double b) const { return first ? a : a + beta * b; }
  // the new r at a staged node: r - alpha (w + beta s)
  __device__ __forceinline__ double value(const Cg1Raw &v) const { return v.r - alpha * dir(v.w, v.s); }
  __device__ __forceinline__ long long fcol(int, int) const { return -1; }
  __device__ __forceinline__ long long fplane() const { return 0; }
  __device__ __forceinline__ double fval(long long) const { return 0.0; }
  template <int S>
  __device__ __forceinline__ void center(int, int, int, long long idx) {
    cu[S] = u[idx];
    cp[S] = p[idx];
    cr[S] = r[idx];
    cw[S] = w[idx];
    cs[S] = s[idx];
  }
  template <int S>
  __device__ __forceinline__ void consume(int, int, int, long long idx, double rn, double out, double, double,
                                          double &acc0, double &acc1) {
    const double pn = dir(cr[S], cp[S]);
    u[idx] = cu[S] + alpha * pn;
    p[idx] = pn;
    so[idx] = dir(cw[S], cs[S]);
    ro[idx] = rn;
    wo[idx] = out;
    acc0 += rn * rn;
    acc1 += out * rn;
  }
};

template <int D, int TY>
__global__ __launch_bounds__(Tile<TY>::NT) void cg1_init_kernel(Sweep sw, const double *r, double *w, double *parts) {
  __shared__ double tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[Tile<TY>::NT / 64];
  PolCg1Init pol{r, w};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double, D, TY>(sw, pol, a0, a1, tile, nullptr, blockIdx.x, gridDim.x, true);
  const double v[2] = {a0, a1};
  write_partials<2, Tile<TY>::NT>(v, parts, sh, blockIdx.x, gridDim.x);
}

// Iteration k of the single-reduction CG: from r, w, s (read with halos) into ro, wo, so; u and p in place.  par (the
// launch's parity, 0 for k = 0) picks the state's iteration counter to read (iterA, or iterB) and the one to write,
// so that no launch writes what its own workgroups read (the host alternates the vector sets the same way); partsIn: the
// previous launch's partial sums of gamma and delta (the init sweep's at k = 0), gridDim.x each; partsR: the residual
// sweep's (r.r, b.b), nbR each, whose b.b is used at k = 0.  The stopping test on gamma = r_k.r_k comes first
// (Algorithm 1), as in the two-pass CG.
template <int D, int TY>
__global__ __launch_bounds__(Tile<TY>::NT) void cg1_iter_kernel(Sweep sw, double *u, double *p, const double *r,
                                                                const double *w, const double *s, double *ro,
                                                                double *wo, double *so, CgState *cs, int par,
                                                                const double *partsIn, const double *partsR, int nbR,
                                                                double tol, double *partsOut) {
  constexpr int NTB = Tile<TY>::NT;
  __shared__ double tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[NTB / 64];
  __shared__ double shf[NTB];
  const int nb = gridDim.x;
  const int done = cs->done;
  const int k = par ? cs->iterB : cs->iterA;
  const double g1 = strided_sum<NTB>(partsIn, nb), d1 = strided_sum<NTB>(partsIn + nb, nb);
  const double b1 = strided_sum<NTB>(partsR + nbR, nbR);
  keep(g1);
  keep(d1);
  keep(b1);
  if (done) return;
  const double gamma = block_fixed_finish<NTB>(g1, shf);
  const double delta = block_fixed_finish<NTB>(d1, shf);
  double bb, stop2, alpha, beta;
  if (k == 0) {
    bb = block_fixed_finish<NTB>(b1, shf) + cs->gbnd2;
    stop2 = tol * tol * bb;
    beta = 0.0;
    alpha = gamma / delta;
  } else {
    bb = cs->bnorm2;
    stop2 = cs->stop2;
    beta = gamma / cs->rhoA[(k - 1) & 1];
    alpha = gamma / (delta - beta * gamma / cs->alphaA[(k - 1) & 1]);
  }
  const bool finite = isfinite(gamma) && isfinite(bb);
  const bool conv = finite && gamma <= stop2;
  const bool cap = finite && !conv && k >= cs->max_iters;
  const bool bad = finite && !conv && !cap && !(alpha > 0.0 && isfinite(alpha));
  const bool stop = !finite || conv || cap || bad;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (k == 0) {
      cs->bnorm2 = bb;
      cs->stop2 = stop2;
      cs->rho0 = gamma;
    }
    if (cs->hist_on && k < EXCMG_MAX_HISTORY) cs->hist[k] = bb > 0.0 ? sqrt(gamma / bb) : 0.0;
    cs->rhoA[k & 1] = gamma;
    cs->alphaA[k & 1] = alpha;
    cs->rho = gamma;
    cs->iter = k;
    if (par) cs->iterA = k + 1;
    else cs->iterB = k + 1;
    if (!finite || bad) cs->status = EXCMG_ERR_BREAKDOWN;
    if (cap) cs->status = EXCMG_ERR_NOCONV;
    if (stop) cs->done = 1;
  }
  if (stop) return;
  PolCg1<D> pol{u, p, r, w, s, ro, wo, so, alpha, beta, k == 0, {}, {}, {}, {}, {}};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double, D, TY>(sw, pol, a0, a1, tile, nullptr, blockIdx.x, gridDim.x, true);
  const double v[2] = {a0, a1};
  write_partials<2, NTB>(v, partsOut, sh, blockIdx.x, gridDim.x);
}

__global__ void selfred_init_kernel(CgState *cs, int max_iters, int hist_on, int preset) {
  cs->iterA = 0;
  cs->iterB = 0;
  cs->iter = 0;
  cs->done = 0;
  cs->status = 0;
  cs->max_iters = max_iters;
  cs->hist_on = hist_on;
  cs->preset = preset;
}

// r = b - M u; u and r share the level layout.
template <bool NTP = false>
struct PolResid {
  static constexpr bool kRhs = true;
  const double *u;
  double *r;
  RhsPart rp;
  using Raw = double;
  __device__ __forceinline__ double operand(long long idx) const { return u[idx]; }
  __device__ __forceinline__ double value(double v) const { return v; }
  __device__ __forceinline__ long long fcol(int gi, int gj) const { return rp.fcol(gi, gj); }
  __device__ __forceinline__ long long fplane() const { return rp.fplane(); }
  __device__ __forceinline__ double fval(long long idx) const { return rp.fval(idx); }
  template <int S>
  __device__ __forceinline__ void center(int i, int j, int k, long long idx) { rp.template boundary<S>(i, j, k, idx); }
  template <int S>
  __device__ __forceinline__ void consume(int, int, int, long long idx, double, double out, double cf, double rf,
                                          double &acc0, double &acc1) {
    const double bv = rp.template b<S>(cf, rf);
    const double rn = bv - out;
    st1<NTP>(rn, &r[idx]);
    acc0 += rn * rn;
    acc1 += stop_norm_term(rp.rs, bv, rf);
  }
};

template <int D, bool NTP>
__global__ __launch_bounds__(NT) void residual_kernel(Sweep sw, const double *u, RhsSrc rs, double *r,
                                                      double *partials) {
  __shared__ double tile[2][kTileRows][TX + 2];
  __shared__ double sh[NT / 64];
  __shared__ double tileF[2][kTileRows][TX + 2];
  PolResid<NTP> pol{u, r, RhsPart{rs, sw.g.nx, sw.g.ny, sw.g.nz, r, {0.0, 0.0, 0.0}}};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double, D>(sw, pol, a0, a1, tile, tileF, blockIdx.x, gridDim.x, true);
  const double v[2] = {a0, a1};
  write_partials<2>(v, partials, sh, blockIdx.x, gridDim.x);
}

// r32 = (float)(b - M u), d32 = 0; the FP32 arrays use their own layout g32.
template <bool NTP = false>
struct PolResidCast {
  static constexpr bool kRhs = true;
  const double *u;
  Grid g32;
  float *r32;
  float *d32;
  RhsPart rp;
  double acc2;  // sum of the squared FP32-rounded residual
  using Raw = double;
  __device__ __forceinline__ double operand(long long idx) const { return u[idx]; }
  __device__ __forceinline__ double value(double v) const { return v; }
  __device__ __forceinline__ long long fcol(int gi, int gj) const { return rp.fcol(gi, gj); }
  __device__ __forceinline__ long long fplane() const { return rp.fplane(); }
  __device__ __forceinline__ double fval(long long idx) const { return rp.fval(idx); }
  template <int S>
  __device__ __forceinline__ void center(int i, int j, int k, long long idx) { rp.template boundary<S>(i, j, k, idx); }
  template <int S>
  __device__ __forceinline__ void consume(int i, int j, int k, long long, double, double out, double cf, double rf,
                                          double &acc0, double &acc1) {
    const double bv = rp.template b<S>(cf, rf);
    const double rn = bv - out;
    const float rf32 = (float)rn;
    const long long q = g32.at(i, j, k);
    st1<NTP>(rf32, &r32[q]);
    st1<NTP>(0.0f, &d32[q]);
    acc0 += rn * rn;
    acc1 += stop_norm_term(rp.rs, bv, rf);
    acc2 += (double)rf32 * (double)rf32;
  }
};

template <int D, bool NTP>
__global__ __launch_bounds__(NT) void residual_cast_kernel(Sweep sw, const double *u, RhsSrc rs,
                                                           const double *bterm, Grid g32, float *r32, float *d32,
                                                           double *partials) {
  __shared__ double tile[2][kTileRows][TX + 2];
  __shared__ double sh[NT / 64];
  __shared__ double tileF[2][kTileRows][TX + 2];
  PolResidCast<NTP> pol{u, g32, r32, d32, RhsPart{rs, sw.g.nx, sw.g.ny, sw.g.nz, bterm, {0.0, 0.0, 0.0}}, 0.0};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double, D>(sw, pol, a0, a1, tile, tileF, blockIdx.x, gridDim.x, true);
  const double v[3] = {a0, a1, pol.acc2};
  write_partials<3>(v, partials, sh, blockIdx.x, gridDim.x);
}

// y = M x with x and y in possibly different layouts.
struct PolApply {
  static constexpr bool kRhs = false;
  const double *x;
  Grid gy;
  double *y;
  using Raw = double;
  __device__ __forceinline__ double operand(long long idx) const { return x[idx]; }
  __device__ __forceinline__ double value(double v) const { return v; }
  __device__ __forceinline__ long long fcol(int, int) const { return -1; }
  __device__ __forceinline__ long long fplane() const { return 0; }
  __device__ __forceinline__ double fval(long long) const { return 0.0; }
  template <int S>
  __device__ __forceinline__ void center(int, int, int, long long) {}
  template <int S>
  __device__ __forceinline__ void consume(int i, int j, int k, long long, double, double out, double, double,
                                          double &, double &) {
    y[gy.at(i, j, k)] = out;
  }
};

__global__ __launch_bounds__(NT) void apply_kernel(Sweep sw, const double *x, Grid gy, double *y) {
  __shared__ double tile[2][kTileRows][TX + 2];
  PolApply pol{x, gy, y};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double>(sw, pol, a0, a1, tile, nullptr, blockIdx.x, gridDim.x, true);
}

// A's couplings to the Dirichlet values, written at every interior node next to the boundary (the six layers
// i = 1, i = nx-1, j = 1, ...; nodes on two layers are written twice with the same value).  blockIdx.z = layer.
__device__ __forceinline__ void boundary_terms_block(const RhsSrc &rs, const Grid &g, double *out, int bx, int by,
                                                     int layer) {
  // layer 0,1: x layers; 2,3: y layers; 4,5: z layers
  const int a = 1 + bx * 256 + threadIdx.x;
  const int b = 1 + by;
  int i, j, k;
  if (layer < 2) {
    if (a >= g.ny || b >= g.nz) return;
    i = layer == 0 ? 1 : g.nx - 1; j = a; k = b;
  } else if (layer < 4) {
    if (a >= g.nx || b >= g.nz) return;
    i = a; j = layer == 2 ? 1 : g.ny - 1; k = b;
  } else {
    if (a >= g.nx || b >= g.ny) return;
    i = a; j = b; k = layer == 4 ? 1 : g.nz - 1;
  }
  out[g.at(i, j, k)] = rhs_boundary_terms_inl(rs, g.nx, g.ny, g.nz, i, j, k);
}

__global__ __launch_bounds__(256) void boundary_terms_kernel(RhsSrc rs, Grid g, double *out) {
  boundary_terms_block(rs, g, out, blockIdx.x, blockIdx.y, blockIdx.z);
}

// cs->gbnd2 = the sum of g^2 over the boundary nodes of grid g, the boundary half of the squared norm of the stopping
// test under EXCMG_STOP_F_G (0 otherwise).  Node m of the enumeration: the planes k = 0 and k = nz whole, then per
// inner plane the rows j = 0 and j = ny whole and the two end nodes i = 0, nx of every inner row.  One workgroup,
// fixed order.
__global__ __launch_bounds__(FT) void boundary_g2_kernel(RhsSrc rs, Grid g, CgState *cs) {
  __shared__ double sh[FT / 64 + 1];
  const long long px = g.nx + 1, py = g.ny + 1;
  const long long full = 2 * px * py;               // the two end planes
  const long long per = 2 * px + 2 * (g.ny - 1);     // boundary nodes of one inner plane
  const long long total = rs.fg ? full + (long long)(g.nz - 1) * per : 0;
  const int s = rs.s;
  double acc = 0.0;
  for (long long m = threadIdx.x; m < total; m += FT) {
    int i, j, k;
    if (m < full) {
      const long long t = m % (px * py);
      k = m < px * py ? 0 : g.nz;
      i = (int)(t % px);
      j = (int)(t / px);
    } else {
      const long long q = m - full;
      k = 1 + (int)(q / per);
      const long long t = q % per;
      if (t < 2 * px) {
        i = (int)(t % px);
        j = t < px ? 0 : g.ny;
      } else {
        const long long e = t - 2 * px;
        i = (e & 1) ? g.nx : 0;
        j = 1 + (int)(e >> 1);
      }
    }
    const double v = rs.g[rs.gf.at(i * s, j * s, k * s)];
    acc += v * v;
  }
  const double t = block_sum<FT>(acc, sh);
  if (threadIdx.x == 0) cs->gbnd2 = t;
}

__global__ void clear_gbnd2_kernel(CgState *a, CgState *b) {
  a->gbnd2 = 0.0;
  b->gbnd2 = 0.0;
}

// --------------------------------------------------------------------------------------------------------- finalize

__global__ __launch_bounds__(FT) void finalize_init_kernel(CgState *cs, const double *partials, int nparts, double tol,
                                                           int max_iters, int hist_on) {
  __shared__ double sh[FT / 64 + 1];
  const double rho = fixed_sum(partials, nparts, sh);
  const double bb = fixed_sum(partials + nparts, nparts, sh) + cs->gbnd2;
  if (threadIdx.x == 0) state_init(cs, rho, bb, tol, max_iters, hist_on);
}

__global__ __launch_bounds__(FT) void finalize_ir_kernel(CgState *outer, CgState *inner, const double *partials,
                                                         int nparts, double tol, double eta, int outer_step,
                                                         int max_outer, int max_inner) {
  __shared__ double sh[FT / 64 + 1];
  const double r64 = fixed_sum(partials, nparts, sh);
  const double bb = fixed_sum(partials + nparts, nparts, sh) + outer->gbnd2;
  const double r32 = fixed_sum(partials + 2 * nparts, nparts, sh);
  if (threadIdx.x == 0) state_ir(outer, inner, r64, bb, r32, tol, eta, outer_step, max_outer, max_inner);
}

__global__ __launch_bounds__(FT) void finalize_a_kernel(CgState *cs, const double *partials, int nparts) {
  __shared__ double sh[FT / 64 + 1];
  if (cs->done) return;
  const double pq = fixed_sum(partials, nparts, sh);
  if (threadIdx.x == 0) state_after_a(cs, pq);
}

__global__ __launch_bounds__(FT) void finalize_b_kernel(CgState *cs, const double *partials, int nparts) {
  __shared__ double sh[FT / 64 + 1];
  if (cs->done) return;
  const double rho = fixed_sum(partials, nparts, sh);
  if (threadIdx.x == 0) state_after_b(cs, rho);
}

// ------------------------------------------------------------------------------------------------------ small kernels

// CG state for the autotuner's trial launches: a later iteration (pass A then reads r and p_old, as it does in
// every iteration but the first), never converged, alpha = beta = 0.  The trials' results are discarded: a solve
// writes these work buffers before it reads them.
__device__ void tune_state(CgState *cs) {
  cs->rho = 1.0;
  cs->rho_old = 1.0;
  cs->pq = 1.0;
  cs->alpha = 0.0;
  cs->beta = 0.0;
  cs->bnorm2 = 1.0;
  cs->stop2 = -1.0;
  cs->iter = 1;
  cs->done = 0;
  cs->status = 0;
  cs->max_iters = 1 << 30;
  cs->hist_on = 0;
}

// the same at iteration iter: 0 for the trials of a first iteration's passes (p = r)
__global__ void tune_state_kernel(CgState *cs, int iter) {
  tune_state(cs);
  cs->iter = iter;
}

// the trial state of a self-finalizing pass (iteration 1 of both passes, never converged) and n partial sums of 1 for
// it to read, so that neither pass stops at its reduction
// (also the trial state of the single-reduction CG, whose launches of parity 1 then all run iteration 1 with
// beta ~ 1e-200 n and alpha = 1; the two-pass passes take beta from rhoA[0] and alpha from rhoA[1])
__global__ void tune_selfred_kernel(CgState *cs, double *parts, int n) {
  if (threadIdx.x == 0) {
    tune_state(cs);
    cs->iterA = 1;
    cs->iterB = 1;
    cs->preset = 0;
    cs->rhoA[0] = 1e200;
    cs->rhoA[1] = 1.0;
    cs->alphaA[0] = 1.0;
    cs->alphaA[1] = 1.0;
  }
  for (int q = threadIdx.x; q < n; q += blockDim.x) parts[q] = 1.0;
}

// Holds the stream for about `ticks` of the constant 100 MHz wall clock (at most 2^20 sleeps of ~0.3 us), so that
// the launches queued behind it run back to back when it ends.
__global__ void delay_kernel(long long ticks) {
  const long long t0 = wall_clock64();
  for (int q = 0; q < (1 << 20) && wall_clock64() - t0 < ticks; ++q) __builtin_amdgcn_s_sleep(10);
}

// copy of a small device record (n 8-byte words) into host memory the device can write (the host reads it after a
// stream synchronisation; no staged copy)
__global__ void publish_kernel(const unsigned long long *src, unsigned long long *dst, int n) {
  for (int q = threadIdx.x; q < n; q += blockDim.x) dst[q] = src[q];
}

__device__ __forceinline__ void add_correction_block(const Grid &gu, double *u, const Grid &g32, const float *d,
                                                     int bx, int by, int bz) {
  const int i = 1 + bx * 256 + threadIdx.x;
  const int j = 1 + by;
  const int k = 1 + bz;
  if (i >= gu.nx) return;
  u[gu.at(i, j, k)] += (double)d[g32.at(i, j, k)];
}

__global__ __launch_bounds__(256) void add_correction_kernel(Grid gu, double *u, Grid g32, const float *d) {
  add_correction_block(gu, u, g32, d, blockIdx.x, blockIdx.y, blockIdx.z);
}

// ----------------------------------------------------------------------------------------------------------- DSOLVE

constexpr int DT = 1024;

__device__ __forceinline__ double stencil_direct(const Grid &g, const double *x, int i, int j, int k,
                                                 const Stencil &s) {
  auto X = [&](int a, int b, int c) -> double {
    const int ii = i + a, jj = j + b, kk = k + c;
    if (ii <= 0 || jj <= 0 || kk <= 0 || ii >= g.nx || jj >= g.ny || kk >= g.nz) return 0.0;
    return x[g.at(ii, jj, kk)];
  };
  double v = s.c0 * X(0, 0, 0);
  v += s.cx * (X(1, 0, 0) + X(-1, 0, 0));
  v += s.cy * (X(0, 1, 0) + X(0, -1, 0));
  v += s.cz * (X(0, 0, 1) + X(0, 0, -1));
  v += s.cxy * ((X(1, 1, 0) + X(-1, 1, 0)) + (X(1, -1, 0) + X(-1, -1, 0)));
  v += s.cxz * ((X(1, 0, 1) + X(-1, 0, 1)) + (X(1, 0, -1) + X(-1, 0, -1)));
  v += s.cyz * ((X(0, 1, 1) + X(0, -1, 1)) + (X(0, 1, -1) + X(0, -1, -1)));
  return v;
}

__device__ double dsum(double v, double *sh) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int q = 0; q < DT / 64; ++q) t += sh[q];
  return t;  // every thread holds the same value
}

// Conjugate gradients on M u = b for a small grid, in one workgroup of 1024 threads, all iterations in one launch
// (b formed on the fly by rhs_at).  Two uses:
//   exact = 1: the direct solve of the two coarsest grids (Algorithm 1, first two lines): iterate until the recursive
//              relative residual is 1e-15 (rounding level) or the iteration cap;
//   exact = 0: the relaxation of a small grid (Algorithm 1, the while loop): the same Hestenes-Stiefel iteration and
//              stopping test as the multi-workgroup sweeps, ||r|| <= tol ||b|| checked before every iteration.
// Small grids are latency-bound: one workgroup with every iteration in registers and L2 beats two sweep launches
// plus two reductions per iteration.
__device__ void small_cg_body(const Grid &gu, double *u, const RhsSrc &rs, const Grid &gw, double *r, double *p,
                              double *q, const Stencil &st, CgState *cs, double tol, int cap, int exact, int hist_on) {
  __shared__ double sh[DT / 64];
  const long long nx1 = gu.nx - 1, ny1 = gu.ny - 1, nz1 = gu.nz - 1;
  const long long n = nx1 * ny1 * nz1;
  auto coords = [&](long long m, int &i, int &j, int &k) {
    i = (int)(1 + m % nx1);
    const long long t = m / nx1;
    j = (int)(1 + t % ny1);
    k = (int)(1 + t / ny1);
  };
  // r = b - M u (u's interior), p = r
  double rr = 0.0, bb = 0.0;
  for (long long m = threadIdx.x; m < n; m += DT) {
    int i, j, k;
    coords(m, i, j, k);
    double rf;
    const double bv = rhs_at<true>(rs, gu.nx, gu.ny, gu.nz, i, j, k, rf);
    const double rv = bv - stencil_direct(gu, u, i, j, k, st);
    r[gw.at(i, j, k)] = rv;
    p[gw.at(i, j, k)] = rv;
    rr += rv * rv;
    bb += stop_norm_term(rs, bv, rf);
  }
  double rho = dsum(rr, sh);
  const double bnorm2 = dsum(bb, sh) + cs->gbnd2;
  const double stop2 = (exact ? 1e-30 : tol * tol) * bnorm2;
  if (hist_on && threadIdx.x == 0) cs->hist[0] = bnorm2 > 0.0 ? sqrt(rho / bnorm2) : 0.0;
  int it = 0;
  int status = 0;
  if (!isfinite(rho) || !isfinite(bnorm2)) status = EXCMG_ERR_BREAKDOWN;
  while (status == 0 && rho > stop2) {
    if (it >= cap) {  // also a direct solve that has not reached rounding level: reported, never silent
      status = EXCMG_ERR_NOCONV;
      break;
    }
    __syncthreads();  // p complete
    double pq = 0.0;
    for (long long m = threadIdx.x; m < n; m += DT) {
      int i, j, k;
      coords(m, i, j, k);
      const double qv = stencil_direct(gw, p, i, j, k, st);
      q[gw.at(i, j, k)] = qv;
      pq += p[gw.at(i, j, k)] * qv;
    }
    pq = dsum(pq, sh);
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = EXCMG_ERR_BREAKDOWN;
      break;
    }
    const double alpha = rho / pq;
    double rn = 0.0;
    for (long long m = threadIdx.x; m < n; m += DT) {
      int i, j, k;
      coords(m, i, j, k);
      const long long w = gw.at(i, j, k);
      u[gu.at(i, j, k)] += alpha * p[w];
      const double rv = r[w] - alpha * q[w];
      r[w] = rv;
      rn += rv * rv;
    }
    const double rho_new = dsum(rn, sh);
    const double beta = rho_new / rho;
    rho = rho_new;
    ++it;
    if (hist_on && threadIdx.x == 0 && it < EXCMG_MAX_HISTORY) cs->hist[it] = sqrt(rho / bnorm2);
    if (!isfinite(rho)) {
      status = EXCMG_ERR_BREAKDOWN;
      break;
    }
    __syncthreads();  // all reads of p (in q) are done before p is overwritten
    for (long long m = threadIdx.x; m < n; m += DT) {
      int i, j, k;
      coords(m, i, j, k);
      const long long w = gw.at(i, j, k);
      p[w] = r[w] + beta * p[w];
    }
  }
  if (threadIdx.x == 0) {
    cs->iter = it;
    cs->rho = rho;
    cs->bnorm2 = bnorm2;
    cs->status = status;
    cs->done = 1;
  }
}

// The same CG with the search direction p in LDS: the grid's node array (boundary nodes held at 0, which is the halo
// of the stencil) and every thread's own unknowns (node m = threadIdx.x + q*DT, q < SK) with their u, r, p and M p in
// registers.  An iteration is then one stencil evaluation from LDS and two workgroup reductions.
constexpr int SK = 4;  // unknowns per thread: up to SK * DT = 4096 unknowns

__host__ __device__ inline long long small_lds_nodes(const Grid &g) {
  return (long long)(g.nx + 1) * (g.ny + 1) * (g.nz + 1);
}
constexpr long long kSmallLdsMax = 8192;  // nodes that fit the LDS path (64 KB)

__device__ void small_cg_lds_body(const Grid &gu, double *u, const RhsSrc &rs, const Grid &gw, double *r,
                                  const Stencil &st, CgState *cs, double tol, int cap, int exact, int hist_on,
                                  double *P) {
  __shared__ double sh[DT / 64];
  const int nx1 = gu.nx - 1, ny1 = gu.ny - 1, nz1 = gu.nz - 1;
  const int n = nx1 * ny1 * nz1;
  const int sy = gu.nx + 1, sz = (gu.nx + 1) * (gu.ny + 1);
  const int nodes = sz * (gu.nz + 1);
  const double c0 = st.c0, cx = st.cx, cy = st.cy, cz = st.cz, cxy = st.cxy, cxz = st.cxz, cyz = st.cyz;
  auto apply = [&](int c) {  // (M x)(node c) from LDS
    const double *x = P + c;
    double v = c0 * x[0];
    v += cx * (x[1] + x[-1]);
    v += cy * (x[sy] + x[-sy]);
    v += cz * (x[sz] + x[-sz]);
    v += cxy * ((x[1 + sy] + x[-1 + sy]) + (x[1 - sy] + x[-1 - sy]));
    v += cxz * ((x[1 + sz] + x[-1 + sz]) + (x[1 - sz] + x[-1 - sz]));
    v += cyz * ((x[sy + sz] + x[-sy + sz]) + (x[sy - sz] + x[-sy - sz]));
    return v;
  };
  auto coords = [&](int m, int &i, int &j, int &k) {
    i = 1 + m % nx1;
    const int t = m / nx1;
    j = 1 + t % ny1;
    k = 1 + t / ny1;
  };
  // 1. r = b - M u into the global work array (b formed on the fly; nothing else is live across its calls)
  double r2 = 0.0, b2 = 0.0;
  for (int m = threadIdx.x; m < n; m += DT) {
    int i, j, k;
    coords(m, i, j, k);
    double rf;
    const double bv = rhs_at<true>(rs, gu.nx, gu.ny, gu.nz, i, j, k, rf);
    const double rv = bv - stencil_direct(gu, u, i, j, k, st);
    r[gw.at(i, j, k)] = rv;
    r2 += rv * rv;
    b2 += stop_norm_term(rs, bv, rf);
  }
  double rho = dsum(r2, sh);  // its barriers also make r visible to the whole workgroup
  const double bnorm2 = dsum(b2, sh) + cs->gbnd2;
  const double rho_start = rho;
  // 2. own unknowns into registers, p = r into LDS (boundary nodes 0)
  for (int c = threadIdx.x; c < nodes; c += DT) P[c] = 0.0;
  __syncthreads();
  int li[SK];
  double uu[SK], rr[SK], pp[SK], qq[SK];
#pragma unroll
  for (int q = 0; q < SK; ++q) {
    const int m = threadIdx.x + q * DT;
    li[q] = -1;
    uu[q] = rr[q] = pp[q] = qq[q] = 0.0;
    if (m < n) {
      int i, j, k;
      coords(m, i, j, k);
      li[q] = i + j * sy + k * sz;
      uu[q] = u[gu.at(i, j, k)];
      rr[q] = r[gw.at(i, j, k)];
      pp[q] = rr[q];
      P[li[q]] = pp[q];
    }
  }
  const double stop2 = (exact ? 1e-30 : tol * tol) * bnorm2;
  if (hist_on && threadIdx.x == 0) cs->hist[0] = bnorm2 > 0.0 ? sqrt(rho / bnorm2) : 0.0;
  int it = 0, status = 0;
  if (!isfinite(rho) || !isfinite(bnorm2)) status = EXCMG_ERR_BREAKDOWN;
  while (status == 0 && rho > stop2) {
    if (it >= cap) {  // also a direct solve that has not reached rounding level: reported, never silent
      status = EXCMG_ERR_NOCONV;
      break;
    }
    __syncthreads();  // p complete in LDS
    double pq = 0.0;
#pragma unroll
    for (int q = 0; q < SK; ++q) {
      if (li[q] < 0) continue;
      qq[q] = apply(li[q]);
      pq += pp[q] * qq[q];
    }
    pq = dsum(pq, sh);  // its barriers order every read of p above before the writes of p below
    if (!(pq > 0.0) || !isfinite(pq)) {
      status = EXCMG_ERR_BREAKDOWN;
      break;
    }
    const double alpha = rho / pq;
    double rn = 0.0;
#pragma unroll
    for (int q = 0; q < SK; ++q) {
      if (li[q] < 0) continue;
      uu[q] += alpha * pp[q];
      rr[q] -= alpha * qq[q];
      rn += rr[q] * rr[q];
    }
    const double rho_new = dsum(rn, sh);
    const double beta = rho_new / rho;
    rho = rho_new;
    ++it;
    if (hist_on && threadIdx.x == 0 && it < EXCMG_MAX_HISTORY) cs->hist[it] = sqrt(rho / bnorm2);
    if (!isfinite(rho)) {
      status = EXCMG_ERR_BREAKDOWN;
      break;
    }
#pragma unroll
    for (int q = 0; q < SK; ++q) {
      if (li[q] < 0) continue;
      pp[q] = rr[q] + beta * pp[q];
      P[li[q]] = pp[q];
    }
  }
#pragma unroll
  for (int q = 0; q < SK; ++q) {
    if (li[q] < 0) continue;
    int i, j, k;
    coords(threadIdx.x + q * DT, i, j, k);
    u[gu.at(i, j, k)] = uu[q];
  }
  if (threadIdx.x == 0) {
    cs->iter = it;
    cs->rho = rho;
    cs->rho0 = rho_start;
    cs->bnorm2 = bnorm2;
    cs->status = status;
    cs->done = 1;
  }
}

// ----------------------------------------------------------------------------------------- direct solve by sines
//
// With zero Dirichlet data, M (the 19-point operator on the interior) is diagonalised by the products of DST-I
// vectors s_p(i) = sin(pi p i / N), p, i = 1..N-1 per axis: M S = S diag(lambda) with
//   lambda_pqr = c0 + 2 cx Cx + 2 cy Cy + 2 cz Cz + 4 cxy Cx Cy + 4 cxz Cx Cz + 4 cyz Cy Cz,  Cx = cos(pi p / Nx), ...
// (c* the stencil's coefficients), and S^2 = (Nx Ny Nz / 8) I.  So M^-1 b = (8 / (Nx Ny Nz)) S diag(1/lambda) S b: three
// one-dimensional sine transforms, a division, three more.  This is DSOLVE of Algorithm 1 as an exact direct solve
// (to rounding), in one workgroup, for grids of at most kDstMax cells per axis; the transforms are dense
// (N-1) x (N-1) products along each axis through the work arrays A and B (the grid's layout), with the sine table of
// the current axis in LDS.

__device__ void dst_solve_body(const Grid &gu, double *u, const RhsSrc &rs, const Stencil &st, CgState *cs,
                               double *A, double *B) {
  __shared__ double tab[(kDstMax - 1) * (kDstMax - 1)];
  __shared__ double cosv[3][kDstMax];
  __shared__ double sh[DT / 64];
  const int n1[3] = {gu.nx - 1, gu.ny - 1, gu.nz - 1};
  const int N[3] = {gu.nx, gu.ny, gu.nz};
  const int n = n1[0] * n1[1] * n1[2];
  auto coords = [&](int m, int &i, int &j, int &k) {
    i = 1 + m % n1[0];
    const int t = m / n1[0];
    j = 1 + t % n1[1];
    k = 1 + t / n1[1];
  };
  // A = b (formed from the level data), and the cosines of every axis
  double b2 = 0.0;
  for (int m = threadIdx.x; m < n; m += DT) {
    int i, j, k;
    coords(m, i, j, k);
    double rf;
    const double bv = rhs_at<true>(rs, gu.nx, gu.ny, gu.nz, i, j, k, rf);
    A[gu.at(i, j, k)] = bv;
    b2 += stop_norm_term(rs, bv, rf);
  }
  for (int e = threadIdx.x; e < 3 * kDstMax; e += DT) {
    const int d = e / kDstMax, p = e % kDstMax;
    cosv[d][p] = (p >= 1 && p < N[d]) ? cospi((double)p / N[d]) : 0.0;
  }
  // one transform along axis d: dst(.., i, ..) = sum_i' sin(pi i i' / N_d) src(.., i', ..)
  auto transform = [&](int d, const double *src, double *dst) {
    const int L = n1[d];
    __syncthreads();  // src complete; the previous table no longer read
    for (int e = threadIdx.x; e < L * L; e += DT) {
      const int p = e / L + 1, q = e % L + 1;
      tab[e] = sinpi((double)((p * q) % (2 * N[d])) / N[d]);
    }
    __syncthreads();
    const long long stride = d == 0 ? 1 : (d == 1 ? gu.sy : gu.sz);
    for (int m = threadIdx.x; m < n; m += DT) {
      int i, j, k;
      coords(m, i, j, k);
      const int t = d == 0 ? i : (d == 1 ? j : k);
      const long long base = gu.at(i, j, k) - (long long)t * stride;  // the line's node 0
      const double *row = tab + (t - 1) * L;
      double v = 0.0;
      for (int q = 1; q <= L; ++q) v += row[q - 1] * src[base + (long long)q * stride];
      dst[gu.at(i, j, k)] = v;
    }
  };
  transform(0, A, B);
  transform(1, B, A);
  transform(2, A, B);
  // divide by the eigenvalues (with the scale of the inverse transform)
  __syncthreads();
  const double scale = 8.0 / ((double)N[0] * N[1] * N[2]);
  for (int m = threadIdx.x; m < n; m += DT) {
    int i, j, k;
    coords(m, i, j, k);
    const double Cx = cosv[0][i], Cy = cosv[1][j], Cz = cosv[2][k];
    const double lam = st.c0 + 2.0 * (st.cx * Cx + st.cy * Cy + st.cz * Cz) +
                       4.0 * (st.cxy * Cx * Cy + st.cxz * Cx * Cz + st.cyz * Cy * Cz);
    B[gu.at(i, j, k)] *= scale / lam;
  }
  transform(0, B, A);
  transform(1, A, B);
  transform(2, B, A);
  __syncthreads();
  for (int m = threadIdx.x; m < n; m += DT) {
    int i, j, k;
    coords(m, i, j, k);
    u[gu.at(i, j, k)] = A[gu.at(i, j, k)];
  }
  __syncthreads();
  // residual of the solve, for the record
  double r2 = 0.0;
  for (int m = threadIdx.x; m < n; m += DT) {
    int i, j, k;
    coords(m, i, j, k);
    const double rv = rhs_at<true>(rs, gu.nx, gu.ny, gu.nz, i, j, k) - stencil_direct(gu, u, i, j, k, st);
    r2 += rv * rv;
  }
  const double rho = dsum(r2, sh);
  const double bnorm2 = dsum(b2, sh) + cs->gbnd2;
  if (threadIdx.x == 0) {
    cs->iter = 0;
    cs->rho = rho;
    cs->rho0 = rho;
    cs->bnorm2 = bnorm2;
    cs->status = (isfinite(rho) && isfinite(bnorm2)) ? 0 : EXCMG_ERR_BREAKDOWN;
    cs->done = 1;
  }
}

__host__ __device__ inline bool small_fits_lds(const Grid &g) {
  return small_lds_nodes(g) <= kSmallLdsMax && g.interior() <= (long long)SK * DT;
}

__global__ __launch_bounds__(DT) void small_cg_kernel(Grid gu, double *u, RhsSrc rs, Grid gw, double *r, double *p,
                                                      double *q, Stencil st, CgState *cs, double tol, int cap,
                                                      int exact, int hist_on) {
  extern __shared__ double lds_p[];
  if (exact && dst_fits(gu))
    dst_solve_body(gu, u, rs, st, cs, r, p);
  else if (small_fits_lds(gu))
    small_cg_lds_body(gu, u, rs, gw, r, st, cs, tol, cap, exact, hist_on, lds_p);
  else
    small_cg_body(gu, u, rs, gw, r, p, q, st, cs, tol, cap, exact, hist_on);
}

// ---------------------------------------------------------------------------------------------------- batched form
//
// The same sweeps, reductions and small-grid CG over a table of problems (one entry per problem; see BatchEntry).

// entry of flattened workgroup b: the largest e with pre[e] <= b (entries with no workgroups have pre[e] = pre[e+1])
__device__ __forceinline__ int find_entry(const int *pre, int n, int b) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (pre[mid] <= b) lo = mid;
    else hi = mid;
  }
  return lo;
}

// copy of a CG state's scalars for the host; the finest grid's completion time is stamped once
__device__ void mirror(const BatchEntry &E, const CgState *cs, BatchStatus *stat, int slot, bool final_state) {
  BatchMirror &m = stat[E.problem].m[slot];
  m.done = cs->done;
  m.iter = cs->iter;
  m.status = cs->status;
  m.rho = cs->rho;
  m.bnorm2 = cs->bnorm2;
  m.rho0 = cs->rho0;
  m.stop2 = cs->stop2;
  if (final_state && E.finest && cs->done && stat[E.problem].t_done == 0)
    stat[E.problem].t_done = (long long)wall_clock64();
}

__global__ void b_init_kernel(BatchStatus *stat, int count, long long *t0) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < count) {
    BatchStatus z = {};
    stat[q] = z;
  }
  if (q == 0) *t0 = (long long)wall_clock64();
}

// lds_nodes: the dynamic LDS of the launch, in doubles (entries whose grid does not fit use the global-memory form)
__global__ __launch_bounds__(DT) void b_small_cg_kernel(BatchList L, BatchStatus *stat, int lds_nodes) {
  extern __shared__ double lds_p[];
  const BatchEntry &E = *L.ent[blockIdx.x];
  const int cap = E.cap;  // grids 0 and 1: the direct solve's cap
  if (E.exact && dst_fits(E.g))
    dst_solve_body(E.g, E.u, E.rs, E.st, E.cs, E.r, E.p0);
  else if (small_fits_lds(E.g) && small_lds_nodes(E.g) <= lds_nodes)
    small_cg_lds_body(E.g, E.u, E.rs, E.g, E.r, E.st, E.cs, E.tol, cap, E.exact, 0, lds_p);
  else
    small_cg_body(E.g, E.u, E.rs, E.g, E.r, E.p0, E.p1, E.st, E.cs, E.tol, cap, E.exact, 0);
  if (threadIdx.x == 0) mirror(E, E.cs, stat, 0, true);
}

__global__ __launch_bounds__(256) void b_boundary_terms_kernel(BatchList L) {
  const int e = find_entry(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const Grid g = E.g;
  const int m = max(g.nx, max(g.ny, g.nz)) - 1;
  const int gx = (m + 255) / 256;
  const int lb = blockIdx.x - L.pre[e];
  boundary_terms_block(E.rs, g, E.r, lb % gx, (lb / gx) % m, lb / (gx * m));
}

__global__ __launch_bounds__(NT) void b_residual_kernel(BatchList L) {
  __shared__ double tile[2][kTileRows][TX + 2];
  __shared__ double sh[NT / 64];
  __shared__ double tileF[2][kTileRows][TX + 2];
  const int e = find_entry(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const int bid = blockIdx.x - L.pre[e], nb = L.pre[e + 1] - L.pre[e];
  const Sweep sw = E.swR;
  PolResid<true> pol{E.u, E.r, RhsPart{E.rs, sw.g.nx, sw.g.ny, sw.g.nz, E.r, {0.0, 0.0, 0.0}}};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double>(sw, pol, a0, a1, tile, tileF, bid, nb, false);
  const double v[2] = {a0, a1};
  write_partials<2>(v, E.parts, sh, bid, nb);
}

__global__ __launch_bounds__(FT) void b_finalize_init_kernel(BatchList L, BatchStatus *stat) {
  __shared__ double sh[FT / 64 + 1];
  const BatchEntry &E = *L.ent[blockIdx.x];
  const int nb = L.pre[blockIdx.x + 1] - L.pre[blockIdx.x];
  const double rho = fixed_sum(E.parts, nb, sh);
  const double bb = fixed_sum(E.parts + nb, nb, sh);
  if (threadIdx.x == 0) {
    state_init(E.cs, rho, bb, E.tol, E.cap, 0);
    mirror(E, E.cs, stat, 0, true);
  }
}

// FP64 residual and its FP32 copy for outer step aux[e] of the refinement
__global__ __launch_bounds__(NT) void b_residual_cast_kernel(BatchList L) {
  __shared__ double tile[2][kTileRows][TX + 2];
  __shared__ double sh[NT / 64];
  __shared__ double tileF[2][kTileRows][TX + 2];
  const int e = find_entry(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const int bid = blockIdx.x - L.pre[e], nb = L.pre[e + 1] - L.pre[e];
  const Sweep sw = E.swR;
  PolResidCast<true> pol{E.u, E.g32, E.r32, E.d32, RhsPart{E.rs, sw.g.nx, sw.g.ny, sw.g.nz, E.r, {0.0, 0.0, 0.0}}, 0.0};
  double a0 = 0.0, a1 = 0.0;
  zmarch<double>(sw, pol, a0, a1, tile, tileF, bid, nb, false);
  const double v[3] = {a0, a1, pol.acc2};
  write_partials<3>(v, E.parts, sh, bid, nb);
}

__global__ __launch_bounds__(FT) void b_finalize_ir_kernel(BatchList L, BatchStatus *stat) {
  __shared__ double sh[FT / 64 + 1];
  const BatchEntry &E = *L.ent[blockIdx.x];
  const int nb = L.pre[blockIdx.x + 1] - L.pre[blockIdx.x];
  const double r64 = fixed_sum(E.parts, nb, sh);
  const double bb = fixed_sum(E.parts + nb, nb, sh);
  const double r32 = fixed_sum(E.parts + 2 * nb, nb, sh);
  if (threadIdx.x == 0) {
    state_ir(E.cs, E.cs2, r64, bb, r32, E.tol, E.eta, L.aux[blockIdx.x], E.max_outer, E.cap);
    mirror(E, E.cs, stat, 0, true);
    mirror(E, E.cs2, stat, 1, false);
  }
}

template <typename T, int TY, int D>
__global__ __launch_bounds__(Tile<TY>::NT) void b_pass_a_kernel(BatchList L) {
  constexpr bool F = sizeof(T) == 4;
  __shared__ T tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[Tile<TY>::NT / 64];
  const int e = find_entry(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const CgState *cs = F ? E.cs2 : E.cs;
  if (cs->done) return;
  const int bid = blockIdx.x - L.pre[e], nb = L.pre[e + 1] - L.pre[e];
  const int it = cs->iter;
  T *p0, *p1, *r;
  if constexpr (F) {
    r = E.r32; p0 = E.p32a; p1 = E.p32b;
  } else {
    r = E.r; p0 = E.p0; p1 = E.p1;
  }
  const CgBufs<T> bf = cg_bufs(it, r, p0, p1);
  const Sweep sw = F ? E.swA32 : E.swA;
  double a0 = 0.0;
  // the batch's working set is far larger than the caches: streaming policy
  pass_a_march<T, D, true, TY>(sw, it, bf, (T)cs->beta, a0, tile, bid, nb, false);
  const double v[1] = {a0};
  write_partials<1, Tile<TY>::NT>(v, E.parts, sh, bid, nb);
}

template <typename T, int TY, int D>
__global__ __launch_bounds__(Tile<TY>::NT) void b_pass_b_kernel(BatchList L) {
  constexpr bool F = sizeof(T) == 4;
  __shared__ T tile[2][Tile<TY>::Rows][TX + 2];
  __shared__ double sh[Tile<TY>::NT / 64];
  const int e = find_entry(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const CgState *cs = F ? E.cs2 : E.cs;
  if (cs->done) return;
  const int bid = blockIdx.x - L.pre[e], nb = L.pre[e + 1] - L.pre[e];
  const int it = cs->iter;
  T *p0, *p1, *r, *uu;
  if constexpr (F) {
    r = E.r32; p0 = E.p32a; p1 = E.p32b;
    uu = E.d32;
  } else {
    r = E.r; p0 = E.p0; p1 = E.p1;
    uu = E.u;
  }
  const CgBufs<T> bf = cg_bufs(it, r, p0, p1);
  const Sweep sw = F ? E.swB32 : E.swB;
  double a0 = 0.0;
  pass_b_march<T, D, true, TY>(sw, it, bf, uu, (T)cs->alpha, a0, tile, bid, nb, false);
  const double v[1] = {a0};
  write_partials<1, Tile<TY>::NT>(v, E.parts, sh, bid, nb);
}

// reduction after pass A (PASS 0) or pass B (PASS 1) of the FP64 CG (F = 0) or the FP32 inner CG (F = 1)
template <int PASS, int F>
__global__ __launch_bounds__(FT) void b_finalize_pass_kernel(BatchList L, BatchStatus *stat) {
  __shared__ double sh[FT / 64 + 1];
  const BatchEntry &E = *L.ent[blockIdx.x];
  CgState *cs = F ? E.cs2 : E.cs;
  if (cs->done) return;
  const int nb = L.pre[blockIdx.x + 1] - L.pre[blockIdx.x];
  const double v = fixed_sum(E.parts, nb, sh);
  if (threadIdx.x == 0) {
    if (PASS == 0) state_after_a(cs, v);
    else state_after_b(cs, v);
    mirror(E, cs, stat, F, F == 0);
  }
}

// the trial state of the autotuner in both CG states of every entry of L (one thread per entry)
__global__ void b_tune_state_kernel(BatchList L) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= L.n) return;
  tune_state(L.ent[q]->cs);
  tune_state(L.ent[q]->cs2);
}

__global__ __launch_bounds__(256) void b_add_correction_kernel(BatchList L) {
  const int e = find_entry(L.pre, L.n, blockIdx.x);
  const BatchEntry &E = *L.ent[e];
  const Grid g = E.g;
  const int gx = (g.nx - 1 + 255) / 256, gy = g.ny - 1;
  const int lb = blockIdx.x - L.pre[e];
  add_correction_block(g, E.u, E.g32, E.d32, lb % gx, (lb / gx) % gy, lb / (gx * gy));
}

}  // namespace

// ------------------------------------------------------------------------------------------------------- launchers

// z chunk per workgroup (even, so that the first output plane of every workgroup is odd).  Default: 16 planes, or
// fewer while the grid has under 2048 workgroups (8 per CU).  The autotuner replaces it per grid and pass.
Sweep make_sweep(const Grid &g, const Stencil &s, int zc, int depth, int nt, int ty) {
  Sweep sw;
  sw.depth = (depth == 3 || depth == 4 || depth == 6) ? depth : 2;
  sw.nt = nt ? 1 : 0;
  sw.ty = (ty == 8 || ty == 16) ? ty : kTy;
  sw.g = g;
  sw.st = s;
  sw.ntx = (g.nx - 1 + TX - 1) / TX;
  sw.nty = (g.ny - 1 + sw.ty - 1) / sw.ty;
  const long long tiles = (long long)sw.ntx * sw.nty;
  if (zc <= 0) {
    zc = 16;
    while (zc > 2 && tiles * ((g.nz - 1 + zc - 1) / zc) < 2048) zc /= 2;
  }
  zc = zc < 2 ? 2 : (zc & ~1);
  sw.zc = zc;
  sw.nzc = (g.nz - 1 + zc - 1) / zc;
  return sw;
}

int sweep_blocks(const Sweep &sw) { return sw.ntx * sw.nty * sw.nzc; }

Sweep with_height(const Sweep &sw, int ty) {
  return sw.ty == ty ? sw : make_sweep(sw.g, sw.st, sw.zc, sw.depth, sw.nt, ty);
}

Sweep default_height(const Sweep &sw) { return with_height(sw, kTy); }

long long cg_partials_needed(const Grid &g) {
  const Sweep sw = make_sweep(g, Stencil{}, 2, 2, 0, 4);  // the smallest chunk and tile give the most workgroups
  return 3LL * sweep_blocks(sw) + 64;
}

// f(depth, policy, height) with the sweep's prefetch depth, cache policy and tile height as compile-time constants.
template <typename F>
static void with_shape(const Sweep &sw, F &&f) {
  auto height = [&](auto d, auto n) {
    switch (sw.ty) {
      case 8: f(d, n, std::integral_constant<int, 8>{}); break;
      case 16: f(d, n, std::integral_constant<int, 16>{}); break;
      default: f(d, n, std::integral_constant<int, kTy>{}); break;
    }
  };
  auto pol = [&](auto d) {
    if (sw.nt) height(d, std::true_type{});
    else height(d, std::false_type{});
  };
  switch (sw.depth) {
    case 3: pol(std::integral_constant<int, 3>{}); break;
    case 4: pol(std::integral_constant<int, 4>{}); break;
    case 6: pol(std::integral_constant<int, 6>{}); break;
    default: pol(std::integral_constant<int, 2>{}); break;
  }
}

static void launch_boundary_terms(const RhsSrc &rs, const Grid &g, double *out, hipStream_t st) {
  if (rs.mode != 0) return;
  const int m = (g.nx > g.ny ? (g.nx > g.nz ? g.nx : g.nz) : (g.ny > g.nz ? g.ny : g.nz)) - 1;
  dim3 grid((m + 255) / 256, m, 6);
  boundary_terms_kernel<<<grid, 256, 0, st>>>(rs, g, out);
}

static void launch_resid(const Sweep &sw_in, const double *u, const RhsSrc &rs, double *r, double *parts,
                         hipStream_t st) {
  const Sweep sw = default_height(sw_in);  // the residual kernels are built for 4-row tiles only
  const int nb = sweep_blocks(sw);
  const int v = (sw.depth == 3 ? 2 : 0) + sw.nt;
  if (v == 0) residual_kernel<2, false><<<nb, NT, 0, st>>>(sw, u, rs, r, parts);
  else if (v == 1) residual_kernel<2, true><<<nb, NT, 0, st>>>(sw, u, rs, r, parts);
  else if (v == 2) residual_kernel<3, false><<<nb, NT, 0, st>>>(sw, u, rs, r, parts);
  else residual_kernel<3, true><<<nb, NT, 0, st>>>(sw, u, rs, r, parts);
}

void launch_residual_partials(const Sweep &sw, const double *u, const RhsSrc &rs, double *r, double *parts,
                              hipStream_t st) {
  launch_boundary_terms(rs, sw.g, r, st);
  launch_resid(sw, u, rs, r, parts, st);
}

void launch_boundary_g2(const RhsSrc &rs, const Grid &g, CgState *cs, hipStream_t st) {
  boundary_g2_kernel<<<1, FT, 0, st>>>(rs, g, cs);
}

void launch_clear_gbnd2(CgState *a, CgState *b, hipStream_t st) { clear_gbnd2_kernel<<<1, 1, 0, st>>>(a, b); }

void launch_selfred_init(CgState *cs, int max_iters, int hist_on, int preset, hipStream_t st) {
  selfred_init_kernel<<<1, 1, 0, st>>>(cs, max_iters, hist_on, preset);
}

template <typename T>
void launch_selfred_a(const Sweep &swA, T *r, T *p0, T *p1, CgState *cs, const double *partsB, int nb_prev,
                      double tol, double *partsA, hipStream_t st) {
  with_shape(swA, [&](auto d, auto n, auto ty) {
    constexpr int TY = decltype(ty)::value;
    cg_selfred_a_kernel<T, decltype(d)::value, decltype(n)::value, TY>
        <<<sweep_blocks(swA), Tile<TY>::NT, 0, st>>>(swA, r, p0, p1, cs, partsB, nb_prev, tol, partsA);
  });
}

template <typename T>
void launch_selfred_b(const Sweep &swB, T *u, T *r, T *p0, T *p1, CgState *cs, const double *partsA,
                      int nbA, double *partsB, hipStream_t st) {
  with_shape(swB, [&](auto d, auto n, auto ty) {
    constexpr int TY = decltype(ty)::value;
    cg_selfred_b_kernel<T, decltype(d)::value, decltype(n)::value, TY>
        <<<sweep_blocks(swB), Tile<TY>::NT, 0, st>>>(swB, u, r, p0, p1, cs, partsA, nbA, partsB);
  });
}

template void launch_selfred_a<double>(const Sweep &, double *, double *, double *, CgState *, const double *,
                                       int, double, double *, hipStream_t);
template void launch_selfred_a<float>(const Sweep &, float *, float *, float *, CgState *, const double *, int,
                                      double, double *, hipStream_t);
template void launch_selfred_b<double>(const Sweep &, double *, double *, double *, double *, CgState *,
                                       const double *, int, double *, hipStream_t);
template void launch_selfred_b<float>(const Sweep &, float *, float *, float *, float *, CgState *,
                                      const double *, int, double *, hipStream_t);

int selfred_max_blocks() { return kSelfRedMaxBlocks; }

// f(depth, height) for the single-reduction CG sweeps, which prefetch 2 or 3 planes (a deeper depth runs as 3)
template <typename F>
static void with_cg1_shape(const Sweep &sw, F &&f) {
  auto height = [&](auto d) {
    switch (sw.ty) {
      case 8: f(d, std::integral_constant<int, 8>{}); break;
      case 16: f(d, std::integral_constant<int, 16>{}); break;
      default: f(d, std::integral_constant<int, kTy>{}); break;
    }
  };
  if (sw.depth >= 3) height(std::integral_constant<int, 3>{});
  else height(std::integral_constant<int, 2>{});
}

void launch_cg1_init(const Sweep &sw, const double *r, double *w, double *parts, hipStream_t st) {
  with_cg1_shape(sw, [&](auto d, auto ty) {
    constexpr int TY = decltype(ty)::value;
    cg1_init_kernel<decltype(d)::value, TY><<<sweep_blocks(sw), Tile<TY>::NT, 0, st>>>(sw, r, w, parts);
  });
}

void launch_cg1_iteration(const Sweep &sw, double *u, double *p, const double *r, const double *w, const double *s,
                          double *ro, double *wo, double *so, CgState *cs, int par, const double *partsIn,
                          const double *partsR, int nbR, double tol, double *partsOut, hipStream_t st) {
  with_cg1_shape(sw, [&](auto d, auto ty) {
    constexpr int TY = decltype(ty)::value;
    cg1_iter_kernel<decltype(d)::value, TY><<<sweep_blocks(sw), Tile<TY>::NT, 0, st>>>(
        sw, u, p, r, w, s, ro, wo, so, cs, par, partsIn, partsR, nbR, tol, partsOut);
  });
}

void launch_residual(const Sweep &sw_in, const double *u, const RhsSrc &rs, double *r, CgState *cs, double *partials,
                     double tol, int max_iters, int hist_on, hipStream_t st) {
  const Sweep sw = default_height(sw_in);
  const int nb = sweep_blocks(sw);
  launch_boundary_terms(rs, sw.g, r, st);
  launch_resid(sw, u, rs, r, partials, st);
  finalize_init_kernel<<<1, FT, 0, st>>>(cs, partials, nb, tol, max_iters, hist_on);
}

void launch_residual_cast(const Sweep &sw_in, const double *u, const RhsSrc &rs, double *bterm, const Grid &g32,
                          float *r32, float *d32, CgState *outer, CgState *inner, double *partials, double tol,
                          double eta, int outer_step, int max_outer, int max_inner, hipStream_t st) {
  const Sweep sw = default_height(sw_in);
  const int nb = sweep_blocks(sw);
  launch_boundary_terms(rs, sw.g, bterm, st);
  const int v = (sw.depth == 3 ? 2 : 0) + sw.nt;
  if (v == 0) residual_cast_kernel<2, false><<<nb, NT, 0, st>>>(sw, u, rs, bterm, g32, r32, d32, partials);
  else if (v == 1) residual_cast_kernel<2, true><<<nb, NT, 0, st>>>(sw, u, rs, bterm, g32, r32, d32, partials);
  else if (v == 2) residual_cast_kernel<3, false><<<nb, NT, 0, st>>>(sw, u, rs, bterm, g32, r32, d32, partials);
  else residual_cast_kernel<3, true><<<nb, NT, 0, st>>>(sw, u, rs, bterm, g32, r32, d32, partials);
  finalize_ir_kernel<<<1, FT, 0, st>>>(outer, inner, partials, nb, tol, eta, outer_step, max_outer, max_inner);
}

template <typename T>
void launch_cg_pass_a(const Sweep &sw, T *r, T *p0, T *p1, CgState *cs, double *partials, hipStream_t st) {
  const int nb = sweep_blocks(sw);
  with_shape(sw, [&](auto d, auto n, auto ty) {
    constexpr int TY = decltype(ty)::value;
    cg_pass_a_kernel<T, decltype(d)::value, decltype(n)::value, TY>
        <<<nb, Tile<TY>::NT, 0, st>>>(sw, r, p0, p1, cs, partials);
  });
  finalize_a_kernel<<<1, FT, 0, st>>>(cs, partials, nb);
}

template <typename T>
void launch_cg_pass_b(const Sweep &sw, T *u, T *r, T *p0, T *p1, CgState *cs, double *partials,
                      hipStream_t st) {
  const int nb = sweep_blocks(sw);
  with_shape(sw, [&](auto d, auto n, auto ty) {
    constexpr int TY = decltype(ty)::value;
    cg_pass_b_kernel<T, decltype(d)::value, decltype(n)::value, TY>
        <<<nb, Tile<TY>::NT, 0, st>>>(sw, u, r, p0, p1, cs, partials);
  });
  finalize_b_kernel<<<1, FT, 0, st>>>(cs, partials, nb);
}

template void launch_cg_pass_a<double>(const Sweep &, double *, double *, double *, CgState *, double *,
                                       hipStream_t);
template void launch_cg_pass_a<float>(const Sweep &, float *, float *, float *, CgState *, double *,
                                      hipStream_t);
template void launch_cg_pass_b<double>(const Sweep &, double *, double *, double *, double *, CgState *,
                                       double *, hipStream_t);
template void launch_cg_pass_b<float>(const Sweep &, float *, float *, float *, float *, CgState *,
                                      double *, hipStream_t);

void launch_tune_state(CgState *cs, int iter, hipStream_t st) { tune_state_kernel<<<1, 1, 0, st>>>(cs, iter); }

void launch_tune_selfred(CgState *cs, double *parts, int n, hipStream_t st) {
  tune_selfred_kernel<<<1, 256, 0, st>>>(cs, parts, n);
}

void launch_delay(double us, hipStream_t st) { delay_kernel<<<1, 64, 0, st>>>((long long)(us * 100.0)); }

void launch_add_correction(const Grid &gu, double *u, const Grid &g32, const float *d32, hipStream_t st) {
  dim3 grid((gu.nx - 1 + 255) / 256, gu.ny - 1, gu.nz - 1);
  add_correction_kernel<<<grid, 256, 0, st>>>(gu, u, g32, d32);
}

void launch_small_cg(const Grid &gu, double *u, const RhsSrc &rs, const Grid &gw, double *r, double *p, double *q,
                     const Stencil &s, CgState *cs, double tol, int max_iters, int exact, int hist_on,
                     hipStream_t st) {
  const int cap = exact ? dsolve_cap(gu.interior()) : max_iters;
  const size_t lds = (!(exact && dst_fits(gu)) && small_fits_lds(gu)) ? (size_t)small_lds_nodes(gu) * sizeof(double)
                                                                        : 0;
  small_cg_kernel<<<1, DT, lds, st>>>(gu, u, rs, gw, r, p, q, s, cs, tol, cap, exact, hist_on);
}

void launch_apply(const Grid &gx, const double *x, const Grid &gy, double *y, const Stencil &s, hipStream_t st) {
  const Sweep sw = make_sweep(gx, s, 0);
  apply_kernel<<<sweep_blocks(sw), NT, 0, st>>>(sw, x, gy, y);
}


// ---------------------------------------------------------------------------------------------- batched launchers

int b_blocks_interior(const Grid &g) { return ((g.nx - 1 + 255) / 256) * (g.ny - 1) * (g.nz - 1); }

int b_blocks_bterms(const Grid &g) {
  const int m = (g.nx > g.ny ? (g.nx > g.nz ? g.nx : g.nz) : (g.ny > g.nz ? g.ny : g.nz)) - 1;
  return ((m + 255) / 256) * m * 6;
}

void launch_b_init(BatchStatus *stat, int count, long long *t0, hipStream_t st) {
  b_init_kernel<<<(count + 255) / 256, 256, 0, st>>>(stat, count, t0);
}

void launch_b_small_cg(const BatchList &L, int lds_nodes, BatchStatus *stat, hipStream_t st) {
  if (L.n > 0) b_small_cg_kernel<<<L.n, DT, (size_t)lds_nodes * sizeof(double), st>>>(L, stat, lds_nodes);
}

int b_small_lds_nodes(const Grid &g) { return small_fits_lds(g) ? (int)small_lds_nodes(g) : 0; }

void launch_b_boundary_terms(const BatchList &L, hipStream_t st) {
  if (L.total > 0) b_boundary_terms_kernel<<<L.total, 256, 0, st>>>(L);
}

void launch_b_residual(const BatchList &L, BatchStatus *stat, hipStream_t st) {
  if (L.total <= 0) return;
  b_residual_kernel<<<L.total, NT, 0, st>>>(L);
  b_finalize_init_kernel<<<L.n, FT, 0, st>>>(L, stat);
}

void launch_b_residual_cast(const BatchList &L, BatchStatus *stat, hipStream_t st) {
  if (L.total <= 0) return;
  b_residual_cast_kernel<<<L.total, NT, 0, st>>>(L);
  b_finalize_ir_kernel<<<L.n, FT, 0, st>>>(L, stat);
}

// f(integral_constant<int, ty>, integral_constant<int, depth>) for a batched pass shape: tile height 4, 8 or 16 rows
// (4 for anything else) and prefetch depth 2, 3, 4 or 6 (2 for anything else)
template <typename F>
static void with_batch_shape(int ty, int depth, F &&f) {
  auto dep = [&](auto h) {
    switch (depth) {
      case 3: f(h, std::integral_constant<int, 3>{}); break;
      case 4: f(h, std::integral_constant<int, 4>{}); break;
      case 6: f(h, std::integral_constant<int, 6>{}); break;
      default: f(h, std::integral_constant<int, 2>{}); break;
    }
  };
  switch (ty) {
    case 8: dep(std::integral_constant<int, 8>{}); break;
    case 16: dep(std::integral_constant<int, 16>{}); break;
    default: dep(std::integral_constant<int, kTy>{}); break;
  }
}

void launch_b_iteration(int fp32, int ty, int depth, const BatchList &A, const BatchList &B, BatchStatus *stat,
                        hipStream_t st) {
  if (A.total <= 0 || B.total <= 0) return;
  with_batch_shape(ty, depth, [&](auto h, auto d) {
    constexpr int TY = decltype(h)::value, D = decltype(d)::value;
    if (fp32) {
      b_pass_a_kernel<float, TY, D><<<A.total, Tile<TY>::NT, 0, st>>>(A);
      b_finalize_pass_kernel<0, 1><<<A.n, FT, 0, st>>>(A, stat);
      b_pass_b_kernel<float, TY, D><<<B.total, Tile<TY>::NT, 0, st>>>(B);
      b_finalize_pass_kernel<1, 1><<<B.n, FT, 0, st>>>(B, stat);
    } else {
      b_pass_a_kernel<double, TY, D><<<A.total, Tile<TY>::NT, 0, st>>>(A);
      b_finalize_pass_kernel<0, 0><<<A.n, FT, 0, st>>>(A, stat);
      b_pass_b_kernel<double, TY, D><<<B.total, Tile<TY>::NT, 0, st>>>(B);
      b_finalize_pass_kernel<1, 0><<<B.n, FT, 0, st>>>(B, stat);
    }
  });
}

void launch_b_tune_state(const BatchList &L, hipStream_t st) {
  if (L.n > 0) b_tune_state_kernel<<<(L.n + 255) / 256, 256, 0, st>>>(L);
}

void launch_b_passes(int fp32, int ty, int depth, const BatchList &A, const BatchList &B, hipStream_t st) {
  if (A.total <= 0 || B.total <= 0) return;
  with_batch_shape(ty, depth, [&](auto h, auto d) {
    constexpr int TY = decltype(h)::value, D = decltype(d)::value;
    if (fp32) {
      b_pass_a_kernel<float, TY, D><<<A.total, Tile<TY>::NT, 0, st>>>(A);
      b_pass_b_kernel<float, TY, D><<<B.total, Tile<TY>::NT, 0, st>>>(B);
    } else {
      b_pass_a_kernel<double, TY, D><<<A.total, Tile<TY>::NT, 0, st>>>(A);
      b_pass_b_kernel<double, TY, D><<<B.total, Tile<TY>::NT, 0, st>>>(B);
    }
  });
}

void launch_b_add_correction(const BatchList &L, hipStream_t st) {
  if (L.total > 0) b_add_correction_kernel<<<L.total, 256, 0, st>>>(L);
}

void launch_publish(const void *src, void *dst, size_t bytes, hipStream_t st) {
  publish_kernel<<<1, 256, 0, st>>>((const unsigned long long *)src, (unsigned long long *)dst, (int)(bytes / 8));
}

}  // namespace excmg
