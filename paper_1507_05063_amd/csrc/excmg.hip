// Host driver and C ABI of the gfx950 EXCMG solver (Algorithm 1 of Pan, He & Hu, arXiv 1507.05063).
//
// Per grid of the cascade (coarsest first):
//   level data   b_l = -R f_l + A_IB g_l, with f_l, g_l the finest arrays at stride 2^(L-1-l)  (Section 2, eq. compact),
//                formed on the fly by every kernel that needs it (never stored)
//   grids 0, 1   DSOLVE: single-workgroup CG to rounding                                     (Algorithm 1, coarsest grids)
//   grids >= 2   w = EXP_finite(u_{l-1}, u_{l-2}), then CG from w until ||r|| <= tol ||b||   (Algorithm 1, the loop):
//                one single-workgroup launch on grids of at most 8000 unknowns, otherwise two stencil sweeps and
//                two single-workgroup reductions per iteration
//   finest       u_ext = EXP_true(u_h, u_2h) on request; u copied to the caller's dense array
// The library allocates no device memory: every array lives in the caller's workspace.  The host reads the CG state
// back (one small copy and a stream sync) after every batch of iterations; iterations launched after convergence
// return at once (every CG kernel checks the device-side done flag first).
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <vector>

#include "excmg_internal.h"

using namespace excmg;

namespace {

struct Level {
  int n[3];
  double h[3];
  int stride;  // sampling stride into the finest arrays
  Grid g;      // pitched FP64 layout of this grid's arrays
  Grid g32;    // pitched FP32 layout
  Stencil st;
  Sweep sw, sw32;  // stencil sweeps over g and g32 (residual kernels)
  Sweep swA, swB, swA32, swB32;  // CG passes A and B in FP64 and FP32 (z chunk chosen by the autotuner)
  Sweep swA0, swB0;  // the FP64 passes of a grid's first iteration (p = r), on grids whose passes finalize apart
  double *u;   // this grid's solution, all nodes (boundary = g)
};

struct Layout {
  int L;
  int nc[3];
  Level lev[EXCMG_MAX_LEVELS];
  Grid gdense;
  Grid gfin, gfin32;
  // byte offsets into the workspace
  size_t off_u[EXCMG_MAX_LEVELS];
  size_t off_r, off_p0, off_p1;
  size_t off_r32, off_p32a, off_p32b, off_d32;
  size_t off_part, off_cs, off_cs2, off_defer, off_invm[3], off_flag;
  long long npart;
  size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

int plan_levels(const excmg_problem *p, int *L_out, int nc[3]) {
  for (int d = 0; d < 3; ++d)
    if (p->n[d] < 2) return EXCMG_ERR_SHAPE;
  int c[3] = {p->n_coarse[0], p->n_coarse[1], p->n_coarse[2]};
  if (c[0] == 0 && c[1] == 0 && c[2] == 0) {
    c[0] = p->n[0]; c[1] = p->n[1]; c[2] = p->n[2];
    // halve while the halved counts are all even (so they can feed EXP_finite), >= 2, and the largest is >= 4
    for (;;) {
      const bool even = !(c[0] & 1) && !(c[1] & 1) && !(c[2] & 1);
      const int h0 = c[0] / 2, h1 = c[1] / 2, h2 = c[2] / 2;
      const bool heven = !(h0 & 1) && !(h1 & 1) && !(h2 & 1);
      const int mx = h0 > h1 ? (h0 > h2 ? h0 : h2) : (h1 > h2 ? h1 : h2);
      if (!even || !heven || h0 < 2 || h1 < 2 || h2 < 2 || mx < 4) break;
      c[0] = h0; c[1] = h1; c[2] = h2;
    }
  }
  if (c[0] < 2 || c[1] < 2 || c[2] < 2) return EXCMG_ERR_SHAPE;
  int L = -1;
  for (int t = 0; t < EXCMG_MAX_LEVELS; ++t) {
    if ((long long)c[0] << t == p->n[0] && (long long)c[1] << t == p->n[1] && (long long)c[2] << t == p->n[2]) {
      L = t + 1;
      break;
    }
  }
  if (L < 0) return EXCMG_ERR_SHAPE;
  if (L >= 3 && ((c[0] & 1) || (c[1] & 1) || (c[2] & 1))) return EXCMG_ERR_SHAPE;
  *L_out = L;
  nc[0] = c[0]; nc[1] = c[1]; nc[2] = c[2];
  return EXCMG_OK;
}

int validate(const excmg_problem *p) {
  if (!p) return EXCMG_ERR_ARG;
  for (int d = 0; d < 3; ++d)
    if (!(p->box[d] > 0.0) || !isfinite(p->box[d])) return EXCMG_ERR_ARG;
  if (!(p->tol > 0.0) || !isfinite(p->tol)) return EXCMG_ERR_ARG;
  if (p->precision != EXCMG_FP64 && p->precision != EXCMG_FP32_IR) return EXCMG_ERR_ARG;
  if (p->inner_tol < 0.0 || !isfinite(p->inner_tol) || p->inner_tol >= 1.0) return EXCMG_ERR_ARG;
  if (p->max_iters < 0) return EXCMG_ERR_ARG;
  if (p->flags & ~(EXCMG_WANT_HISTORY | EXCMG_WANT_TIMING | EXCMG_NO_GRAPHS | EXCMG_GUESS_QUADRATIC |
                   EXCMG_GUESS_LINEAR | EXCMG_STOP_F_G | EXCMG_STOP_F_G_BELOW_FINEST | EXCMG_TWO_PASS_CG))
    return EXCMG_ERR_ARG;
  if ((p->flags & EXCMG_GUESS_QUADRATIC) && (p->flags & EXCMG_GUESS_LINEAR)) return EXCMG_ERR_ARG;
  if ((p->flags & EXCMG_STOP_F_G) && (p->flags & EXCMG_STOP_F_G_BELOW_FINEST)) return EXCMG_ERR_ARG;
  if (!(p->tol_order >= 0.0) || p->tol_order > 16.0) return EXCMG_ERR_ARG;
  if (!(p->tol_coarse >= 0.0) || !(p->tol_coarse < 1.0) || (p->tol_coarse > 0.0 && p->tol_order > 0.0))
    return EXCMG_ERR_ARG;
  return EXCMG_OK;
}

// z planes per workgroup of the residual sweeps on large grids
constexpr int kResidChunk = 64;

// The relative-residual tolerance of grid l: tol on every grid; with tol_coarse > 0, tol_coarse on every grid below
// the finest; or with tol_order = p > 0, tol * 2^(p (L-1-l)) capped at max(tol, 1e-2) (tol on the finest grid, looser
// on each coarser one).
double level_tol(const excmg_problem &p, int l, int L) {
  if (p.tol_coarse > 0.0) return l < L - 1 ? p.tol_coarse : p.tol;
  if (!(p.tol_order > 0.0)) return p.tol;
  const double cap = p.tol > 1e-2 ? p.tol : 1e-2;
  const double t = p.tol * exp2(p.tol_order * (double)(L - 1 - l));
  return t < cap ? t : cap;
}

// Tolerance and iteration cap of grid l's CG: the direct solves (grids 0 and 1) iterate to rounding
double grid_tol(const excmg_problem &p, int l, int L) { return l <= 1 ? kDsolveTol : level_tol(p, l, L); }

int guess_kind(uint32_t flags) {
  if (flags & EXCMG_GUESS_QUADRATIC) return kGuessQuadratic;
  if (flags & EXCMG_GUESS_LINEAR) return kGuessLinear;
  return kGuessQuartic;
}

// Events that only take timestamps: no system-scope fence at record (the cache write-back and invalidation it
// costs would sit between the timed kernels).  Results are read on the host only after a stream synchronization.
constexpr unsigned kTimingEvent = hipEventDisableSystemFence;

// bytes of a CG state that the host reads after a solve (everything but the history)
constexpr size_t kStateHead = offsetof(CgState, hist);

int make_layout(const excmg_problem *p, Layout *Lo) {
  int e = validate(p);
  if (e) return e;
  e = plan_levels(p, &Lo->L, Lo->nc);
  if (e) return e;
  const int L = Lo->L;
  size_t off = 0;
  for (int l = 0; l < L; ++l) {
    Level &lv = Lo->lev[l];
    for (int d = 0; d < 3; ++d) {
      lv.n[d] = Lo->nc[d] << l;
      lv.h[d] = p->box[d] / lv.n[d];
    }
    lv.stride = 1 << (L - 1 - l);
    lv.g = pitched_grid<double>(lv.n[0], lv.n[1], lv.n[2]);
    lv.g32 = pitched_grid<float>(lv.n[0], lv.n[1], lv.n[2]);
    lv.st = make_stencil(lv.h[0], lv.h[1], lv.h[2]);
    // The residual sweep runs once or twice per grid.  On grids far larger than the caches: streaming stores, and
    // long z chunks, since every chunk reads two extra planes of u and of f.
    const bool big = lv.g.interior() >= (1LL << 23);
    lv.sw = make_sweep(lv.g, lv.st, big ? kResidChunk : 0, 2, big ? 1 : 0);
    lv.sw32 = make_sweep(lv.g32, lv.st, 0);
    lv.swA = lv.swB = make_sweep(lv.g, lv.st, 0, 2, big ? 1 : 0);
    lv.swA0 = lv.swB0 = lv.swA;
    lv.swA32 = lv.swB32 = lv.sw32;
    lv.u = nullptr;
    Lo->off_u[l] = off;
    off = align256(off + (size_t)lv.g.elems * sizeof(double));
  }
  const Level &fin = Lo->lev[L - 1];
  Lo->gdense = dense_grid(fin.n[0], fin.n[1], fin.n[2]);
  Lo->gfin = fin.g;
  Lo->gfin32 = fin.g32;
  // no right-hand-side array: every kernel that needs b forms it from the finest f and g (rhs_at)
  const size_t v64 = align256((size_t)fin.g.elems * sizeof(double));
  Lo->off_r = off; off += v64;
  Lo->off_p0 = off; off += v64;
  Lo->off_p1 = off; off += v64;
  if (p->precision == EXCMG_FP32_IR) {
    const size_t v32 = align256((size_t)fin.g32.elems * sizeof(float));
    Lo->off_r32 = off; off += v32;
    Lo->off_p32a = off; off += v32;
    Lo->off_p32b = off; off += v32;
    Lo->off_d32 = off; off += v32;
  } else {
    Lo->off_r32 = Lo->off_p32a = Lo->off_p32b = Lo->off_d32 = 0;
  }
  Lo->npart = cg_partials_needed(fin.g);
  Lo->off_part = off; off = align256(off + 2 * (size_t)Lo->npart * sizeof(double));  // two halves: A and B
  Lo->off_cs = off; off = align256(off + sizeof(CgState));
  Lo->off_cs2 = off; off = align256(off + sizeof(CgState));
  Lo->off_defer = off; off = align256(off + EXCMG_MAX_LEVELS * kStateHead);
  for (int d = 0; d < 3; ++d) {
    Lo->off_invm[d] = off;
    off = align256(off + (size_t)(fin.n[d] + 1) * sizeof(double));
  }
  Lo->off_flag = off; off = align256(off + 64);
  Lo->total = off;
  return EXCMG_OK;
}

struct TimedLaunch {
  int cls;
  int level;
  int iter;  // CG iteration index of a CG-class launch (-1: always counted)
  int outer; // FP32_IR outer step (-1 otherwise)
  hipEvent_t a, b;
};

}  // namespace

struct excmg_handle {
  // tile height and prefetch depth of the batched CG passes (FP64, FP32) when this handle leads a batch
  // (excmg_autotune_batched, excmg_set_batch_shape)
  int bty[2] = {4, 4};
  int bdepth[2] = {2, 2};
  excmg_problem p;
  Layout lo;
  hipStream_t stream;
  int device;
  char *ws;
  double *r, *p0, *p1;
  float *r32, *p32a, *p32b, *d32;
  double *partials;
  CgState *cs, *cs2;
  char *defer_dev;  // per grid, the CG state (without its history) of a one-launch solve, read after the cascade
  double *inv_m[3];
  int *flag;
  std::vector<double> inv_m_host[3];
  hipEvent_t lev_ev[EXCMG_MAX_LEVELS + 1];
  // kernel timing
  std::vector<hipEvent_t> pool;
  std::vector<TimedLaunch> timed;
  size_t pool_used;
  bool timing;
  // pinned host memory the device writes CG states (and batch status words) into; pin_dev is its device address
  void *pin_host = nullptr, *pin_dev = nullptr;
  size_t pin_bytes = 0;
  // graphs of 8, 16 and 32 CG iterations per grid (FP64, FP32 inner), captured on first use on a private stream
  hipStream_t cap = nullptr;
  hipGraphExec_t gexec[EXCMG_MAX_LEVELS][2][3] = {};
  // a handle of excmg_solve_noalloc: no events, graphs, capture stream or pinned memory; CG states are read back with
  // plain stream copies
  bool noalloc = false;
  // graphs of a batched round's CG iterations (excmg_solve_batched, on the batch's first handle), by launch shape
  struct BatchGraph {
    std::vector<long long> key;
    hipGraphExec_t ex;
    long long used;  // the count of lookups when last used (the least recently used goes first)
  };
  std::vector<BatchGraph> bgraphs;
  long long bgraph_hits = 0, bgraph_misses = 0;

  void drop_graphs() {
    for (auto &row : gexec)
      for (auto &sizes : row)
        for (auto &ex : sizes)
          if (ex) {
            (void)hipGraphExecDestroy(ex);
            ex = nullptr;
          }
    for (auto &bg : bgraphs) (void)hipGraphExecDestroy(bg.ex);
    bgraphs.clear();
  }

  ~excmg_handle() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
    for (int l = 0; l <= EXCMG_MAX_LEVELS; ++l)
      if (lev_ev[l]) (void)hipEventDestroy(lev_ev[l]);
    for (auto &ev : pool)
      if (ev) (void)hipEventDestroy(ev);
    if (pin_host) (void)hipHostFree(pin_host);
  }
};

namespace {

struct DeviceGuard {
  int prev = -1;
  bool changed = false;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) {
      if (hipSetDevice(dev) == hipSuccess) changed = true;
    }
  }
  ~DeviceGuard() {
    if (changed) (void)hipSetDevice(prev);
  }
};

#define HIPCHECK(x)                       \
  do {                                    \
    if ((x) != hipSuccess) return EXCMG_ERR_HIP; \
  } while (0)

inline int last_error() { return hipGetLastError() == hipSuccess ? EXCMG_OK : EXCMG_ERR_HIP; }

// Kernel timing: a pair of events around each launch on the finest grid when EXCMG_WANT_TIMING is set (the coarser
// grids' launches are replayed from graphs, and their event records would cost as much as the kernels they time).

struct Tick {
  excmg_handle *h;
  int idx;
  Tick(excmg_handle *h_, int cls, int level, int iter = -1, int outer = -1);
  ~Tick() {
    if (idx >= 0) (void)hipEventRecord(h->timed[idx].b, h->stream);
  }
};

Tick::Tick(excmg_handle *h_, int cls, int level, int iter, int outer) : h(h_), idx(-1) {
    if (!h->timing || h->pool_used + 2 > h->pool.size()) return;
    if (level != h->lo.L - 1) return;
    TimedLaunch t;
    t.cls = cls;
    t.level = level;
    t.iter = iter;
    t.outer = outer;
    t.a = h->pool[h->pool_used++];
    t.b = h->pool[h->pool_used++];
    (void)hipEventRecord(t.a, h->stream);
    h->timed.push_back(t);
    idx = (int)h->timed.size() - 1;
}

// Pinned host memory of at least bytes for the handle's published records (grown on demand).
int ensure_pinned(excmg_handle *h, size_t bytes) {
  if (h->pin_bytes >= bytes) return EXCMG_OK;
  if (h->pin_host) {
    HIPCHECK(hipStreamSynchronize(h->stream));
    (void)hipHostFree(h->pin_host);
    h->pin_host = h->pin_dev = nullptr;
    h->pin_bytes = 0;
  }
  bytes = (bytes + 4095) & ~(size_t)4095;
  HIPCHECK(hipHostMalloc(&h->pin_host, bytes, hipHostMallocMapped | hipHostMallocCoherent));
  HIPCHECK(hipHostGetDevicePointer(&h->pin_dev, h->pin_host, 0));
  h->pin_bytes = bytes;
  return EXCMG_OK;
}

// Copy `bytes` of a device record to the host: a one-workgroup kernel writes it into the pinned buffer, then the host
// waits for the stream and reads it there.
int read_record(excmg_handle *h, void *dst, const void *src, size_t bytes) {
  if (h->noalloc) {
    HIPCHECK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, h->stream));
    HIPCHECK(hipStreamSynchronize(h->stream));
    return EXCMG_OK;
  }
  int e = ensure_pinned(h, bytes);
  if (e) return e;
  launch_publish(src, h->pin_dev, bytes, h->stream);
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(h->stream));
  memcpy(dst, h->pin_host, bytes);
  return EXCMG_OK;
}

int read_state(excmg_handle *h, CgState *dst, const CgState *src) {
  return read_record(h, dst, src, offsetof(CgState, hist));
}

int read_hist(excmg_handle *h, CgState *dst, const CgState *src) { return read_record(h, dst, src, sizeof(CgState)); }

// Per-level iteration counts of CG-class timed launches, to drop launches made after convergence.
struct LevelIters {
  int iters[EXCMG_MAX_LEVELS];
  std::vector<int> inner[EXCMG_MAX_LEVELS];  // FP32_IR: inner iterations of each outer step
};

// Iterations launched before the first look at the CG state, and at most per look: in a single solve (launched as
// graphs of kGraphSizes iterations), and in each round of a batched solve.
constexpr int kSolveFirst = 8, kSolveMax = 32;
constexpr int kBatch = 4, kBatchMax = 16;
constexpr int kGraphSizes[3] = {8, 16, 32};

// CG iterations to launch before the next look at the state: from the residual decay since the start (rho0 -> rho over
// `done` iterations), the geometric rate predicts how many remain; a few more are launched than predicted, since
// iterations launched after convergence cost a near-empty launch each while a look costs a round trip.  first: the
// count without a rate yet; cap: the most.
int next_batch(double rho, double rho0, int done, double stop2, int first, int cap) {
  if (done <= 0 || !(rho > 0.0) || !(rho0 > rho) || !(stop2 > 0.0)) return first;
  if (rho <= stop2) return 1;
  const double rate = log(rho / rho0) / done;  // < 0
  const double need = log(stop2 / rho) / rate;
  int n = (int)ceil(1.15 * need) + 1;
  if (n < 2) n = 2;
  if (n > cap) n = cap;
  return n;
}

// Grids smaller than this relax in FP64 under EXCMG_FP32_IR as well: their sweeps are launch- and latency-bound, so
// halving their bytes saves nothing, while the extra outer steps of the refinement would cost launches.
constexpr long long kIrMinUnknowns = 1LL << 20;

// Grids with at most kSmallCg interior unknowns (16^3 cells and below) relax in one single-workgroup launch, and so
// are the direct solves that fit the sine transforms; every other grid runs the multi-workgroup CG sweeps (a direct
// solve then iterates to the relative residual kDsolveTol).
bool swept(const Layout &lo, int l) {
  const Level &lv = lo.lev[l];
  if (lv.g.interior() <= kSmallCg) return false;
  return l >= 2 || !dst_fits(lv.g);
}

bool self_finalizing(const Level &lv, bool fp32) {
  const int m = selfred_max_blocks();
  const Sweep &a = fp32 ? lv.swA32 : lv.swA, &b = fp32 ? lv.swB32 : lv.swB;
  return sweep_blocks(a) <= m && sweep_blocks(b) <= m && sweep_blocks(lv.sw) <= m;
}

// The single-reduction CG (launch_cg1_*) on grid l: FP64 self-finalizing grids of at most kCg1MaxUnknowns from the
// third to the one below the finest (the direct solves keep the two-pass form), unless EXCMG_TWO_PASS_CG.  Its vectors: u; p in p1's buffer;
// two sets of (r, w, s), one after the other in r's buffer (set 0, where the residual sweep leaves r) and in p0's
// (set 1), which the iterations read and write alternately (each buffer holds the finest grid, three times a grid
// below it).  Its partial sums: the iterations' alternately in the two halves of the partials buffer, the residual
// sweep's in the second quarter, the init sweep's in the second half.
constexpr long long kCg1Align = 32;  // doubles (256 bytes)
// Grids up to this many unknowns, where an iteration's two launches cost more than their bytes: 512^3 step, grids
// 32^3 / 64^3 / 128^3 / 256^3 0.476 / 0.585 / 1.06 / 1.72 ms in the two-pass form, 0.374 / 0.540 / 1.115 / 2.91 ms in
// this one (which moves 80 bytes per unknown and iteration against 64, plus the sweep w = M r at the start)
constexpr long long kCg1MaxUnknowns = 1LL << 18;
long long cg1_stride(const Level &lv) { return (lv.g.elems + kCg1Align - 1) / kCg1Align * kCg1Align; }
Sweep cg1_sweep(const Level &lv) { return lv.swB; }
// everything use_cg1 asks of grid l but that its passes finalize themselves with the sweep of at most 1/4 of the
// partials buffer's half
bool cg1_eligible(const excmg_handle *h, int l) {
  const Layout &lo = h->lo;
  const Level &lv = lo.lev[l];
  if ((h->p.flags & EXCMG_TWO_PASS_CG) || l < 2 || l >= lo.L - 1 || lv.g.interior() > kCg1MaxUnknowns) return false;
  return 4LL * sweep_blocks(lv.sw) <= lo.npart && 2 * cg1_stride(lv) + lv.g.elems <= lo.gfin.elems;
}
bool use_cg1(const excmg_handle *h, int l) {
  const Level &lv = h->lo.lev[l];
  return cg1_eligible(h, l) && self_finalizing(lv, false) && 4LL * sweep_blocks(cg1_sweep(lv)) <= h->lo.npart;
}
double *cg1_resid_parts(const excmg_handle *h) { return h->partials + h->lo.npart / 2; }
// vector j (0 r, 1 w, 2 s) of set q
double *cg1_vec(excmg_handle *h, const Level &lv, int q, int j) { return (q ? h->p0 : h->r) + j * cg1_stride(lv); }

// Iteration `launched` of the single-reduction CG on grid l (par: its parity): reads set par, writes set 1 - par
void launch_cg1_step(excmg_handle *h, int l, hipStream_t s, int par) {
  Level &lv = h->lo.lev[l];
  double *pa = h->partials, *pb = h->partials + h->lo.npart;
  launch_cg1_iteration(cg1_sweep(lv), lv.u, h->p1, cg1_vec(h, lv, par, 0), cg1_vec(h, lv, par, 1),
                       cg1_vec(h, lv, par, 2), cg1_vec(h, lv, 1 - par, 0), cg1_vec(h, lv, 1 - par, 1),
                       cg1_vec(h, lv, 1 - par, 2), h->cs, par, par ? pa : pb, cg1_resid_parts(h),
                       sweep_blocks(lv.sw), grid_tol(h->p, l, h->lo.L), par ? pb : pa, s);
}

// One CG iteration of grid l on stream s: FP64 (fp32 = 0) on u, r, p, or the FP32 inner solve (fp32 = 1) on d32, r32,
// p32.  first: the first FP64 iteration of a self-finalizing grid, whose pass A sums the residual sweep's partials.
// launched: iteration index for the kernel timing.
void launch_iteration(excmg_handle *h, int l, int fp32, bool first, hipStream_t s, int launched, int outer) {
  Level &lv = h->lo.lev[l];
  const double tol = grid_tol(h->p, l, h->lo.L);
  double *pa = h->partials, *pb = h->partials + h->lo.npart;
  if (fp32) {
    if (self_finalizing(lv, true)) {
      {
        Tick t(h, EXCMG_K_CG_A32, l, launched, outer);
        launch_selfred_a<float>(lv.swA32, h->r32, h->p32a, h->p32b, h->cs2, pb, sweep_blocks(lv.swB32), tol,
                                pa, s);
      }
      Tick t(h, EXCMG_K_CG_B32, l, launched, outer);
      launch_selfred_b<float>(lv.swB32, h->d32, h->r32, h->p32a, h->p32b, h->cs2, pa, sweep_blocks(lv.swA32), pb, s);
    } else {
      {
        Tick t(h, EXCMG_K_CG_A32, l, launched, outer);
        launch_cg_pass_a<float>(lv.swA32, h->r32, h->p32a, h->p32b, h->cs2, h->partials, s);
      }
      Tick t(h, EXCMG_K_CG_B32, l, launched, outer);
      launch_cg_pass_b<float>(lv.swB32, h->d32, h->r32, h->p32a, h->p32b, h->cs2, h->partials, s);
    }
    return;
  }
  if (use_cg1(h, l)) {  // (never the finest grid: no kernel timing)
    launch_cg1_step(h, l, s, launched & 1);
    return;
  }
  if (self_finalizing(lv, false)) {
    {
      Tick t(h, EXCMG_K_CG_A, l, launched);
      launch_selfred_a<double>(lv.swA, h->r, h->p0, h->p1, h->cs, pb,
                               first ? sweep_blocks(lv.sw) : sweep_blocks(lv.swB), tol, pa, s);
    }
    Tick t(h, EXCMG_K_CG_B, l, launched);
    launch_selfred_b<double>(lv.swB, lv.u, h->r, h->p0, h->p1, h->cs, pa, sweep_blocks(lv.swA), pb, s);
  } else {
    // the first iteration (launched 0; launches past it always follow it) in its own tuned shapes: each pass's
    // finalize kernel sums as many partials as that launch wrote
    const bool it0 = launched == 0;
    {
      Tick t(h, EXCMG_K_CG_A, l, launched);
      launch_cg_pass_a<double>(it0 ? lv.swA0 : lv.swA, h->r, h->p0, h->p1, h->cs, h->partials, s);
    }
    Tick t(h, EXCMG_K_CG_B, l, launched);
    launch_cg_pass_b<double>(it0 ? lv.swB0 : lv.swB, lv.u, h->r, h->p0, h->p1, h->cs, h->partials, s);
  }
}

// Graphs replace the iteration launches on every grid but the finest (where launches are long and may be timed),
// unless EXCMG_NO_GRAPHS is set.
bool use_graphs(const excmg_handle *h, int l) {
  return !h->noalloc && !(h->p.flags & EXCMG_NO_GRAPHS) && l < h->lo.L - 1;
}

// kGraphSizes[si] CG iterations of grid l (not the first of a self-finalizing FP64 solve) as one graph launch on the
// handle's stream.  The graph holds kernel launches only; it is captured on first use and kept until the sweeps change.
int launch_iteration_graph(excmg_handle *h, int l, int fp32, int si) {
  hipGraphExec_t &ex = h->gexec[l][fp32][si];
  if (!ex) {
    hipGraph_t g = nullptr;
    HIPCHECK(hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal));
    // (the single-reduction CG: graphs start at odd iterations, after the first one's direct launch)
    const bool cg1 = !fp32 && use_cg1(h, l);
    for (int q = 0; q < kGraphSizes[si]; ++q) {
      if (cg1) launch_cg1_step(h, l, h->cap, (1 + q) & 1);
      else launch_iteration(h, l, fp32, false, h->cap, -1, -1);
    }
    const hipError_t ec = hipStreamEndCapture(h->cap, &g);
    if (ec != hipSuccess) return EXCMG_ERR_HIP;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) {
      ex = nullptr;
      return EXCMG_ERR_HIP;
    }
  }
  HIPCHECK(hipGraphLaunch(ex, h->stream));
  return EXCMG_OK;
}

// Launch nb iterations (where graphs are used: rounded up to a multiple of 8, which leaves the prediction of
// next_batch some slack against another look, and launched as the fewest graphs of 32, 16 and 8 iterations); returns
// the new launched count.
int launch_iterations(excmg_handle *h, int l, int fp32, int nb, int launched, int outer, int *err) {
  *err = EXCMG_OK;
  const bool selfred64 = !fp32 && self_finalizing(h->lo.lev[l], false);
  if (!use_graphs(h, l)) {
    for (int q = 0; q < nb; ++q, ++launched)
      launch_iteration(h, l, fp32, selfred64 && launched == 0, h->stream, launched, outer);
    return launched;
  }
  int q = 0;
  if (selfred64 && launched == 0) {
    launch_iteration(h, l, fp32, true, h->stream, launched, outer);
    ++q;
    ++launched;
  }
  int rem = nb > q ? (nb - q + 7) / 8 * 8 : 0;
  for (int si = 2; si >= 0; --si) {
    while (rem >= kGraphSizes[si]) {
      *err = launch_iteration_graph(h, l, fp32, si);
      if (*err) return launched;
      rem -= kGraphSizes[si];
      launched += kGraphSizes[si];
    }
  }
  return launched;
}

// CG iterations allowed on grid l (the direct solves: their own cap, from the grid's size)
int grid_cap(const excmg_handle *h, int l) {
  if (l <= 1) return dsolve_cap(h->lo.lev[l].g.interior());
  return h->p.max_iters > 0 ? h->p.max_iters : 10000;
}

// FP64 CG on level l from the current u (Algorithm 1, the while loop; one iteration per pass; on grids 0 and 1 the
// direct solve, to the relative residual kDsolveTol).

int cg64(excmg_handle *h, int l, const RhsSrc &rs, bool finest, int *iters, double *relres, excmg_stats *st) {
  Level &lv = h->lo.lev[l];
  const hipStream_t s = h->stream;
  const int hist_on = (finest && st && (h->p.flags & EXCMG_WANT_HISTORY)) ? 1 : 0;
  const int maxit = grid_cap(h, l);
  const bool selfred = self_finalizing(lv, false);
  double *partsB = h->partials + h->lo.npart;
  {
    Tick t(h, EXCMG_K_RESID, l);
    if (use_cg1(h, l)) {  // r, then w = M r with the partials of the first iteration's two inner products
      launch_residual_partials(lv.sw, lv.u, rs, h->r, cg1_resid_parts(h), s);
      launch_selfred_init(h->cs, maxit, hist_on, 0, s);
      launch_cg1_init(cg1_sweep(lv), cg1_vec(h, lv, 0, 0), cg1_vec(h, lv, 0, 1), partsB, s);
    } else if (selfred) {
      launch_residual_partials(lv.sw, lv.u, rs, h->r, partsB, s);
      launch_selfred_init(h->cs, maxit, hist_on, 0, s);
    } else {
      launch_residual(lv.sw, lv.u, rs, h->r, h->cs, h->partials, grid_tol(h->p, l, h->lo.L), maxit, hist_on, s);
    }
  }
  int e = last_error();
  if (e) return e;
  CgState hs;
  int launched = 0;
  for (int nb = kSolveFirst;;) {
    launched = launch_iterations(h, l, 0, nb, launched, -1, &e);
    if (e) return e;
    e = last_error();
    if (e) return e;
    e = read_state(h, &hs, h->cs);
    if (e) return e;
    if (hs.done) break;
    nb = next_batch(hs.rho, hs.rho0, hs.iter, hs.stop2, kSolveFirst, kSolveMax);
  }
  *iters = hs.iter;
  *relres = hs.bnorm2 > 0.0 ? sqrt(hs.rho / hs.bnorm2) : 0.0;
  if (!isfinite(hs.bnorm2)) return EXCMG_ERR_NONFINITE;
  if (hist_on) {
    CgState full;
    e = read_hist(h, &full, h->cs);
    if (e) return e;
    const int n = hs.iter + 1 < EXCMG_MAX_HISTORY ? hs.iter + 1 : EXCMG_MAX_HISTORY;
    st->history_len = n;
    for (int q = 0; q < n; ++q) st->history[q] = full.hist[q];
  }
  return hs.status;
}

// FP32 CG sweeps inside FP64 iterative refinement on level l.
int cg_ir(excmg_handle *h, int l, const RhsSrc &rs, bool finest, int *iters, int *outer_out, double *relres,
          excmg_stats *st, std::vector<int> *inner_counts) {
  Level &lv = h->lo.lev[l];
  const hipStream_t s = h->stream;
  const double eta = h->p.inner_tol > 0.0 ? h->p.inner_tol : 1e-5;
  const double tol = level_tol(h->p, l, h->lo.L);
  const int maxit = h->p.max_iters > 0 ? h->p.max_iters : 10000;
  const int max_outer = 30;
  int total = 0;
  CgState ho, hi;
  int status = EXCMG_OK;
  int outer = 0;
  for (;; ++outer) {
    {
      Tick t(h, EXCMG_K_RESID, l);
      launch_residual_cast(lv.sw, lv.u, rs, h->r, lv.g32, h->r32, h->d32, h->cs, h->cs2, h->partials, tol, eta,
                           outer, max_outer, maxit, s);
    }
    int e = last_error();
    if (e) return e;
    e = read_state(h, &ho, h->cs);
    if (e) return e;
    if (ho.done) {
      status = ho.status;
      break;
    }
    int launched = 0;
    for (int nb = kSolveFirst;;) {
      launched = launch_iterations(h, l, 1, nb, launched, outer, &e);
      if (e) return e;
      e = last_error();
      if (e) return e;
      e = read_state(h, &hi, h->cs2);
      if (e) return e;
      if (hi.done) break;
      nb = next_batch(hi.rho, hi.rho0, hi.iter, hi.stop2, kSolveFirst, kSolveMax);
    }
    total += hi.iter;
    if (inner_counts) inner_counts->push_back(hi.iter);
    if (hi.status == EXCMG_ERR_BREAKDOWN) return EXCMG_ERR_BREAKDOWN;
    {
      Tick t(h, EXCMG_K_OTHER, l);
      launch_add_correction(lv.g, lv.u, lv.g32, h->d32, s);
    }
  }
  *iters = total;
  *outer_out = outer;
  *relres = ho.bnorm2 > 0.0 ? sqrt(ho.rho / ho.bnorm2) : 0.0;
  if (!isfinite(ho.bnorm2)) return EXCMG_ERR_NONFINITE;
  if (finest && st && (h->p.flags & EXCMG_WANT_HISTORY)) st->history_len = 0;
  return status;
}

// Single-workgroup CG on a small grid: exact = 1 is DSOLVE (grids 0 and 1), exact = 0 the relaxation of a grid with
// at most kSmallCg unknowns.
// The outcome of a one-launch solve of grid l from its CG state hs: iterations and relative residual into the stats,
// and its status.
int small_cg_outcome(const CgState &hs, int l, bool exact, int *iters, double *relres, excmg_stats *st) {
  if (exact && st && l < 2) st->dsolve_iters[l] = hs.iter;
  *iters = exact ? 0 : hs.iter;
  *relres = hs.bnorm2 > 0.0 ? sqrt(hs.rho / hs.bnorm2) : 0.0;
  if (!isfinite(hs.bnorm2)) return EXCMG_ERR_NONFINITE;
  return hs.status;
}

// defer: nothing on the host waits for this grid's outcome (it is not the finest): its state is copied on the device
// to the grid's slot of defer_dev, which the cascade reads once at its end, so the stream runs on to the next grid
// without a round trip to the host.
int small_cg(excmg_handle *h, int l, const RhsSrc &rs, bool exact, bool finest, int *iters, double *relres,
             excmg_stats *st, bool defer = false) {
  Level &lv = h->lo.lev[l];
  const int hist_on = (!exact && finest && st && (h->p.flags & EXCMG_WANT_HISTORY)) ? 1 : 0;
  const int maxit = grid_cap(h, l);
  {
    Tick t(h, EXCMG_K_DSOLVE, l);
    launch_small_cg(lv.g, lv.u, rs, lv.g, h->r, h->p0, h->p1, lv.st, h->cs, grid_tol(h->p, l, h->lo.L), maxit,
                    exact ? 1 : 0, hist_on, h->stream);
  }
  int e = last_error();
  if (e) return e;
  if (defer && !hist_on) {
    launch_publish(h->cs, h->defer_dev + (size_t)l * kStateHead, kStateHead, h->stream);
    *iters = 0;
    *relres = 0.0;
    return last_error();
  }
  CgState hs;
  e = hist_on ? read_hist(h, &hs, h->cs) : read_state(h, &hs, h->cs);
  if (e) return e;
  if (exact && st && l < 2) st->dsolve_iters[l] = hs.iter;
  *iters = exact ? 0 : hs.iter;
  *relres = hs.bnorm2 > 0.0 ? sqrt(hs.rho / hs.bnorm2) : 0.0;
  if (hist_on) {
    const int n = hs.iter + 1 < EXCMG_MAX_HISTORY ? hs.iter + 1 : EXCMG_MAX_HISTORY;
    st->history_len = n;
    for (int q = 0; q < n; ++q) st->history[q] = hs.hist[q];
  }
  if (!isfinite(hs.bnorm2)) return EXCMG_ERR_NONFINITE;
  return hs.status;
}

// Kernel timing on or off; the event pool is created the first time it is turned on.
int set_timing(excmg_handle *h, bool on) {
  if (on && h->pool.empty()) {
    h->pool.assign(8192, nullptr);
    for (auto &ev : h->pool)
      if (hipEventCreateWithFlags(&ev, kTimingEvent) != hipSuccess) return EXCMG_ERR_HIP;
  }
  h->timing = on;
  if (on) h->p.flags |= EXCMG_WANT_TIMING;
  else h->p.flags &= ~EXCMG_WANT_TIMING;
  return EXCMG_OK;
}

void reset_timing(excmg_handle *h) {
  h->timed.clear();
  h->pool_used = 0;
}

// Sum the timed launches into the stats, dropping CG launches made after their level converged.
int collect_timing(excmg_handle *h, excmg_stats *st, const LevelIters &li) {
  if (!h->timing || !st) return EXCMG_OK;
  HIPCHECK(hipStreamSynchronize(h->stream));
  const int Lf = h->lo.L - 1;
  for (const TimedLaunch &t : h->timed) {
    if (t.iter >= 0) {
      int limit;
      if (t.outer >= 0) {
        const std::vector<int> &v = li.inner[t.level];
        limit = (t.outer < (int)v.size()) ? v[t.outer] : 0;
      } else {
        limit = li.iters[t.level];
      }
      if (t.iter >= limit) continue;
    }
    float ms = 0.0f;
    HIPCHECK(hipEventElapsedTime(&ms, t.a, t.b));
    // the first iteration (p = r) moves fewer bytes than the others: its own classes
    int cls = t.cls;
    if (t.iter == 0 && t.outer < 0 && cls == EXCMG_K_CG_A) cls = EXCMG_K_CG_A0;
    if (t.iter == 0 && t.outer < 0 && cls == EXCMG_K_CG_B) cls = EXCMG_K_CG_B0;
    st->kernel_ms[cls] += ms;
    st->kernel_calls[cls] += 1;
    if (t.level == Lf) {
      st->kernel_ms_finest[cls] += ms;
      st->kernel_calls_finest[cls] += 1;
    }
  }
  return EXCMG_OK;
}

void bind_workspace(excmg_handle *h) {
  char *w = h->ws;
  Layout &lo = h->lo;
  for (int l = 0; l < lo.L; ++l) lo.lev[l].u = (double *)(w + lo.off_u[l]);
  h->r = (double *)(w + lo.off_r);
  h->p0 = (double *)(w + lo.off_p0);
  h->p1 = (double *)(w + lo.off_p1);
  if (h->p.precision == EXCMG_FP32_IR) {
    h->r32 = (float *)(w + lo.off_r32);
    h->p32a = (float *)(w + lo.off_p32a);
    h->p32b = (float *)(w + lo.off_p32b);
    h->d32 = (float *)(w + lo.off_d32);
  } else {
    h->r32 = h->p32a = h->p32b = h->d32 = nullptr;
  }
  h->partials = (double *)(w + lo.off_part);
  h->cs = (CgState *)(w + lo.off_cs);
  h->cs2 = (CgState *)(w + lo.off_cs2);
  h->defer_dev = w + lo.off_defer;
  for (int d = 0; d < 3; ++d) h->inv_m[d] = (double *)(w + lo.off_invm[d]);
  h->flag = (int *)(w + lo.off_flag);
}

// The cascade shared by the solve and the adjoint.  mode 0: level data from (f, g); mode 1: from G, zero boundary.
int cascade(excmg_handle *h, int mode, const double *f, const double *g, excmg_stats *st, LevelIters *li) {
  Layout &lo = h->lo;
  const int L = lo.L;
  const hipStream_t s = h->stream;
  int final_status = EXCMG_OK;
  bool deferred[EXCMG_MAX_LEVELS] = {};  // grids solved in one launch whose outcome is read after the loop
  // The outcomes of the deferred solves of the grids below `upto`, in one read: their stats, NOCONV into
  // final_status, and the first other error (as it would have ended the cascade at that grid).
  auto resolve = [&](int upto) -> int {
    int nd = 0;
    for (int l = 0; l < upto; ++l) nd = deferred[l] ? l + 1 : nd;
    if (nd == 0) return EXCMG_OK;
    std::vector<char> buf((size_t)nd * kStateHead);
    int e = read_record(h, buf.data(), h->defer_dev, buf.size());
    if (e) return e;
    for (int l = 0; l < nd; ++l) {
      if (!deferred[l]) continue;
      CgState hs;
      memcpy(&hs, buf.data() + (size_t)l * kStateHead, kStateHead);
      const bool exact = l <= 1;
      int it = 0;
      double rr = 0.0;
      e = small_cg_outcome(hs, l, exact, &it, &rr, st);
      if (e == EXCMG_ERR_NOCONV)
        final_status = EXCMG_ERR_NOCONV;
      else if (e)
        return e;
      if (li) li->iters[l] = exact ? 0 : it;
      if (st) {
        st->iters[l] = it;
        st->relres[l] = rr;
      }
    }
    return EXCMG_OK;
  };
  for (int l = 0; l < L; ++l) {
    Level &lv = lo.lev[l];
    if (h->lev_ev[l]) HIPCHECK(hipEventRecord(h->lev_ev[l], s));
    RhsSrc rs;
    rs.gf = lo.gdense;
    rs.f = f;
    rs.g = g;
    rs.s = lv.stride;
    rs.mode = mode;
    rs.a = 1.0 / (lv.h[0] * lv.h[0]);
    rs.b = 1.0 / (lv.h[1] * lv.h[1]);
    rs.c = 1.0 / (lv.h[2] * lv.h[2]);
    // the stopping test's norm on this grid: (R f, g) under EXCMG_STOP_F_G, and under EXCMG_STOP_F_G_BELOW_FINEST
    // on every grid but the finest; else b (and always b for the adjoint)
    const bool fg_here = (h->p.flags & EXCMG_STOP_F_G) || ((h->p.flags & EXCMG_STOP_F_G_BELOW_FINEST) && l < L - 1);
    rs.fg = (mode == 0 && fg_here) ? 1 : 0;
    if (h->p.flags & (EXCMG_STOP_F_G | EXCMG_STOP_F_G_BELOW_FINEST)) {
      // the boundary half of the stopping test's norm for this grid (0 for the adjoint, whose test stays on ||b||)
      Tick t(h, EXCMG_K_OTHER, l);
      launch_boundary_g2(rs, lv.g, h->cs, s);
    }
    int e = EXCMG_OK;
    int it = 0, outer = 0, dit = 0;
    double rr = 0.0;
    if (l <= 1) {
      {
        Tick t(h, EXCMG_K_OTHER, l);
        launch_set_boundary(lo.gdense, mode == 0 ? g : nullptr, lv.stride, lv.g, lv.u, 1, s);
      }
      // DSOLVE: the sine-transform solve or single-workgroup CG, or on larger grids the CG sweeps from u = 0
      if (swept(lo, l)) {
        e = cg64(h, l, rs, l == L - 1, &dit, &rr, st);
        if (st) st->dsolve_iters[l] = dit;
      } else {
        deferred[l] = l < L - 1;
        e = small_cg(h, l, rs, true, l == L - 1, &it, &rr, st, deferred[l]);
      }
      if (e == EXCMG_ERR_NOCONV) {
        final_status = EXCMG_ERR_NOCONV;
      } else if (e) {
        const int d = resolve(l);  // an error of an earlier grid comes first
        return d ? d : e;
      }
    } else {
      {
        Tick t(h, EXCMG_K_EXP_FINITE, l);
        launch_initial_guess(guess_kind(h->p.flags), lo.lev[l - 1].g, lo.lev[l - 1].u, lo.lev[l - 2].g,
                             lo.lev[l - 2].u, lo.gdense, mode == 0 ? g : nullptr, lv.stride, lv.g, lv.u, s);
      }
      e = last_error();
      if (e) return e;
      if (!swept(lo, l)) {
        deferred[l] = l < L - 1;
        e = small_cg(h, l, rs, false, l == L - 1, &it, &rr, st, deferred[l]);
      }
      else if (h->p.precision == EXCMG_FP64 || lv.g.interior() < kIrMinUnknowns)
        e = cg64(h, l, rs, l == L - 1, &it, &rr, st);
      else
        e = cg_ir(h, l, rs, l == L - 1, &it, &outer, &rr, st, li ? &li->inner[l] : nullptr);
      if (e == EXCMG_ERR_NOCONV) {
        final_status = EXCMG_ERR_NOCONV;
      } else if (e) {
        const int d = resolve(l);  // an error of an earlier grid comes first
        return d ? d : e;
      }
    }
    if (li) li->iters[l] = l <= 1 ? dit : it;
    if (st) {
      st->iters[l] = it;
      st->ir_outer[l] = outer;
      st->relres[l] = rr;
    }
  }
  if (h->lev_ev[L]) HIPCHECK(hipEventRecord(h->lev_ev[L], s));
  const int e = resolve(L);
  return e ? e : final_status;
}

void fill_level_stats(excmg_handle *h, excmg_stats *st) {
  if (!st) return;
  const bool ev = h->lev_ev[h->lo.L] != nullptr;
  if (ev) (void)hipEventSynchronize(h->lev_ev[h->lo.L]);
  st->levels = h->lo.L;
  for (int l = 0; l < h->lo.L; ++l) {
    for (int d = 0; d < 3; ++d) st->n[l][d] = h->lo.lev[l].n[d];
    float ms = 0.0f;
    if (ev && hipEventElapsedTime(&ms, h->lev_ev[l], h->lev_ev[l + 1]) == hipSuccess) st->ms_level[l] = ms;
  }
}

void clear_stats(excmg_stats *st) {
  if (st) memset(st, 0, sizeof(*st));
}

// ------------------------------------------------------------------------------------------------ batched solve
//
// Every problem of a batch walks its own cascade; the host keeps each problem's grid and phase and, in rounds, issues
// one launch per kind of work for all problems that need it (flattened workgroup ranges, or one workgroup per
// problem), whatever grid each is on: grid starts (boundary values, or EXP_finite), direct and small-grid solves,
// residuals, refinement corrections, then a batch of CG iterations for every problem that is iterating.  After each
// round one look at the problems' status words (pinned host memory) moves them on.  Fast problems thus reach their
// finest grids while slow ones are still relaxing coarse ones, and a problem that has converged takes no workgroups.
//
// Per (problem, grid) the device tables hold an entry (layouts, arrays in the problem's own workspace, level data,
// tolerances), built on the host and uploaded once; each round uploads only the launch lists (entry pointers and
// workgroup prefixes).

enum BatchListKind { kListSetB, kListExp, kListSmall, kListBterm, kListR64, kListRC, kListCorr, kListI64, kListI32,
                     kListCopy, kListKinds };

size_t batch_table_bytes(int count) { return align256(sizeof(BatchEntry) * (size_t)count); }

size_t batch_list_bytes(int count) {
  return align256(sizeof(void *) * (size_t)count + sizeof(int) * (2 * (size_t)(count + 1) + (size_t)count));
}

size_t batch_ws_bytes(int count) {
  return align256(sizeof(BatchStatus) * (size_t)count) + 256 + (size_t)EXCMG_MAX_LEVELS * batch_table_bytes(count) +
         (size_t)kListKinds * batch_list_bytes(count);
}

int batch_kind(const excmg_handle *h, int l) {
  if (l >= h->lo.L) return kBNone;
  const Level &lv = h->lo.lev[l];
  if (!swept(h->lo, l)) return kBSmall;
  if (l <= 1 || h->p.precision == EXCMG_FP64 || lv.g.interior() < kIrMinUnknowns) return kBCg64;
  return kBIr;
}

void batch_entry(excmg_handle *h, int problem, int l, const double *f, const double *g, double *u, BatchEntry *E,
                 int blocks[kLaunchKinds], const int bty[2]) {
  memset(E, 0, sizeof(*E));
  for (int k = 0; k < kLaunchKinds; ++k) blocks[k] = 0;
  E->kind = batch_kind(h, l);
  E->problem = problem;
  if (E->kind == kBNone) return;
  const Layout &lo = h->lo;
  const Level &lv = lo.lev[l];
  E->finest = (l == lo.L - 1);
  E->exact = (l <= 1);
  E->level = l;
  E->cap = grid_cap(h, l);
  E->max_outer = 30;
  E->tol = grid_tol(h->p, l, h->lo.L);
  E->eta = h->p.inner_tol > 0.0 ? h->p.inner_tol : 1e-5;
  // every entry of a batched launch has the launch's tile height (bty: the batch's, for the FP64 and the FP32
  // passes); a grid tuned alone to another keeps its z chunk here
  E->swA = with_height(lv.swA, bty[0]);
  E->swB = with_height(lv.swB, bty[0]);
  E->swR = default_height(lv.sw);
  E->swA32 = with_height(lv.swA32, bty[1]);
  E->swB32 = with_height(lv.swB32, bty[1]);
  E->g = lv.g;
  E->g32 = lv.g32;
  E->gd = lo.gdense;
  if (l >= 1) E->g2 = lo.lev[l - 1].g;
  if (l >= 2) E->g4 = lo.lev[l - 2].g;
  E->st = lv.st;
  E->rs.gf = lo.gdense;
  E->rs.f = f;
  E->rs.g = g;
  E->rs.s = lv.stride;
  E->rs.mode = 0;
  E->rs.fg = 0;
  E->rs.a = 1.0 / (lv.h[0] * lv.h[0]);
  E->rs.b = 1.0 / (lv.h[1] * lv.h[1]);
  E->rs.c = 1.0 / (lv.h[2] * lv.h[2]);
  E->u = lv.u;
  E->r = h->r;
  E->p0 = h->p0;
  E->p1 = h->p1;
  E->r32 = h->r32;
  E->p32a = h->p32a;
  E->p32b = h->p32b;
  E->d32 = h->d32;
  E->cs = h->cs;
  E->cs2 = h->cs2;
  E->parts = h->partials;
  E->u2 = l >= 1 ? lo.lev[l - 1].u : nullptr;
  E->u4 = l >= 2 ? lo.lev[l - 2].u : nullptr;
  E->gb = g;
  E->out = u;
  if (E->kind == kBCg64) {
    blocks[kLA64] = sweep_blocks(E->swA);
    blocks[kLB64] = sweep_blocks(E->swB);
    blocks[kLR64] = sweep_blocks(E->swR);
  }
  if (E->kind == kBIr) {
    blocks[kLA32] = sweep_blocks(E->swA32);
    blocks[kLB32] = sweep_blocks(E->swB32);
    blocks[kLRC] = sweep_blocks(E->swR);
    blocks[kLCorr] = b_blocks_interior(lv.g);
  }
  if (E->kind == kBCg64 || E->kind == kBIr) blocks[kLBterm] = b_blocks_bterms(lv.g);
  if (l >= 2) blocks[kLExp] = b_blocks_exp_finite(lv.g);
  if (l <= 1) blocks[kLSetB] = b_blocks_nodes(lv.g);
  if (E->finest) blocks[kLCopy] = b_blocks_nodes(lv.g);
}

// a problem's place in its cascade
enum BatchPhase { kPhStart, kPhSmall, kPhIter64, kPhIter32, kPhOuter, kPhCopy, kPhDone };

// A round's CG iterations: it rounds of one iteration of the FP64 entries (the first nb64 rounds) and of the FP32 inner
// solves (the first nb32), in a graph replayed from the first handle's cache when the round has the launch shape of
// an earlier one (the same workspace, iteration counts and, per list, numbers of entries and workgroups; the lists
// themselves are read from the batch workspace when the kernels run), else captured and instantiated; directly
// launched under EXCMG_NO_GRAPHS or for a single iteration.
constexpr size_t kBatchGraphCache = 1024;

int batch_iterations(excmg_handle *h0, const char *ws, int it, int nb64, int nb32, const BatchList (&l64)[2],
                     const BatchList (&l32)[2], BatchStatus *stat) {
  const hipStream_t s = h0->stream;
  auto launch_all = [&](hipStream_t st) {
    for (int q = 0; q < it; ++q) {
      if (q < nb64) launch_b_iteration(0, h0->bty[0], h0->bdepth[0], l64[0], l64[1], stat, st);
      if (q < nb32) launch_b_iteration(1, h0->bty[1], h0->bdepth[1], l32[0], l32[1], stat, st);
    }
  };
  if (it <= 1 || (h0->p.flags & EXCMG_NO_GRAPHS) || h0->noalloc) {
    launch_all(s);
    return last_error();
  }
  const std::vector<long long> key = {(long long)(uintptr_t)ws, h0->bty[0], h0->bty[1], h0->bdepth[0], h0->bdepth[1],
                                      it, nb64, nb32, l64[0].n, l64[0].total, l64[1].total,
                                      l32[0].n, l32[0].total, l32[1].total};
  const long long now = h0->bgraph_hits + h0->bgraph_misses;
  for (auto &bg : h0->bgraphs)
    if (bg.key == key) {
      ++h0->bgraph_hits;
      bg.used = now;
      HIPCHECK(hipGraphLaunch(bg.ex, s));
      return EXCMG_OK;
    }
  ++h0->bgraph_misses;
  hipGraph_t gr = nullptr;
  HIPCHECK(hipStreamBeginCapture(h0->cap, hipStreamCaptureModeThreadLocal));
  launch_all(h0->cap);
  const hipError_t ec = hipStreamEndCapture(h0->cap, &gr);
  if (ec != hipSuccess) return EXCMG_ERR_HIP;
  hipGraphExec_t ex = nullptr;
  const hipError_t ei = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (ei != hipSuccess) return EXCMG_ERR_HIP;
  if (h0->bgraphs.size() >= kBatchGraphCache) {  // the least recently used goes
    size_t lru = 0;
    for (size_t q = 1; q < h0->bgraphs.size(); ++q)
      if (h0->bgraphs[q].used < h0->bgraphs[lru].used) lru = q;
    (void)hipGraphExecDestroy(h0->bgraphs[lru].ex);
    h0->bgraphs.erase(h0->bgraphs.begin() + (long)lru);
  }
  h0->bgraphs.push_back({key, ex, now});
  HIPCHECK(hipGraphLaunch(ex, s));
  return EXCMG_OK;
}

int batched_solve(excmg_handle *const *hs, int count, const double *const *f, const double *const *g,
                  double *const *u, char *ws, excmg_stats *stats, double *ms_per_problem) {
  const hipStream_t s = hs[0]->stream;
  const auto t_host = std::chrono::steady_clock::now();
  int S = 0;
  for (int b = 0; b < count; ++b) S = hs[b]->lo.L > S ? hs[b]->lo.L : S;
  const size_t stat_bytes = align256(sizeof(BatchStatus) * (size_t)count);
  BatchStatus *stat = (BatchStatus *)ws;
  long long *t0 = (long long *)(ws + stat_bytes);
  char *tables = ws + stat_bytes + 256;
  const size_t tb = batch_table_bytes(count);
  char *lists_dev = tables + (size_t)EXCMG_MAX_LEVELS * tb;
  const size_t lb = batch_list_bytes(count);
  const int n1 = count + 1;

  // the entry of every (grid, problem), and its workgroup counts per launch kind
  std::vector<char> host((size_t)S * tb, 0);
  std::vector<int> blocks((size_t)S * count * kLaunchKinds, 0);
  for (int l = 0; l < S; ++l)
    for (int b = 0; b < count; ++b)
      batch_entry(hs[b], b, l, f[b], g[b], u[b], (BatchEntry *)(host.data() + l * tb) + b,
                  &blocks[((size_t)l * count + b) * kLaunchKinds], hs[0]->bty);
  int e;
  HIPCHECK(hipMemcpyAsync(tables, host.data(), host.size(), hipMemcpyHostToDevice, s));
  HIPCHECK(hipStreamSynchronize(s));  // the host tables may go out of scope on any early return below
  launch_b_init(stat, count, t0, s);
  if ((e = last_error())) return e;
  auto entry = [&](int l, int b) { return (const BatchEntry *)(tables + l * tb) + b; };
  auto nblk = [&](int l, int b, int k) { return blocks[((size_t)l * count + b) * kLaunchKinds + k]; };

  // pinned host memory: the status words, then the launch lists of a round (copied to lists_dev in one piece)
  if ((e = ensure_pinned(hs[0], stat_bytes + (size_t)kListKinds * lb))) return e;
  char *lists_host = (char *)hs[0]->pin_host + stat_bytes;
  std::vector<BatchStatus> hstat(count);
  auto read_stat = [&]() -> int {
    return read_record(hs[0], hstat.data(), stat, sizeof(BatchStatus) * (size_t)count);
  };
  struct HostList {
    const BatchEntry **ent;
    int *preA, *preB, *aux;
    int n;
  };
  HostList hl[kListKinds];
  BatchList dl[kListKinds][2];
  for (int k = 0; k < kListKinds; ++k) {
    char *hb = lists_host + k * lb, *db = lists_dev + k * lb;
    hl[k].ent = (const BatchEntry **)hb;
    hl[k].preA = (int *)(hb + sizeof(void *) * count);
    hl[k].preB = hl[k].preA + n1;
    hl[k].aux = hl[k].preB + n1;
    for (int q = 0; q < 2; ++q) {
      dl[k][q].ent = (const BatchEntry *const *)db;
      dl[k][q].pre = (const int *)(db + sizeof(void *) * count) + q * n1;
      dl[k][q].aux = (const int *)(db + sizeof(void *) * count) + 2 * n1;
    }
  }
  auto add = [&](int k, int l, int b, int wa, int wb, int aux) {
    HostList &L = hl[k];
    L.ent[L.n] = entry(l, b);
    L.preA[L.n + 1] = L.preA[L.n] + wa;
    L.preB[L.n + 1] = L.preB[L.n] + wb;
    L.aux[L.n] = aux;
    ++L.n;
  };

  if (stats)
    for (int b = 0; b < count; ++b) {
      memset(&stats[b], 0, sizeof(excmg_stats));
      stats[b].levels = hs[b]->lo.L;
      for (int l = 0; l < hs[b]->lo.L; ++l)
        for (int d = 0; d < 3; ++d) stats[b].n[l][d] = hs[b]->lo.lev[l].n[d];
    }
  std::vector<int> lev(count, 0), ph(count, kPhStart), outer(count, 0), inner(count, 0), fresh(count, 0);
  int final_status = EXCMG_OK, remaining = count;
  // a problem's grid is finished: record it, then start its next grid (or copy it out)
  auto finish_grid = [&](int b) -> int {
    const int l = lev[b];
    const int kind = batch_kind(hs[b], l);
    const BatchMirror &m = hstat[b].m[0];
    if (!isfinite(m.bnorm2)) return EXCMG_ERR_NONFINITE;
    if (m.status == EXCMG_ERR_BREAKDOWN) return EXCMG_ERR_BREAKDOWN;
    if (m.status == EXCMG_ERR_NOCONV) final_status = EXCMG_ERR_NOCONV;
    if (stats) {
      excmg_stats &o = stats[b];
      o.iters[l] = kind == kBIr ? inner[b] : (l <= 1 ? 0 : m.iter);
      o.ir_outer[l] = kind == kBIr ? m.iter : 0;
      if (l <= 1) o.dsolve_iters[l] = m.iter;
      o.relres[l] = m.bnorm2 > 0.0 ? sqrt(m.rho / m.bnorm2) : 0.0;
    }
    if (l == hs[b]->lo.L - 1) {
      ph[b] = kPhCopy;
    } else {
      lev[b] = l + 1;
      ph[b] = kPhStart;
    }
    return EXCMG_OK;
  };

  int nb64 = kBatch, nb32 = kBatch;
  for (int round = 0; remaining > 0; ++round) {
    if (round > 4 * 1000 * 1000) return EXCMG_ERR_NOCONV;  // every device loop is capped; not reached
    for (int k = 0; k < kListKinds; ++k) {
      hl[k].n = 0;
      hl[k].preA[0] = hl[k].preB[0] = 0;
    }
    int lds = 0;
    for (int b = 0; b < count; ++b) {
      const int l = lev[b];
      fresh[b] = 0;
      switch (ph[b]) {
        case kPhStart: {
          const int kind = batch_kind(hs[b], l);
          if (l <= 1) add(kListSetB, l, b, nblk(l, b, kLSetB), 0, 0);
          else add(kListExp, l, b, nblk(l, b, kLExp), 0, 0);
          if (kind == kBSmall) {
            add(kListSmall, l, b, 0, 0, 0);
            const int v = b_small_lds_nodes(hs[b]->lo.lev[l].g);
            lds = v > lds ? v : lds;
            ph[b] = kPhSmall;
          } else if (kind == kBCg64) {
            add(kListBterm, l, b, nblk(l, b, kLBterm), 0, 0);
            add(kListR64, l, b, nblk(l, b, kLR64), 0, 0);
            add(kListI64, l, b, nblk(l, b, kLA64), nblk(l, b, kLB64), 0);
            ph[b] = kPhIter64;
            fresh[b] = 1;
          } else {
            add(kListBterm, l, b, nblk(l, b, kLBterm), 0, 0);
            outer[b] = 0;
            inner[b] = 0;
            add(kListRC, l, b, nblk(l, b, kLRC), 0, 0);
            add(kListI32, l, b, nblk(l, b, kLA32), nblk(l, b, kLB32), 0);
            ph[b] = kPhIter32;
            fresh[b] = 1;
          }
          break;
        }
        case kPhIter64:
          add(kListI64, l, b, nblk(l, b, kLA64), nblk(l, b, kLB64), 0);
          break;
        case kPhIter32:
          add(kListI32, l, b, nblk(l, b, kLA32), nblk(l, b, kLB32), 0);
          break;
        case kPhOuter:  // the inner solve finished: u += d, then the next outer residual and inner solve
          add(kListCorr, l, b, nblk(l, b, kLCorr), 0, 0);
          add(kListRC, l, b, nblk(l, b, kLRC), 0, outer[b]);
          add(kListI32, l, b, nblk(l, b, kLA32), nblk(l, b, kLB32), 0);
          ph[b] = kPhIter32;
          fresh[b] = 1;
          break;
        case kPhCopy:
          add(kListCopy, l, b, nblk(l, b, kLCopy), 0, 0);
          ph[b] = kPhDone;
          --remaining;
          break;
        default:
          break;
      }
    }
    HIPCHECK(hipMemcpyAsync(lists_dev, lists_host, (size_t)kListKinds * lb, hipMemcpyHostToDevice, s));
    for (int k = 0; k < kListKinds; ++k)
      for (int q = 0; q < 2; ++q) {
        dl[k][q].n = hl[k].n;
        dl[k][q].total = q ? hl[k].preB[hl[k].n] : hl[k].preA[hl[k].n];
      }
    launch_b_copy(dl[kListCopy][0], s);
    launch_b_set_boundary(dl[kListSetB][0], s);
    launch_b_exp_finite(dl[kListExp][0], s);
    launch_b_small_cg(dl[kListSmall][0], lds, stat, s);
    launch_b_boundary_terms(dl[kListBterm][0], s);
    launch_b_residual(dl[kListR64][0], stat, s);
    launch_b_add_correction(dl[kListCorr][0], s);
    launch_b_residual_cast(dl[kListRC][0], stat, s);
    const int it = hl[kListI64].n || hl[kListI32].n ? (nb64 > nb32 ? nb64 : nb32) : 0;
    if ((e = batch_iterations(hs[0], ws, it, nb64, nb32, dl[kListI64], dl[kListI32], stat))) return e;
    if ((e = last_error()) || (e = read_stat())) return e;
    // move every problem on, and size the next round's iteration batches from the residual decay seen so far
    nb64 = nb32 = 1;
    bool any64 = false, any32 = false;
    for (int b = 0; b < count; ++b) {
      switch (ph[b]) {
        case kPhSmall:
          if ((e = finish_grid(b))) return e;
          break;
        case kPhIter64: {
          const BatchMirror &m = hstat[b].m[0];
          if (m.done) {
            if ((e = finish_grid(b))) return e;
          } else {
            const int want = fresh[b] ? kBatch : next_batch(m.rho, m.rho0, m.iter, m.stop2, kBatch, kBatchMax);
            nb64 = want > nb64 ? want : nb64;
            any64 = true;
          }
          break;
        }
        case kPhIter32: {
          const BatchMirror &mo = hstat[b].m[0], &mi = hstat[b].m[1];
          if (mo.done) {  // the outer residual met the tolerance (or the outer steps ran out)
            if ((e = finish_grid(b))) return e;
          } else if (mi.done) {
            inner[b] += mi.iter;
            if (mi.status == EXCMG_ERR_BREAKDOWN) return EXCMG_ERR_BREAKDOWN;
            ++outer[b];
            ph[b] = kPhOuter;
          } else {
            const int want = fresh[b] ? kBatch : next_batch(mi.rho, mi.rho0, mi.iter, mi.stop2, kBatch, kBatchMax);
            nb32 = want > nb32 ? want : nb32;
            any32 = true;
          }
          break;
        }
        default:
          break;
      }
    }
    if (!any64) nb64 = kBatch;
    if (!any32) nb32 = kBatch;
  }
  long long t_start = 0;
  if ((e = read_record(hs[0], &t_start, t0, sizeof(long long)))) return e;
  int rate_khz = 0;
  HIPCHECK(hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, hs[0]->device));
  const double host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_host).count();
  for (int b = 0; b < count; ++b) {
    const double ms = (rate_khz > 0 && hstat[b].t_done > 0) ? (double)(hstat[b].t_done - t_start) / rate_khz : -1.0;
    if (ms_per_problem) ms_per_problem[b] = ms;
    if (stats) stats[b].ms_total = host_ms;
  }
  return final_status;
}

// Autotuner of the batched sweeps.  In a batched launch the workgroups of every problem concerned run together, so the
// z chunk that suits one problem alone (small chunks, to give a small grid enough workgroups to fill the GPU) is not
// the one that suits the batch.  Per grid counted from each problem's finest (t = 0 the finest, 1 the next coarser,
// ...) and per precision, every candidate chunk is timed as one flattened launch of pass A and one of pass B over all
// the problems whose grid t relaxes in that precision (the batched kernels' prefetch depth 2 and streaming policy),
// at each tile height; a batched launch holds every grid of the batch, so the height is one per precision: the one
// whose fastest chunks sum to the least time over the grids.  The chunks and height are kept in those problems'
// sweeps, and the height on every handle of the batch (for the batches it leads).  zc_out[2 t + prec] (nullable):
// the chunk chosen, 0 where no problem relaxes that grid in that precision.
int batched_autotune(excmg_handle *const *hs, int count, char *ws, int32_t *zc_out) {
  const hipStream_t s = hs[0]->stream;
  int S = 0;
  for (int b = 0; b < count; ++b) S = hs[b]->lo.L > S ? hs[b]->lo.L : S;
  static const int cand[] = {2, 4, 8, 16, 32, 64, 128};
  const size_t stat_bytes = align256(sizeof(BatchStatus) * (size_t)count);
  char *table_dev = ws + stat_bytes + 256;
  char *list_dev = table_dev + (size_t)EXCMG_MAX_LEVELS * batch_table_bytes(count);
  const int n1 = count + 1;
  std::vector<BatchEntry> ent(count);
  std::vector<char> list_host(batch_list_bytes(count));
  const BatchEntry **lent = (const BatchEntry **)list_host.data();
  int *preA = (int *)(list_host.data() + sizeof(void *) * (size_t)count), *preB = preA + n1;
  hipEvent_t ea, eb;
  HIPCHECK(hipEventCreateWithFlags(&ea, kTimingEvent));
  HIPCHECK(hipEventCreateWithFlags(&eb, kTimingEvent));
  int rc = EXCMG_OK;
  if (zc_out)
    for (int q = 0; q < 2 * EXCMG_MAX_LEVELS; ++q) zc_out[q] = 0;
  // best chunk per (precision, shape, grid t) and the summed time of those bests per (precision, shape), where a shape
  // is a tile height and a prefetch depth: one launch covers every grid of the batch at once, so the shape is chosen
  // for the batch as a whole
  static const int heights[] = {4, 8, 16};
  static const int bdepths[] = {2, 3, 4, 6};
  constexpr int kD = (int)(sizeof(bdepths) / sizeof(bdepths[0]));
  constexpr int kH = (int)(sizeof(heights) / sizeof(heights[0])) * kD;
  std::vector<int> bzc(2 * kH * (size_t)S, 0);
  float total[2][kH] = {};
  bool used[2] = {false, false};
  for (int t = 0; t < S && rc == EXCMG_OK; ++t) {
    for (int prec = 0; prec < 2 && rc == EXCMG_OK; ++prec) {
      std::vector<int> probs;  // the problems whose grid L-1-t relaxes in this precision
      for (int b = 0; b < count; ++b) {
        const int l = hs[b]->lo.L - 1 - t;
        if (l < 0) continue;
        const int kind = batch_kind(hs[b], l);
        if ((prec == 0 && kind == kBCg64) || (prec == 1 && kind == kBIr)) probs.push_back(b);
      }
      if (probs.empty()) continue;
      used[prec] = true;
      for (int hi = 0; hi < kH && rc == EXCMG_OK; ++hi) {
        const int ty = heights[hi / kD], depth = bdepths[hi % kD];
        const int bty[2] = {ty, ty};
        float best = 1e30f;
        int best_zc = 0;
        for (int zc : cand) {
          const int n = (int)probs.size();
          preA[0] = preB[0] = 0;
          for (int q = 0; q < n; ++q) {
            excmg_handle *h = hs[probs[q]];
            const int l = h->lo.L - 1 - t;
            const Level &lv = h->lo.lev[l];
            int blocks[kLaunchKinds];
            batch_entry(h, probs[q], l, nullptr, nullptr, nullptr, &ent[q], blocks, bty);
            const Sweep sw = make_sweep(prec ? lv.g32 : lv.g, lv.st, zc, depth, 1, ty);
            if (prec) ent[q].swA32 = ent[q].swB32 = sw;
            else ent[q].swA = ent[q].swB = sw;
            lent[q] = (const BatchEntry *)table_dev + q;
            preA[q + 1] = preA[q] + sweep_blocks(sw);
            preB[q + 1] = preB[q] + sweep_blocks(sw);
          }
          if (hipMemcpyAsync(table_dev, ent.data(), sizeof(BatchEntry) * (size_t)n, hipMemcpyHostToDevice, s) !=
                  hipSuccess ||
              hipMemcpyAsync(list_dev, list_host.data(), list_host.size(), hipMemcpyHostToDevice, s) != hipSuccess ||
              hipStreamSynchronize(s) != hipSuccess) {
            rc = EXCMG_ERR_HIP;
            break;
          }
          BatchList A, B;
          A.ent = B.ent = (const BatchEntry *const *)list_dev;
          A.pre = A.aux = (const int *)(list_dev + sizeof(void *) * (size_t)count);
          B.pre = B.aux = A.pre + n1;
          A.n = B.n = n;
          A.total = preA[n];
          B.total = preB[n];
          launch_b_tune_state(A, s);
          float tmin = 1e30f;
          for (int rep = 0; rep < 4 && rc == EXCMG_OK; ++rep) {
            float ms = 0.0f;
            if (hipEventRecord(ea, s) != hipSuccess) rc = EXCMG_ERR_HIP;
            launch_b_passes(prec, ty, depth, A, B, s);
            if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
                hipEventElapsedTime(&ms, ea, eb) != hipSuccess || last_error() != EXCMG_OK)
              rc = EXCMG_ERR_HIP;
            if (rep > 0 && ms < tmin) tmin = ms;  // the first launch warms caches and code
          }
          if (tmin < best) {
            best = tmin;
            best_zc = zc;
          }
        }
        bzc[((size_t)prec * kH + hi) * S + t] = best_zc;
        total[prec][hi] += best;
      }
    }
  }
  if (rc == EXCMG_OK) {
    for (int prec = 0; prec < 2; ++prec) {
      if (!used[prec]) continue;
      int hb = 0;
      for (int hi = 1; hi < kH; ++hi)
        if (total[prec][hi] < total[prec][hb]) hb = hi;
      const int ty = heights[hb / kD], depth = bdepths[hb % kD];
      for (int b = 0; b < count; ++b) {
        hs[b]->bty[prec] = ty;
        hs[b]->bdepth[prec] = depth;
      }
      for (int t = 0; t < S; ++t) {
        const int zc = bzc[((size_t)prec * kH + hb) * S + t];
        if (zc == 0) continue;  // no problem relaxes grid t in this precision
        for (int b = 0; b < count; ++b) {
          const int l = hs[b]->lo.L - 1 - t;
          if (l < 0) continue;
          const int kind = batch_kind(hs[b], l);
          if (!((prec == 0 && kind == kBCg64) || (prec == 1 && kind == kBIr))) continue;
          Level &lv = hs[b]->lo.lev[l];
          const Sweep sw = make_sweep(prec ? lv.g32 : lv.g, lv.st, zc, depth, 1, ty);
          if (prec) lv.swA32 = lv.swB32 = sw;
          else lv.swA = lv.swB = sw;
        }
        if (zc_out) zc_out[2 * t + prec] = zc;
      }
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  for (int b = 0; b < count; ++b) hs[b]->drop_graphs();  // captured with the old sweep shapes
  return rc;
}

}  // namespace

// ------------------------------------------------------------------------------------ the solve without allocation
//
// excmg_solve_noalloc's workspace is this fixed device array of the library: each GPU the library is loaded on holds
// its own copy until the process ends.  Host code never uses the array's name as an address: the device address is
// looked up once per device (hipGetSymbolAddress, with that device current) and kept.  Every call on one GPU uses
// the same array, so calls that overlap on one GPU race; each call clears what it needs cleared.
constexpr size_t kScratchBytes = EXCMG_NOALLOC_MAX_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

int solve_on(excmg_handle *h, const double *f, const double *g, double *u, double *u_ext, excmg_stats *st);

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices];

int scratch_address(int dev, void **out) {
  if (dev < 0 || dev >= kMaxDevices) return EXCMG_ERR_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return EXCMG_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return EXCMG_OK;
}

}  // namespace

// ---------------------------------------------------------------------------------------------------------- C ABI

extern "C" {

int excmg_plan(const excmg_problem *p, int32_t *levels, int32_t n_coarse_out[3]) {
  if (!p || !levels || !n_coarse_out) return EXCMG_ERR_ARG;
  int e = validate(p);
  if (e) return e;
  int L, nc[3];
  e = plan_levels(p, &L, nc);
  if (e) return e;
  *levels = L;
  for (int d = 0; d < 3; ++d) n_coarse_out[d] = nc[d];
  return EXCMG_OK;
}

int excmg_workspace_bytes(const excmg_problem *p, size_t *bytes) {
  if (!p || !bytes) return EXCMG_ERR_ARG;
  Layout lo;
  const int e = make_layout(p, &lo);
  if (e) return e;
  *bytes = lo.total;
  return EXCMG_OK;
}

int excmg_setup(const excmg_problem *p, void *workspace, size_t bytes, void *hip_stream, excmg_handle **out) {
  if (!p || !out) return EXCMG_ERR_ARG;
  *out = nullptr;
  excmg_handle *h = new (std::nothrow) excmg_handle();
  if (!h) return EXCMG_ERR_ARG;
  int e = make_layout(p, &h->lo);
  if (e) {
    delete h;
    return e;
  }
  if (!workspace || bytes < h->lo.total || ((uintptr_t)workspace & 255)) {
    delete h;
    return EXCMG_ERR_WORKSPACE;
  }
  h->p = *p;
  h->stream = (hipStream_t)hip_stream;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return EXCMG_ERR_HIP;
  }
  h->ws = (char *)workspace;
  bind_workspace(h);
  // Thomas factors of the (1,4,1) systems: m_1 = 4, m_i = 4 - 1/m_{i-1}; the table holds 1/m_i at index i.
  const Level &fin = h->lo.lev[h->lo.L - 1];
  for (int d = 0; d < 3; ++d) {
    const int N = fin.n[d];
    std::vector<double> &v = h->inv_m_host[d];
    v.assign(N + 1, 0.0);
    double m = 4.0;
    for (int i = 1; i <= N - 1; ++i) {
      if (i > 1) m = 4.0 - 1.0 / m;
      v[i] = 1.0 / m;
    }
    if (hipMemcpyAsync(h->inv_m[d], v.data(), (N + 1) * sizeof(double), hipMemcpyHostToDevice, h->stream) !=
        hipSuccess) {
      delete h;
      return EXCMG_ERR_HIP;
    }
  }
  for (int l = 0; l <= EXCMG_MAX_LEVELS; ++l) {
    if (hipEventCreateWithFlags(&h->lev_ev[l], kTimingEvent) != hipSuccess) {
      delete h;
      return EXCMG_ERR_HIP;
    }
  }
  if (ensure_pinned(h, sizeof(CgState)) != EXCMG_OK ||
      hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking) != hipSuccess) {
    delete h;
    return EXCMG_ERR_HIP;
  }
  h->pool_used = 0;
  if (set_timing(h, (p->flags & EXCMG_WANT_TIMING) != 0) != EXCMG_OK) {
    delete h;
    return EXCMG_ERR_HIP;
  }
  launch_clear_gbnd2(h->cs, h->cs2, h->stream);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(h->stream) != hipSuccess) {
    delete h;
    return EXCMG_ERR_HIP;
  }
  *out = h;
  return EXCMG_OK;
}

int excmg_solve(excmg_handle *h, const double *f, const double *g, double *u, double *u_ext, excmg_stats *st) {
  if (!h || !f || !g || !u) return EXCMG_ERR_ARG;
  if (u_ext && h->lo.L < 2) return EXCMG_ERR_SHAPE;
  DeviceGuard dg(h->device);
  return solve_on(h, f, g, u, u_ext, st);
}

int excmg_solve_noalloc(const excmg_problem *p, const double *f, const double *g, double *u, double *u_ext,
                        void *hip_stream, excmg_stats *st) {
  if (!p || !f || !g || !u) return EXCMG_ERR_ARG;
  excmg_handle h{};  // host state only, on the stack
  int e = make_layout(p, &h.lo);
  if (e) return e;
  if (h.lo.total > kScratchBytes) return EXCMG_ERR_SCRATCH;
  if (u_ext && h.lo.L < 2) return EXCMG_ERR_SHAPE;
  h.p = *p;
  h.p.flags = (p->flags & ~EXCMG_WANT_TIMING) | EXCMG_NO_GRAPHS;
  h.noalloc = true;
  h.stream = (hipStream_t)hip_stream;
  HIPCHECK(hipGetDevice(&h.device));
  void *ws = nullptr;
  if ((e = scratch_address(h.device, &ws))) return e;
  h.ws = (char *)ws;
  bind_workspace(&h);
  launch_clear_gbnd2(h.cs, h.cs2, h.stream);  // what excmg_setup clears: the CG states' boundary norm terms
  if ((e = last_error())) return e;
  return solve_on(&h, f, g, u, u_ext, st);
}

}  // extern "C"

namespace {

// Algorithm 1 on a set-up handle (the device current): the cascade, then EXP_true or the copy of u_h to the caller.
int solve_on(excmg_handle *h, const double *f, const double *g, double *u, double *u_ext, excmg_stats *st) {
  const auto t0 = std::chrono::steady_clock::now();
  clear_stats(st);
  reset_timing(h);
  LevelIters li;
  memset(li.iters, 0, sizeof(li.iters));
  const int status = cascade(h, 0, f, g, st, h->noalloc ? nullptr : &li);
  if (status != EXCMG_OK && status != EXCMG_ERR_NOCONV) return status;
  Layout &lo = h->lo;
  const Level &fin = lo.lev[lo.L - 1];
  if (u_ext) {  // EXP_true also writes u to the caller's array from the same read of u_h
    Tick t(h, EXCMG_K_EXP_TRUE, lo.L - 1);
    launch_exp_true(fin.g, fin.u, lo.lev[lo.L - 2].g, lo.lev[lo.L - 2].u, lo.gdense, u_ext, u, h->stream);
  } else {
    Tick t(h, EXCMG_K_OTHER, lo.L - 1);
    launch_copy(fin.g, fin.u, lo.gdense, u, h->stream);
  }
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(h->stream));
  fill_level_stats(h, st);
  e = collect_timing(h, st, li);
  if (e) return e;
  if (st) st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

}  // namespace

// launches per trial of a self-finalizing pass, and the delay they are queued behind (longer than it takes the host
// to queue them: about 5 us per launch)
constexpr int kTuneBurst = 8;
constexpr double kTuneDelayUs = 120.0;
// candidates timed again after the first round, and the timed launches each gets then
constexpr int kTuneFinal = 4;
constexpr int kTuneFinalReps = 7;

extern "C" {

int excmg_gradient(excmg_handle *h, const double *u, double *ux, double *uy, double *uz) {
  if (!h || !u || !ux || !uy || !uz) return EXCMG_ERR_ARG;
  const Level &fin = h->lo.lev[h->lo.L - 1];
  if (fin.n[0] < 4 || fin.n[1] < 4 || fin.n[2] < 4) return EXCMG_ERR_SHAPE;
  DeviceGuard dg(h->device);
  const Grid &gd = h->lo.gdense;
  launch_gradient(gd, u, gd, ux, uy, uz, fin.h[0], fin.h[1], fin.h[2], h->inv_m[0], h->inv_m[1], h->inv_m[2],
                  h->stream);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(h->stream));
  return EXCMG_OK;
}

int excmg_adjoint(excmg_handle *h, const double *G, double *dLdf, double *dLdg, double *lambda_out,
                  excmg_stats *st) {
  if (!h || !G || !dLdf || !dLdg) return EXCMG_ERR_ARG;
  DeviceGuard dg(h->device);
  const auto t0 = std::chrono::steady_clock::now();
  clear_stats(st);
  reset_timing(h);
  LevelIters li;
  memset(li.iters, 0, sizeof(li.iters));
  const int status = cascade(h, 1, G, nullptr, st, &li);
  if (status != EXCMG_OK && status != EXCMG_ERR_NOCONV) return status;
  Layout &lo = h->lo;
  const Level &fin = lo.lev[lo.L - 1];
  launch_adjoint_transposes(fin.g, fin.u, lo.gdense, G, dLdf, dLdg, fin.h[0], fin.h[1], fin.h[2], h->stream);
  if (lambda_out) launch_copy(fin.g, fin.u, lo.gdense, lambda_out, h->stream);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(h->stream));
  fill_level_stats(h, st);
  e = collect_timing(h, st, li);
  if (e) return e;
  if (st) st->ms_total = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return status;
}

int excmg_autotune(excmg_handle *h, int32_t *zc_out, int32_t *depth_out) {
  if (!h) return EXCMG_ERR_ARG;
  DeviceGuard dg(h->device);
  h->drop_graphs();  // captured with the old sweep shapes
  const hipStream_t s = h->stream;
  Layout &lo = h->lo;
  static const int cand[] = {2, 4, 8, 16, 32, 64, 128, 256, 512};
  static const int depths[] = {2, 3, 4, 6};
  static const int heights[] = {4, 8, 16};
  constexpr int kDp = 2 * (int)(sizeof(depths) / sizeof(depths[0]));  // depth x cache policy
  constexpr int kVar = kDp * (int)(sizeof(heights) / sizeof(heights[0]));  // ... x tile height
  hipEvent_t ea, eb;
  HIPCHECK(hipEventCreateWithFlags(&ea, kTimingEvent));
  HIPCHECK(hipEventCreateWithFlags(&eb, kTimingEvent));
  int rc = EXCMG_OK;
  double *pa = h->partials, *pb = h->partials + lo.npart;
  for (int l = 0; l < lo.L && rc == EXCMG_OK; ++l) {
    Level &lv = lo.lev[l];
    if (!swept(lo, l)) continue;  // solved by the single-workgroup kernel
    const bool ir = l >= 2 && (h->p.precision == EXCMG_FP32_IR) && lv.g.interior() >= kIrMinUnknowns;
    // A grid whose iterations run as graphs of self-finalizing passes is tuned on those kernels, with the shapes that
    // keep it self-finalizing; their launches are short, so each trial times a burst of them queued behind a delay
    // (back to back, as in a graph) instead of one launch between two events, whose own cost would hide the kernel.
    const bool burst = use_graphs(h, l) && sweep_blocks(lv.sw) <= selfred_max_blocks();
    // a grid that will run the single-reduction CG has its pass-B shape (which that CG uses) timed on that CG's
    // iterations (the trial state makes every launch of parity 1 run iteration 1 in full)
    const bool cg1 = burst && cg1_eligible(h, l);
    // kinds: FP64 passes, FP32 passes (refinement grids), and the FP64 passes of the first iteration (p = r: pass A
    // reads r alone, pass B takes p from r's buffer) on grids whose passes finalize apart
    for (int kind = 0; kind < 3 && rc == EXCMG_OK; ++kind) {
      if ((kind == 1 && !ir) || (kind == 2 && burst)) continue;
      const int prec = kind == 1;
      const bool first = kind == 2;
      const Grid &g = prec ? lv.g32 : lv.g;
      for (int pass = 0; pass < 2 && rc == EXCMG_OK; ++pass) {
        float best = 1e30f;
        Sweep &dst = first ? (pass ? lv.swB0 : lv.swA0)
                           : prec ? (pass ? lv.swB32 : lv.swA32) : (pass ? lv.swB : lv.swA);
        Sweep bsw = dst;
        // partial sums the trial pass reads: as many as the other pass's current shape writes (at most the
        // self-finalizing limit; no sweep of a grid has more workgroups than its 2-plane chunks, which the
        // partials' halves hold three times over)
        const int nb_other = std::min(
            sweep_blocks(prec ? (pass ? lv.swA32 : lv.swB32) : (pass ? lv.swA : lv.swB)), selfred_max_blocks());
        // the fastest launch of reps timed trials of shape sw (the first of them only warms caches and code)
        auto trial = [&](const Sweep &sw, int reps) -> float {
          float tmin = 1e30f;
          for (int rep = 0; rep < reps && rc == EXCMG_OK; ++rep) {
            const bool cg1_trial = cg1 && prec == 0 && pass == 1;
            if (burst) {
              launch_tune_selfred(h->cs2, pass ? pa : pb, cg1_trial ? 2 * sweep_blocks(sw) : nb_other, s);
              launch_delay(kTuneDelayUs, s);
            } else {
              launch_tune_state(h->cs2, first ? 0 : 1, s);
            }
            if (hipEventRecord(ea, s) != hipSuccess) rc = EXCMG_ERR_HIP;
            for (int q = 0; q < (burst ? kTuneBurst : 1); ++q) {
              if (cg1_trial) {  // u and p: the first two slots of p1's buffer (the grid's u may not be bound yet)
                launch_cg1_iteration(sw, h->p1 + cg1_stride(lv), h->p1, cg1_vec(h, lv, 1, 0), cg1_vec(h, lv, 1, 1),
                                     cg1_vec(h, lv, 1, 2), cg1_vec(h, lv, 0, 0), cg1_vec(h, lv, 0, 1),
                                     cg1_vec(h, lv, 0, 2), h->cs2, 1, pa, cg1_resid_parts(h), sweep_blocks(lv.sw),
                                     1.0, pb, s);
              } else if (burst && prec == 0) {
                if (pass == 0) launch_selfred_a<double>(sw, h->r, h->p0, h->p1, h->cs2, pb, nb_other, 1.0, pa, s);
                else launch_selfred_b<double>(sw, h->r, h->r, h->p0, h->p1, h->cs2, pa, nb_other, pb, s);
              } else if (burst) {
                if (pass == 0) launch_selfred_a<float>(sw, h->r32, h->p32a, h->p32b, h->cs2, pb, nb_other, 1.0, pa, s);
                else launch_selfred_b<float>(sw, h->d32, h->r32, h->p32a, h->p32b, h->cs2, pa, nb_other, pb, s);
              } else if (prec == 0) {
                if (pass == 0) launch_cg_pass_a<double>(sw, h->r, h->p0, h->p1, h->cs2, h->partials, s);
                // u: a buffer the iteration does not use (iteration 1: r's, with r in p0 and p in p1; iteration 0:
                // p1, with r and p in r's buffer and the new r going to p0), so that the trial touches distinct
                // arrays as a real pass B does
                else launch_cg_pass_b<double>(sw, first ? h->p1 : h->r, h->r, h->p0, h->p1, h->cs2, h->partials, s);
              } else {
                if (pass == 0) launch_cg_pass_a<float>(sw, h->r32, h->p32a, h->p32b, h->cs2, h->partials, s);
                else launch_cg_pass_b<float>(sw, h->d32, h->r32, h->p32a, h->p32b, h->cs2, h->partials, s);
              }
            }
            if (hipEventRecord(eb, s) != hipSuccess || hipEventSynchronize(eb) != hipSuccess) rc = EXCMG_ERR_HIP;
            if (last_error() != EXCMG_OK) rc = EXCMG_ERR_HIP;
            if (rc) break;
            float ms = 0.0f;
            if (hipEventElapsedTime(&ms, ea, eb) != hipSuccess) rc = EXCMG_ERR_HIP;
            ms /= burst ? kTuneBurst : 1;
            if (rep > 0 && ms < tmin) tmin = ms;
          }
          return tmin;
        };
        // every candidate timed twice; then the kTuneFinal fastest again, kTuneFinalReps times each, so that a shape
        // is not kept for a difference within the timing noise of two launches
        std::vector<std::pair<float, Sweep>> timed;
        for (int ci = 0; ci < kVar * (int)(sizeof(cand) / sizeof(cand[0])) && rc == EXCMG_OK; ++ci) {
          const int zc = cand[ci / kVar], ty = heights[(ci % kVar) / kDp], depth = depths[(ci % kDp) / 2];
          const int nt = ci % 2;
          if (zc > 2 * (g.nz - 1) + 2) break;
          if (ty > 4 && ty / 2 >= g.ny - 1) continue;  // a tile at least twice the grid's height
          const Sweep sw = make_sweep(g, lv.st, zc, depth, nt, ty);
          if (3LL * sweep_blocks(sw) > lo.npart) continue;
          if (burst && sweep_blocks(sw) > selfred_max_blocks()) continue;
          if (cg1 && prec == 0 && pass == 1 && 4LL * sweep_blocks(sw) > lo.npart) continue;
          timed.push_back({trial(sw, 3), sw});
        }
        if (rc) break;
        std::sort(timed.begin(), timed.end(),
                  [](const std::pair<float, Sweep> &a, const std::pair<float, Sweep> &b) { return a.first < b.first; });
        for (size_t q = 0; q < timed.size() && q < (size_t)kTuneFinal && rc == EXCMG_OK; ++q) {
          const float t = std::min(timed[q].first, trial(timed[q].second, kTuneFinalReps));
          if (t < best) {
            best = t;
            bsw = timed[q].second;
          }
        }
        if (rc) break;
        dst = bsw;
      }
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  if (rc) return rc;
  if (zc_out) {
    for (int l = 0; l < lo.L; ++l) {
      const Level &lv = lo.lev[l];
      const bool relaxed = swept(lo, l);
      const bool ir = relaxed && l >= 2 && (h->p.precision == EXCMG_FP32_IR) && lv.g.interior() >= kIrMinUnknowns;
      zc_out[4 * l + 0] = relaxed ? lv.swA.zc : 0;
      zc_out[4 * l + 1] = relaxed ? lv.swB.zc : 0;
      zc_out[4 * l + 2] = ir ? lv.swA32.zc : 0;
      zc_out[4 * l + 3] = ir ? lv.swB32.zc : 0;
    }
  }
  if (depth_out) {
    for (int l = 0; l < lo.L; ++l) {
      const Level &lv = lo.lev[l];
      const bool relaxed = swept(lo, l);
      const bool ir = relaxed && l >= 2 && (h->p.precision == EXCMG_FP32_IR) && lv.g.interior() >= kIrMinUnknowns;
      auto code = [](const Sweep &sw) { return sw.depth + 10 * sw.nt + 100 * sw.ty; };
      depth_out[4 * l + 0] = relaxed ? code(lv.swA) : 0;
      depth_out[4 * l + 1] = relaxed ? code(lv.swB) : 0;
      depth_out[4 * l + 2] = ir ? code(lv.swA32) : 0;
      depth_out[4 * l + 3] = ir ? code(lv.swB32) : 0;
    }
  }
  return EXCMG_OK;
}

int excmg_batch_graph_counts(const excmg_handle *h, int64_t *replays, int64_t *captures) {
  if (!h || !replays || !captures) return EXCMG_ERR_ARG;
  *replays = h->bgraph_hits;
  *captures = h->bgraph_misses;
  return EXCMG_OK;
}

namespace {
// the sweep of grid l that kind names (EXCMG_SWEEP_*), or null
Sweep *sweep_of(excmg_handle *h, int l, int kind) {
  if (!h || l < 0 || l >= h->lo.L) return nullptr;
  Level &lv = h->lo.lev[l];
  switch (kind) {
    case EXCMG_SWEEP_A: return &lv.swA;
    case EXCMG_SWEEP_B: return &lv.swB;
    case EXCMG_SWEEP_A32: return &lv.swA32;
    case EXCMG_SWEEP_B32: return &lv.swB32;
    case EXCMG_SWEEP_A_FIRST: return &lv.swA0;
    case EXCMG_SWEEP_B_FIRST: return &lv.swB0;
    default: return nullptr;
  }
}
}  // namespace

int excmg_get_sweep(excmg_handle *h, int32_t level, int32_t kind, int32_t shape[4]) {
  const Sweep *sw = sweep_of(h, level, kind);
  if (!sw || !shape) return EXCMG_ERR_ARG;
  shape[0] = sw->zc;
  shape[1] = sw->depth;
  shape[2] = sw->nt;
  shape[3] = sw->ty;
  return EXCMG_OK;
}

int excmg_set_sweep(excmg_handle *h, int32_t level, int32_t kind, const int32_t shape[4]) {
  Sweep *sw = sweep_of(h, level, kind);
  if (!sw || !shape) return EXCMG_ERR_ARG;
  const int zc = shape[0], depth = shape[1], nt = shape[2], ty = shape[3];
  if (zc < 2 || (zc & 1) || zc > 4096 || !(depth == 2 || depth == 3 || depth == 4 || depth == 6) ||
      !(nt == 0 || nt == 1) || !(ty == 4 || ty == 8 || ty == 16))
    return EXCMG_ERR_ARG;
  const Sweep nw = make_sweep(sw->g, sw->st, zc, depth, nt, ty);
  if (3LL * sweep_blocks(nw) > h->lo.npart) return EXCMG_ERR_ARG;  // more workgroups than the partial sums hold
  DeviceGuard dg(h->device);
  HIPCHECK(hipStreamSynchronize(h->stream));  // no launch of an earlier call still uses the old shape
  *sw = nw;
  h->drop_graphs();  // captured with the old sweep shapes
  return EXCMG_OK;
}

int excmg_get_batch_shape(excmg_handle *h, int32_t shape[4]) {
  if (!h || !shape) return EXCMG_ERR_ARG;
  shape[0] = h->bty[0];
  shape[1] = h->bty[1];
  shape[2] = h->bdepth[0];
  shape[3] = h->bdepth[1];
  return EXCMG_OK;
}

int excmg_set_batch_shape(excmg_handle *h, const int32_t shape[4]) {
  if (!h || !shape) return EXCMG_ERR_ARG;
  for (int q = 0; q < 2; ++q) {
    if (!(shape[q] == 4 || shape[q] == 8 || shape[q] == 16)) return EXCMG_ERR_ARG;
    const int d = shape[2 + q];
    if (!(d == 2 || d == 3 || d == 4 || d == 6)) return EXCMG_ERR_ARG;
  }
  DeviceGuard dg(h->device);
  HIPCHECK(hipStreamSynchronize(h->stream));
  for (int q = 0; q < 2; ++q) {
    h->bty[q] = shape[q];
    h->bdepth[q] = shape[2 + q];
  }
  h->drop_graphs();
  return EXCMG_OK;
}

int excmg_set_timing(excmg_handle *h, int32_t on) {
  if (!h) return EXCMG_ERR_ARG;
  DeviceGuard dg(h->device);
  HIPCHECK(hipStreamSynchronize(h->stream));  // no timed launch of an earlier call is still pending
  return set_timing(h, on != 0);
}

void excmg_destroy(excmg_handle *h) {
  if (!h) return;
  DeviceGuard dg(h->device);
  (void)hipStreamSynchronize(h->stream);
  delete h;  // events and the pinned buffer are released by the handle's destructor
}

const char *excmg_strerror(int code) {
  switch (code) {
    case EXCMG_OK: return "ok";
    case EXCMG_ERR_ARG: return "invalid argument";
    case EXCMG_ERR_SHAPE: return "invalid grid shape or level plan";
    case EXCMG_ERR_NONFINITE: return "non-finite input data";
    case EXCMG_ERR_NOCONV: return "CG reached max_iters before the tolerance";
    case EXCMG_ERR_BREAKDOWN: return "CG breakdown (p.Ap <= 0 or non-finite scalar)";
    case EXCMG_ERR_HIP: return "HIP runtime error";
    case EXCMG_ERR_WORKSPACE: return "workspace missing, too small or not 256-byte aligned";
    case EXCMG_ERR_SCRATCH: return "problem too large for the fixed scratch array of excmg_solve_noalloc";
    default: return "unknown error code";
  }
}

// ---------------------------------------------------------------------------------------------- single steps

static int check_n(const int32_t n[3], int mult) {
  for (int d = 0; d < 3; ++d)
    if (n[d] < 2 || n[d] % mult) return EXCMG_ERR_SHAPE;
  return EXCMG_OK;
}

int excmg_op_apply(const int32_t n[3], const double box[3], const double *x, double *y, void *hip_stream) {
  if (!n || !box || !x || !y) return EXCMG_ERR_ARG;
  if (check_n(n, 1)) return EXCMG_ERR_SHAPE;
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0)) return EXCMG_ERR_ARG;
  const hipStream_t s = (hipStream_t)hip_stream;
  const Grid g = dense_grid(n[0], n[1], n[2]);
  HIPCHECK(hipMemsetAsync(y, 0, (size_t)g.elems * sizeof(double), s));
  launch_apply(g, x, g, y, make_stencil(box[0] / n[0], box[1] / n[1], box[2] / n[2]), s);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(s));
  return EXCMG_OK;
}

int excmg_op_rhs(const int32_t n[3], const double box[3], const double *f, const double *g, double *b,
                 void *hip_stream) {
  if (!n || !box || !f || !g || !b) return EXCMG_ERR_ARG;
  if (check_n(n, 1)) return EXCMG_ERR_SHAPE;
  for (int d = 0; d < 3; ++d)
    if (!(box[d] > 0.0)) return EXCMG_ERR_ARG;
  const hipStream_t s = (hipStream_t)hip_stream;
  const Grid gd = dense_grid(n[0], n[1], n[2]);
  HIPCHECK(hipMemsetAsync(b, 0, (size_t)gd.elems * sizeof(double), s));
  RhsSrc rs;
  rs.gf = gd;
  rs.f = f;
  rs.g = g;
  rs.s = 1;
  rs.mode = 0;
  rs.fg = 0;
  rs.a = (n[0] / box[0]) * (n[0] / box[0]);
  rs.b = (n[1] / box[1]) * (n[1] / box[1]);
  rs.c = (n[2] / box[2]) * (n[2] / box[2]);
  launch_rhs(rs, gd, b, s);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(s));
  return EXCMG_OK;
}

int excmg_op_exp_finite(const int32_t n[3], const double *u2h, const double *u4h, const double *g, double *w,
                        void *hip_stream) {
  if (!n || !u2h || !u4h || !g || !w) return EXCMG_ERR_ARG;
  if (check_n(n, 8)) return EXCMG_ERR_SHAPE;
  const hipStream_t s = (hipStream_t)hip_stream;
  const Grid gw = dense_grid(n[0], n[1], n[2]);
  const Grid g2 = dense_grid(n[0] / 2, n[1] / 2, n[2] / 2);
  const Grid g4 = dense_grid(n[0] / 4, n[1] / 4, n[2] / 4);
  launch_initial_guess(kGuessQuartic, g2, u2h, g4, u4h, gw, g, 1, gw, w, s);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(s));
  return EXCMG_OK;
}

int excmg_op_initial_guess(int32_t kind, const int32_t n[3], const double *u2h, const double *u4h, const double *g,
                           double *w, void *hip_stream) {
  if (kind != kGuessQuartic && kind != kGuessQuadratic && kind != kGuessLinear) return EXCMG_ERR_ARG;
  if (!n || !u2h || (kind != kGuessLinear && !u4h) || !g || !w) return EXCMG_ERR_ARG;
  if (check_n(n, kind == kGuessLinear ? 2 : 8)) return EXCMG_ERR_SHAPE;
  const hipStream_t s = (hipStream_t)hip_stream;
  const Grid gw = dense_grid(n[0], n[1], n[2]);
  const Grid g2 = dense_grid(n[0] / 2, n[1] / 2, n[2] / 2);
  const Grid g4 = dense_grid(n[0] / 4, n[1] / 4, n[2] / 4);
  launch_initial_guess(kind, g2, u2h, g4, u4h, gw, g, 1, gw, w, s);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(s));
  return EXCMG_OK;
}

int excmg_op_exp_true(const int32_t n[3], const double *uh, const double *u2h, double *ut, void *hip_stream) {
  if (!n || !uh || !u2h || !ut) return EXCMG_ERR_ARG;
  if (check_n(n, 2)) return EXCMG_ERR_SHAPE;
  const hipStream_t s = (hipStream_t)hip_stream;
  const Grid gh = dense_grid(n[0], n[1], n[2]);
  const Grid g2 = dense_grid(n[0] / 2, n[1] / 2, n[2] / 2);
  launch_exp_true(gh, uh, g2, u2h, gh, ut, nullptr, s);
  int e = last_error();
  if (e) return e;
  HIPCHECK(hipStreamSynchronize(s));
  return EXCMG_OK;
}

int excmg_bandwidth_probe(void *buf, size_t bytes, int32_t reps, void *hip_stream, double *GBs, int32_t *shapes) {
  if (!buf || bytes < 4096 || reps <= 0 || ((uintptr_t)buf & 15) || !GBs) return EXCMG_ERR_ARG;
  const hipStream_t s = (hipStream_t)hip_stream;
  const long long n = (long long)(bytes / sizeof(double)) & ~7LL;  // doubles, a multiple of 8
  const long long h = (n / 2) & ~1LL;                              // doubles per half (copy), even
  const long long m = (n / 3) & ~1LL;                              // doubles per third (mix), even
  double *a = (double *)buf;
  hipEvent_t e0, e1;
  HIPCHECK(hipEventCreateWithFlags(&e0, kTimingEvent));
  HIPCHECK(hipEventCreateWithFlags(&e1, kTimingEvent));
  HIPCHECK(hipMemsetAsync(buf, 0, (size_t)n * sizeof(double), s));
  // per kind: the sweep kernel's mode, cache policy, and the bytes it moves (read plus written)
  struct Kind {
    int mode;
    bool nt;
    double moved;
  };
  const Kind kinds[EXCMG_PROBE_KINDS] = {
      {0, false, 16.0 * h}, {1, false, 8.0 * n}, {0, true, 16.0 * h}, {1, true, 8.0 * n},
      {2, true, 40.0 * m},  {2, false, 40.0 * m}, {3, false, 8.0 * n}, {3, true, 8.0 * n}};
  // launch shapes: the first kernels of each kind are the fixed-shape originals (kinds 0-4), then the sweep
  static const int wgpc[] = {2, 4, 8, 16, 32, 64};
  static const int lanes[] = {2, 4, 8};
  struct Shape {
    int wg, u, chunk, legacy;
  };
  std::vector<Shape> sh;
  sh.push_back({0, 0, 0, 1});
  for (int w : wgpc)
    for (int u : lanes)
      for (int c = 0; c < 2; ++c) sh.push_back({w, u, c, 0});
  float best[EXCMG_PROBE_KINDS];
  Shape win[EXCMG_PROBE_KINDS];
  for (int k = 0; k < EXCMG_PROBE_KINDS; ++k) {
    best[k] = 1e30f;
    win[k] = {0, 0, 0, 0};
  }
  int rc = EXCMG_OK;
  for (int rep = 0; rep <= reps && rc == EXCMG_OK; ++rep) {
    for (int kind = 0; kind < EXCMG_PROBE_KINDS && rc == EXCMG_OK; ++kind) {
      const Kind &K = kinds[kind];
      for (const Shape &q : sh) {
        if (q.legacy && kind > EXCMG_PROBE_MIX_NT) continue;  // no fixed-shape original for these kinds
        if (hipEventRecord(e0, s) != hipSuccess) rc = EXCMG_ERR_HIP;
        if (q.legacy) {
          switch (kind) {
            case EXCMG_PROBE_COPY: launch_probe_copy(a, a + h, h, s); break;
            case EXCMG_PROBE_READ: launch_probe_read(a, n, a, s); break;
            case EXCMG_PROBE_COPY_NT: launch_probe_copy_nt(a, a + h, h, s); break;
            case EXCMG_PROBE_READ_NT: launch_probe_read_nt(a, n, a, s); break;
            default: launch_probe_mix_nt(a, a + m, a + 2 * m, m, s); break;
          }
        } else if (K.mode == 0) {
          launch_probe_sweep(0, q.u, K.nt, q.chunk != 0, q.wg, a, a + h, nullptr, h, a, s);
        } else if (K.mode == 2) {
          launch_probe_sweep(2, q.u, K.nt, q.chunk != 0, q.wg, a, a + m, a + 2 * m, m, a, s);
        } else {
          launch_probe_sweep(K.mode, q.u, K.nt, q.chunk != 0, q.wg, a, a, nullptr, n, a, s);
        }
        float ms = 0.0f;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
          rc = EXCMG_ERR_HIP;
        if (last_error() != EXCMG_OK) rc = EXCMG_ERR_HIP;
        if (rc) break;
        if (rep > 0 && ms < best[kind]) {  // the first pass warms up
          best[kind] = ms;
          win[kind] = q;
        }
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) return rc;
  for (int kind = 0; kind < EXCMG_PROBE_KINDS; ++kind) {
    GBs[kind] = kinds[kind].moved / (best[kind] * 1e-3) / 1e9;
    if (shapes) {
      const Shape &q = win[kind];
      // the fixed-shape originals run 8 (ordinary) or 32 (non-temporal) workgroups per CU, 4 accesses in flight
      shapes[3 * kind + 0] = q.legacy ? (kinds[kind].nt ? 32 : 8) : q.wg;
      shapes[3 * kind + 1] = q.legacy ? 4 : q.u;
      shapes[3 * kind + 2] = q.legacy ? 0 : q.chunk;
    }
  }
  return EXCMG_OK;
}

int excmg_batch_workspace_bytes(int32_t count, size_t *bytes) {
  if (count <= 0 || !bytes) return EXCMG_ERR_ARG;
  *bytes = batch_ws_bytes(count);
  return EXCMG_OK;
}

int excmg_autotune_batched(excmg_handle *const *hs, int32_t count, void *batch_ws, size_t batch_bytes,
                           int32_t *zc_out) {
  if (!hs || count <= 0) return EXCMG_ERR_ARG;
  for (int b = 0; b < count; ++b)
    if (!hs[b] || hs[b]->device != hs[0]->device) return EXCMG_ERR_ARG;
  if (!batch_ws || ((uintptr_t)batch_ws & 255) || batch_bytes < batch_ws_bytes(count)) return EXCMG_ERR_WORKSPACE;
  DeviceGuard dg(hs[0]->device);
  return batched_autotune(hs, count, (char *)batch_ws, zc_out);
}

int excmg_solve_batched(excmg_handle *const *hs, int32_t count, const double *const *f, const double *const *g,
                        double *const *u, void *batch_ws, size_t batch_bytes, excmg_stats *stats,
                        double *ms_per_problem) {
  if (!hs || count <= 0 || !f || !g || !u) return EXCMG_ERR_ARG;
  for (int b = 0; b < count; ++b)
    if (!hs[b] || !f[b] || !g[b] || !u[b] || hs[b]->device != hs[0]->device ||
        guess_kind(hs[b]->p.flags) != kGuessQuartic ||
        (hs[b]->p.flags & (EXCMG_STOP_F_G | EXCMG_STOP_F_G_BELOW_FINEST)))
      return EXCMG_ERR_ARG;
  if (!batch_ws || ((uintptr_t)batch_ws & 255) || batch_bytes < batch_ws_bytes(count)) return EXCMG_ERR_WORKSPACE;
  DeviceGuard dg(hs[0]->device);
  return batched_solve(hs, count, f, g, u, (char *)batch_ws, stats, ms_per_problem);
}

}  // extern "C"
