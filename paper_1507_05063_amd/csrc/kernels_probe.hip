// Achievable HBM bandwidth on this device, measured with plain streaming kernels of known byte counts: a copy (read
// n doubles, write n doubles) and a read-only sum, with ordinary and with non-temporal accesses, and the access mix
// of the CG's pass B (three reads, two writes).  16-byte accesses, several independent accesses in flight per lane,
// grid-stride loops.  Used as the same-run ceilings beside the solver's sweeps; the ordinary copy also scales the
// hardware traffic counters.
#include <type_traits>

#include "excmg_internal.h"

namespace excmg {

namespace {

constexpr int PT = 256;
constexpr int PU = 4;  // 16-byte accesses in flight per lane

__global__ __launch_bounds__(PT) void probe_copy_kernel(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                        long long n2) {
  const long long stride = (long long)gridDim.x * PT;
  long long q = (long long)blockIdx.x * PT + threadIdx.x;
  for (; q + (PU - 1) * stride < n2; q += PU * stride) {
    double2 v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) v[u] = src[q + u * stride];
#pragma unroll
    for (int u = 0; u < PU; ++u) dst[q + u * stride] = v[u];
  }
  for (; q < n2; q += stride) dst[q] = src[q];
}

__global__ __launch_bounds__(PT) void probe_read_kernel(const double2 *__restrict__ src, long long n2, double *sink) {
  const long long stride = (long long)gridDim.x * PT;
  long long q = (long long)blockIdx.x * PT + threadIdx.x;
  double acc = 0.0;
  for (; q + (PU - 1) * stride < n2; q += PU * stride) {
    double2 v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) v[u] = src[q + u * stride];
#pragma unroll
    for (int u = 0; u < PU; ++u) acc += v[u].x + v[u].y;
  }
  for (; q < n2; q += stride) acc += src[q].x + src[q].y;
  if (acc == 1.2345e300) sink[0] = acc;  // keeps the loads; never true for the probe's data
}

// Non-temporal forms (native 2-wide vectors, which the non-temporal builtins take) and the mix of the CG's pass B:
// three arrays read, two written.  They run 32 workgroups per CU, where these forms measured fastest.
typedef double pv2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(PT) void probe_copy_nt_kernel(const pv2 *__restrict__ src, pv2 *__restrict__ dst,
                                                           long long n2) {
  const long long stride = (long long)gridDim.x * PT;
  long long q = (long long)blockIdx.x * PT + threadIdx.x;
  for (; q + (PU - 1) * stride < n2; q += PU * stride) {
    pv2 v[PU];
#pragma unroll
    for (int u = 0; u < PU; ++u) v[u] = __builtin_nontemporal_load(&src[q + u * stride]);
#pragma unroll
    for (int u = 0; u < PU; ++u) __builtin_nontemporal_store(v[u], &dst[q + u * stride]);
  }
  for (; q < n2; q += stride) __builtin_nontemporal_store(__builtin_nontemporal_load(&src[q]), &dst[q]);
}

__global__ __launch_bounds__(PT) void probe_read_nt_kernel(const pv2 *__restrict__ src, long long n2, double *sink) {
  constexpr int R = 2 * PU;
  const long long stride = (long long)gridDim.x * PT;
  long long q = (long long)blockIdx.x * PT + threadIdx.x;
  double acc = 0.0;
  for (; q + (R - 1) * stride < n2; q += R * stride) {
    pv2 v[R];
#pragma unroll
    for (int u = 0; u < R; ++u) v[u] = __builtin_nontemporal_load(&src[q + u * stride]);
#pragma unroll
    for (int u = 0; u < R; ++u) acc += v[u].x + v[u].y;
  }
  for (; q < n2; q += stride) {
    const pv2 v = __builtin_nontemporal_load(&src[q]);
    acc += v.x + v.y;
  }
  if (acc == 1.2345e300) sink[0] = acc;  // keeps the loads; never true for the probe's data
}

__global__ __launch_bounds__(PT) void probe_mix_nt_kernel(const pv2 *__restrict__ a, pv2 *__restrict__ b,
                                                          pv2 *__restrict__ c, long long m) {
  constexpr int R = PU / 2;
  const long long stride = (long long)gridDim.x * PT;
  long long q = (long long)blockIdx.x * PT + threadIdx.x;
  auto one = [&](long long i, pv2 x, pv2 y, pv2 z) {
    __builtin_nontemporal_store(y + 0.5 * x, &b[i]);
    __builtin_nontemporal_store(z - 0.5 * x, &c[i]);
  };
  for (; q + (R - 1) * stride < m; q += R * stride) {
    pv2 x[R], y[R], z[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      x[u] = __builtin_nontemporal_load(&a[q + u * stride]);
      y[u] = __builtin_nontemporal_load(&b[q + u * stride]);
      z[u] = __builtin_nontemporal_load(&c[q + u * stride]);
    }
#pragma unroll
    for (int u = 0; u < R; ++u) one(q + u * stride, x[u], y[u], z[u]);
  }
  for (; q < m; q += stride) one(q, a[q], b[q], c[q]);
}

// The sweep of launch shapes: one kernel per (access mix, 16-byte accesses in flight per lane, cache policy, pattern).
// MODE 0: copy a -> b; 1: read a; 2: pass B's mix, b += a/2 and c -= a/2 (three arrays read, two written); 3: write b.
// CHUNK: each workgroup streams through one contiguous range of the arrays (the way a stencil sweep's workgroup
// marches through its tile) instead of striding over the whole grid.
template <bool NTP>
__device__ __forceinline__ pv2 pld(const pv2 *p) {
  if constexpr (NTP) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NTP>
__device__ __forceinline__ void pst(pv2 v, pv2 *p) {
  if constexpr (NTP) __builtin_nontemporal_store(v, p);
  else *p = v;
}

template <int MODE, int U, bool NTP, bool CHUNK>
__global__ __launch_bounds__(PT) void probe_sweep_kernel(const pv2 *__restrict__ a, pv2 *__restrict__ b,
                                                         pv2 *__restrict__ c, long long m, double *sink) {
  long long q, end, step;  // this thread's first element, the end of its range, and the distance between its rounds
  long long lane_stride;   // distance between its U accesses of one round
  if constexpr (CHUNK) {
    const long long per = ((m + gridDim.x - 1) / gridDim.x + PT - 1) / PT * PT;
    const long long s0 = (long long)blockIdx.x * per;
    end = s0 + per < m ? s0 + per : m;
    q = s0 + threadIdx.x;
    lane_stride = PT;
  } else {
    end = m;
    q = (long long)blockIdx.x * PT + threadIdx.x;
    lane_stride = (long long)gridDim.x * PT;
  }
  step = U * lane_stride;
  double acc = 0.0;
  const pv2 fill = {1.0, 2.0};
  auto one = [&](long long i, pv2 x, pv2 y, pv2 z) {
    if constexpr (MODE == 0) pst<NTP>(x, &b[i]);
    if constexpr (MODE == 1) acc += x.x + x.y;
    if constexpr (MODE == 2) {
      pst<NTP>(y + 0.5 * x, &b[i]);
      pst<NTP>(z - 0.5 * x, &c[i]);
    }
    if constexpr (MODE == 3) pst<NTP>(fill, &b[i]);
  };
  for (; q + (U - 1) * lane_stride < end; q += step) {
    pv2 x[U], y[U], z[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = q + u * lane_stride;
      if constexpr (MODE != 3) x[u] = pld<NTP>(&a[i]);
      if constexpr (MODE == 2) {
        y[u] = pld<NTP>(&b[i]);
        z[u] = pld<NTP>(&c[i]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) one(q + u * lane_stride, x[u], y[u], z[u]);
  }
  for (; q < end; q += lane_stride) {
    pv2 x = fill, y = fill, z = fill;
    if constexpr (MODE != 3) x = pld<NTP>(&a[q]);
    if constexpr (MODE == 2) {
      y = pld<NTP>(&b[q]);
      z = pld<NTP>(&c[q]);
    }
    one(q, x, y, z);
  }
  if constexpr (MODE == 1)
    if (acc == 1.2345e300) sink[0] = acc;  // keeps the loads; never true for the probe's data
}

int probe_blocks() {
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    hipDeviceProp_t pr;
    if (hipGetDeviceProperties(&pr, dev) == hipSuccess && pr.multiProcessorCount > 0) cus = pr.multiProcessorCount;
  }
  return 8 * cus;
}

}  // namespace

void launch_probe_copy(const double *src, double *dst, long long n, hipStream_t st) {
  probe_copy_kernel<<<probe_blocks(), PT, 0, st>>>((const double2 *)src, (double2 *)dst, n / 2);
}

void launch_probe_read(const double *src, long long n, double *sink, hipStream_t st) {
  probe_read_kernel<<<probe_blocks(), PT, 0, st>>>((const double2 *)src, n / 2, sink);
}

void launch_probe_copy_nt(const double *src, double *dst, long long n, hipStream_t st) {
  probe_copy_nt_kernel<<<4 * probe_blocks(), PT, 0, st>>>((const pv2 *)src, (pv2 *)dst, n / 2);
}

void launch_probe_read_nt(const double *src, long long n, double *sink, hipStream_t st) {
  probe_read_nt_kernel<<<4 * probe_blocks(), PT, 0, st>>>((const pv2 *)src, n / 2, sink);
}

void launch_probe_mix_nt(const double *a, double *b, double *c, long long n, hipStream_t st) {
  probe_mix_nt_kernel<<<4 * probe_blocks(), PT, 0, st>>>((const pv2 *)a, (pv2 *)b, (pv2 *)c, n / 2);
}

int probe_cus() { return probe_blocks() / 8; }

// One launch of the sweep kernel of a shape: mode (0 copy, 1 read, 2 mix, 3 write), 16-byte accesses in flight per
// lane (2, 4 or 8), cache policy, pattern; wg_per_cu workgroups per compute unit.  a, b, c: arrays of n doubles each
// (n even; b and c unused where the mode does not need them; sink: a double the read mode may write).
void launch_probe_sweep(int mode, int u, bool nt, bool chunk, int wg_per_cu, const double *a, double *b, double *c,
                        long long n, double *sink, hipStream_t st) {
  const int grid = wg_per_cu * probe_cus();
  const long long m = n / 2;
  auto go = [&](auto md, auto uu, auto ntp, auto ch) {
    probe_sweep_kernel<decltype(md)::value, decltype(uu)::value, decltype(ntp)::value, decltype(ch)::value>
        <<<grid, PT, 0, st>>>((const pv2 *)a, (pv2 *)b, (pv2 *)c, m, sink);
  };
  auto by_chunk = [&](auto md, auto uu, auto ntp) {
    if (chunk) go(md, uu, ntp, std::true_type{});
    else go(md, uu, ntp, std::false_type{});
  };
  auto by_nt = [&](auto md, auto uu) {
    if (nt) by_chunk(md, uu, std::true_type{});
    else by_chunk(md, uu, std::false_type{});
  };
  auto by_u = [&](auto md) {
    if (u == 2) by_nt(md, std::integral_constant<int, 2>{});
    else if (u == 4) by_nt(md, std::integral_constant<int, 4>{});
    else by_nt(md, std::integral_constant<int, 8>{});
  };
  switch (mode) {
    case 0: by_u(std::integral_constant<int, 0>{}); break;
    case 1: by_u(std::integral_constant<int, 1>{}); break;
    case 2: by_u(std::integral_constant<int, 2>{}); break;
    default: by_u(std::integral_constant<int, 3>{}); break;
  }
}

}  // namespace excmg
