// Achievable HBM bandwidth on this device, measured with plain streaming kernels of known byte counts: a copy (read
// n doubles, write n doubles) and a read-only sum, with ordinary and with non-temporal accesses, and the access mix
// of the CG's pass B (three reads, two writes).  16-byte accesses, several independent accesses in flight per lane,
// grid-stride loops.  Used as the same-run ceilings beside the solver's sweeps; the ordinary copy also scales the
// hardware traffic counters.
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

}  // namespace excmg
