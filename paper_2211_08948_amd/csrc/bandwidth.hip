// Attainable HBM bandwidth of the device, for reading the roofline fractions:
// streaming kernels over FP64 vectors far larger than the last-level cache --
// a copy (1 read, 1 write), a read-only sum, and the access pattern of one
// Newton step of the Leja recurrence at one accumulator (y_{m-1} and the
// state read, y_m written, p read and written: 3 reads, 2 writes) -- at a
// chosen launch shape, number of 16-byte accesses in flight per thread, and
// with ordinary or non-temporal (streaming, cache-bypassing) loads and stores.
#include <hip/hip_runtime.h>

#include "../../include/leja.h"

namespace {

template <bool NT>
__device__ __forceinline__ double2 ld(const double2* p) {
  if constexpr (NT) {
    double2 v;
    v.x = __builtin_nontemporal_load(&p->x);
    v.y = __builtin_nontemporal_load(&p->y);
    return v;
  } else {
    return *p;
  }
}

template <bool NT>
__device__ __forceinline__ void st(double2* p, double2 v) {
  if constexpr (NT) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}

// Each thread handles U grid-stride elements per round: all U loads are
// issued before the first use; elements past n are skipped.
template <int U, bool NT>
__global__ void bw_copy(const double2* __restrict__ a, double2* __restrict__ b, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride * U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n) v[u] = ld<NT>(a + i + u * stride);
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * stride < n) st<NT>(b + i + u * stride, v[u]);
  }
}

template <int U, bool NT>
__global__ void bw_read(const double2* __restrict__ a, long n, double* sink) {
  const long stride = (long)gridDim.x * blockDim.x;
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride * U) {
    double2 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = (i + u * stride < n) ? ld<NT>(a + i + u * stride) : double2{0.0, 0.0};
#pragma unroll
    for (int u = 0; u < U; ++u) s += v[u].x + v[u].y;
  }
  if (s == -1.0) sink[0] = s;  // the inputs are zeros: never taken, but the loads stay
}

template <int U, bool NT>
__global__ void bw_step(const double2* __restrict__ y, const double2* __restrict__ w, double2* __restrict__ yn,
                        double2* __restrict__ p, long n) {
  const long stride = (long)gridDim.x * blockDim.x;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride * U) {
    double2 a[U], b[U], c[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i + u * stride >= n) continue;
      a[u] = ld<NT>(y + i + u * stride);
      b[u] = ld<NT>(w + i + u * stride);
      c[u] = ld<NT>(p + i + u * stride);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (i + u * stride >= n) continue;
      double2 r;
      r.x = a[u].x * b[u].x - 0.5 * a[u].x;
      r.y = a[u].y * b[u].y - 0.5 * a[u].y;
      st<NT>(yn + i + u * stride, r);
      c[u].x += 1e-3 * r.x;
      c[u].y += 1e-3 * r.y;
      st<NT>(p + i + u * stride, c[u]);
    }
  }
}

template <int U, bool NT>
void launch(int kind, int G, int T, double* a, double* b, double* c, double* d, long n2, double* sink) {
  if (kind == 0) hipLaunchKernelGGL((bw_copy<U, NT>), dim3(G), dim3(T), 0, nullptr, (const double2*)a, (double2*)b, n2);
  if (kind == 1) hipLaunchKernelGGL((bw_read<U, NT>), dim3(G), dim3(T), 0, nullptr, (const double2*)a, n2, sink);
  if (kind == 2)
    hipLaunchKernelGGL((bw_step<U, NT>), dim3(G), dim3(T), 0, nullptr, (const double2*)a, (const double2*)b,
                       (double2*)c, (double2*)d, n2);
}

void launch_any(int U, bool nt, int kind, int G, int T, double* a, double* b, double* c, double* d, long n2,
                double* sink) {
  if (U == 1) nt ? launch<1, true>(kind, G, T, a, b, c, d, n2, sink) : launch<1, false>(kind, G, T, a, b, c, d, n2, sink);
  if (U == 2) nt ? launch<2, true>(kind, G, T, a, b, c, d, n2, sink) : launch<2, false>(kind, G, T, a, b, c, d, n2, sink);
  if (U == 4) nt ? launch<4, true>(kind, G, T, a, b, c, d, n2, sink) : launch<4, false>(kind, G, T, a, b, c, d, n2, sink);
}

}  // namespace

extern "C" LJ_API int lj_measure_bandwidth_shape(long long bytes, int blocks, int threads, int unroll,
                                                 int nontemporal, double* gbs) {
  if (!gbs || bytes < (64ll << 20) || bytes % 16 != 0) return LJ_EINVAL;
  if (blocks < 1 || blocks > (1 << 20) || threads < 64 || threads > 1024 || threads % 64 != 0) return LJ_EINVAL;
  if (unroll != 1 && unroll != 2 && unroll != 4) return LJ_EINVAL;
  const long n2 = (long)(bytes / 16);
  double *a = nullptr, *b = nullptr, *c = nullptr, *d = nullptr, *sink = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = LJ_OK;
  if (hipMalloc(&a, bytes) != hipSuccess || hipMalloc(&b, bytes) != hipSuccess || hipMalloc(&c, bytes) != hipSuccess ||
      hipMalloc(&d, bytes) != hipSuccess || hipMalloc(&sink, 8) != hipSuccess) {
    rc = LJ_ENOMEM;
  } else if (hipMemset(a, 0, bytes) != hipSuccess || hipMemset(b, 0, bytes) != hipSuccess ||
             hipMemset(c, 0, bytes) != hipSuccess || hipMemset(d, 0, bytes) != hipSuccess ||
             hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    rc = LJ_EHIP;
  } else {
    for (int kind = 0; kind < 3 && rc == LJ_OK; ++kind) {
      float best = 1e30f;
      for (int r = 0; r < 6; ++r) {
        (void)hipEventRecord(e0, nullptr);
        launch_any(unroll, nontemporal != 0, kind, blocks, threads, a, b, c, d, n2, sink);
        (void)hipEventRecord(e1, nullptr);
        if (hipGetLastError() != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
          rc = LJ_EHIP;
          break;
        }
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (r > 0 && ms < best) best = ms;
      }
      const double moved = (kind == 0 ? 2.0 : kind == 1 ? 1.0 : 5.0) * (double)bytes;
      gbs[kind] = moved / (best * 1e-3) / 1e9;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  for (double* x : {a, b, c, d, sink})
    if (x) (void)hipFree(x);
  return rc;
}

extern "C" LJ_API int lj_measure_bandwidth(long long bytes, double* gbs) {
  return lj_measure_bandwidth_shape(bytes, 1024, 256, 1, 0, gbs);
}
