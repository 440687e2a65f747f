// Attainable HBM bandwidth of the device, for reading the roofline fractions:
// streaming kernels over FP64 vectors far larger than the last-level cache --
// a copy (1 read, 1 write), a read-only sum, and the access pattern of one
// Newton step of the Leja recurrence at one accumulator (y_{m-1} and the
// state read, y_m written, p read and written: 3 reads, 2 writes).
#include <hip/hip_runtime.h>

#include "../../include/leja.h"

namespace {

__global__ __launch_bounds__(256) void bw_copy(const double2* __restrict__ a, double2* __restrict__ b, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) b[i] = a[i];
}

__global__ __launch_bounds__(256) void bw_read(const double2* __restrict__ a, long n, double* sink) {
  double s = 0.0;
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double2 v = a[i];
    s += v.x + v.y;
  }
  if (s == -1.0) sink[0] = s;  // the inputs are zeros: never taken, but the loads stay
}

__global__ __launch_bounds__(256) void bw_step(const double2* __restrict__ y, const double2* __restrict__ u,
                                               double2* __restrict__ yn, double2* __restrict__ p, long n) {
  for (long i = blockIdx.x * 256L + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const double2 a = y[i], b = u[i];
    double2 c = p[i], r;
    r.x = a.x * b.x - 0.5 * a.x;
    r.y = a.y * b.y - 0.5 * a.y;
    yn[i] = r;
    c.x += 1e-3 * r.x;
    c.y += 1e-3 * r.y;
    p[i] = c;
  }
}

}  // namespace

// gbs[0..2] = copy, read, Newton-step pattern in GB/s (best of 5 timed runs
// after one warm-up, 1024 blocks of 256 threads); `bytes` per vector (a
// multiple of 16, at least 64 MiB), four vectors allocated and freed here.
extern "C" LJ_API int lj_measure_bandwidth(long long bytes, double* gbs) {
  if (!gbs || bytes < (64ll << 20) || bytes % 16 != 0) return LJ_EINVAL;
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
    const int G = 1024;
    for (int kind = 0; kind < 3 && rc == LJ_OK; ++kind) {
      float best = 1e30f;
      for (int r = 0; r < 6; ++r) {
        (void)hipEventRecord(e0, nullptr);
        if (kind == 0) hipLaunchKernelGGL(bw_copy, dim3(G), dim3(256), 0, nullptr, (const double2*)a, (double2*)b, n2);
        if (kind == 1) hipLaunchKernelGGL(bw_read, dim3(G), dim3(256), 0, nullptr, (const double2*)a, n2, sink);
        if (kind == 2)
          hipLaunchKernelGGL(bw_step, dim3(G), dim3(256), 0, nullptr, (const double2*)a, (const double2*)b,
                             (double2*)c, (double2*)d, n2);
        (void)hipEventRecord(e1, nullptr);
        if (hipEventSynchronize(e1) != hipSuccess) {
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
