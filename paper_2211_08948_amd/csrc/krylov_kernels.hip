// Arnoldi's process on the augmented matrix of Sec. 2.1 (see
// krylov_kernels.hpp).  Every sum is formed per block in a fixed order and
// combined in block order -- by each block redundantly where the next pass
// needs the value -- so results do not depend on timing.  Once the basis
// breaks down (a zero new vector) the remaining kernels of the basis return
// at once.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "krylov_kernels.hpp"

namespace lj {

namespace {

__device__ __forceinline__ double kry_block_sum(double v, double* red) {
  const double w = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wv] = w;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];  // every thread, same order
  return t;
}

// sum over blocks b < G of part[b * stride + q], identical in every block
__device__ __forceinline__ double kry_grid_sum(const double* part, int G, int stride, int q, double* red) {
  double a = 0.0;
  for (int b = threadIdx.x; b < G; b += blockDim.x) a += part[(size_t)b * stride + q];
  return kry_block_sum(a, red);
}

constexpr int kPartStride = kKryMaxDim + 1;  // per block: dots, then the norm

__global__ __launch_bounds__(kKryBlock) void kry_norm_partial_kernel(KryDev K, const double* __restrict__ w) {
  __shared__ double red[kKryBlock / 64];
  double a = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x)
    a += w[i] * w[i];
  const double t = kry_block_sum(a, red);
  if (threadIdx.x == 0) K.part[(size_t)blockIdx.x * kPartStride + kKryMaxDim] = t;
}

__global__ __launch_bounds__(kKryBlock) void kry_start_scale_kernel(KryDev K, const double* __restrict__ w) {
  __shared__ double red[kKryBlock / 64];
  const double beta = sqrt(kry_grid_sum(K.part, gridDim.x, kPartStride, kKryMaxDim, red));
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    K.scalars[0] = beta;
    K.scalars[1] = 0.0;
  }
  if (!(beta > 0.0)) return;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x)
    K.V[i] = w[i] / beta;
}

__global__ __launch_bounds__(kKryBlock) void kry_tail_dots_kernel(KryDev K, int j, int lo, int d0, int nd,
                                                                 int tail) {
  __shared__ double red[kKryBlock / 64];
  if (K.scalars[1] != 0.0) return;
  const double* vj = K.V + (size_t)j * K.na;
  double y[kKryMaxP];
  for (int k = 0; k < kKryMaxP; ++k) y[k] = (k < K.p) ? vj[K.N + k] : 0.0;
  double acc[kKryChunk];
  for (int d = 0; d < kKryChunk; ++d) acc[d] = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x) {
    double x;
    if (tail) {
      if (i < K.N) {
        x = K.W[i];
        for (int k = 0; k < K.p; ++k)
          if (K.B[k] != nullptr) x = x + y[k] * K.B[k][i];
      } else {
        const long t = i - K.N;  // (K y)_t = y_{t+1}, the last entry 0
        x = (t + 1 < K.p) ? y[t + 1] : 0.0;
      }
      K.W[i] = x;
    } else {
      x = K.W[i];
    }
#pragma unroll
    for (int d = 0; d < kKryChunk; ++d)
      if (d < nd) acc[d] += K.V[(size_t)(lo + d0 + d) * K.na + i] * x;
  }
  for (int d = 0; d < nd; ++d) {
    const double t = kry_block_sum(acc[d], red);
    if (threadIdx.x == 0) K.part[(size_t)blockIdx.x * kPartStride + d0 + d] = t;
  }
}

__global__ __launch_bounds__(kKryBlock) void kry_update_kernel(KryDev K, int j, int lo, int ndt) {
  __shared__ double red[kKryBlock / 64];
  __shared__ double hs[kKryMaxDim];
  if (K.scalars[1] != 0.0) return;
  for (int d = 0; d < ndt; ++d) {
    const double t = kry_grid_sum(K.part, gridDim.x, kPartStride, d, red);
    if (threadIdx.x == 0) hs[d] = t;
  }
  __syncthreads();
  if (blockIdx.x == 0 && threadIdx.x < ndt) K.H[(size_t)(lo + threadIdx.x) * K.m + j] = hs[threadIdx.x];
  double a = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x) {
    double x = K.W[i];
    for (int d = 0; d < ndt; ++d) x = x - hs[d] * K.V[(size_t)(lo + d) * K.na + i];
    K.W[i] = x;
    a += x * x;
  }
  const double t = kry_block_sum(a, red);
  if (threadIdx.x == 0) K.part[(size_t)blockIdx.x * kPartStride + kKryMaxDim] = t;
}

__global__ __launch_bounds__(kKryBlock) void kry_scale_kernel(KryDev K, int j) {
  __shared__ double red[kKryBlock / 64];
  if (K.scalars[1] != 0.0) return;
  const double hn = sqrt(kry_grid_sum(K.part, gridDim.x, kPartStride, kKryMaxDim, red));
  const bool broke = !(hn > 1e-300);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    K.H[(size_t)(j + 1) * K.m + j] = hn;
    if (broke) K.scalars[1] = (double)(j + 1);
  }
  if (broke) return;
  double* vn = K.V + (size_t)(j + 1) * K.na;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x)
    vn[i] = K.W[i] / hn;
}

__global__ __launch_bounds__(kKryBlock) void kry_combine_kernel(KryDev K, int m, double beta, KryCoef F,
                                                               double* __restrict__ out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int c = 0; c < m; ++c) a += K.V[(size_t)c * K.na + i] * F.f[c];
    out[i] = beta * a;
  }
}

__global__ __launch_bounds__(kKryBlock) void kry_init_kernel(double* w, const double* b0, long N, int p) {
  const long na = N + p;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < na; i += (long)gridDim.x * blockDim.x) {
    if (i < N) {
      w[i] = (b0 != nullptr) ? b0[i] : 0.0;
    } else {
      w[i] = (i == na - 1) ? 1.0 : 0.0;
    }
  }
}

// Contiguous point range of this block, chunks of 64 points, consecutive
// chunks on one XCD (blocks are dispatched round-robin over the 8 XCDs).
__device__ __forceinline__ void kry_point_range(int npts, int& p0, int& p1) {
  const int G = gridDim.x;
  const int b = blockIdx.x;
  const int cb = (G % 8 == 0) ? (b % 8) * (G / 8) + (b / 8) : b;
  const int chunk = (((npts + G - 1) / G) + 63) & ~63;
  p0 = min(npts, cb * chunk);
  p1 = min(npts, p0 + chunk);
}

template <int KIND, int NC>
__global__ __launch_bounds__(kKryPBlock) void kry_arnoldi_kernel(KryArnoldi P) {
  const GridSync gs{P.barrier, P.spin_limit};
  __shared__ double red[kKryChunk * (kKryPBlock / 64 + 1)];
  __shared__ double tot[kKryChunk];
  const KryDev& K = P.K;
  const OpDev& op = P.op;
  const long N = K.N, na = K.na;
  const int np = K.p;
  int p0, p1;
  kry_point_range(op.npts, p0, p1);
  // the auxiliary entries N .. N + np - 1 belong to block 0, one per thread
  const bool aux = blockIdx.x == 0 && (int)threadIdx.x < np;
  const long ia = N + threadIdx.x;
  unsigned int epoch = 0;

  // beta = ||w||
  double s1[1] = {0.0};
  for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x)
#pragma unroll
    for (int c = 0; c < NC; ++c) s1[0] += P.w[NC * p + c] * P.w[NC * p + c];
  if (aux) s1[0] += P.w[ia] * P.w[ia];
  block_sum<1>(s1, red);
  double* area = partial_area(P.partials, epoch);
  if (threadIdx.x == 0) put_partial(my_partial(area, 0), s1[0]);
  grid_allreduce(gs, epoch, area, 1, tot);
  double hs = sqrt(tot[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    K.scalars[0] = hs;
    K.scalars[1] = 0.0;
  }
  const double* src = P.w;  // V_j = src / hs
  if (hs > 0.0) {
    for (int j = 0; j < K.m; ++j) {
      double* dst = P.Wb[j & 1];
      double* vj = K.V + (size_t)j * na;
      const int lo = max(0, j - P.window + 1);
      const int nd = j - lo + 1;
      double y[kKryMaxP];
#pragma unroll
      for (int k = 0; k < kKryMaxP; ++k) y[k] = (k < np) ? src[N + k] / hs : 0.0;
      double acc[kKryChunk];
#pragma unroll
      for (int d = 0; d < kKryChunk; ++d) acc[d] = 0.0;
      // (1) x = J V_j + B y (grid part), x = K y (auxiliary part); the dots
      for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
        double xv[5][2], uv[5][2], out[2];
        gather_point<KIND, NC>(op, src, p, xv, uv);
#pragma unroll
        for (int t = 0; t < 5; ++t)
#pragma unroll
          for (int c = 0; c < NC; ++c) xv[t][c] = xv[t][c] / hs;
        stencil_jv<KIND>(op, xv, uv, out);
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const long i = (long)NC * p + c;
          const double v = xv[0][c];
          store_shared(vj + i, v);
          double x = out[c];
          for (int k = 0; k < np; ++k)
            if (K.B[k] != nullptr) x = x + y[k] * K.B[k][i];
          store_shared(dst + i, x);
#pragma unroll
          for (int d = 0; d < kKryChunk; ++d)
            if (d < nd) acc[d] += ((d == nd - 1) ? v : K.V[(size_t)(lo + d) * na + i]) * x;
        }
      }
      if (aux) {
        const double v = src[ia] / hs;
        store_shared(vj + ia, v);
        const int t = threadIdx.x;
        const double x = (t + 1 < np) ? y[t + 1] : 0.0;
        store_shared(dst + ia, x);
#pragma unroll
        for (int d = 0; d < kKryChunk; ++d)
          if (d < nd) acc[d] += ((d == nd - 1) ? v : K.V[(size_t)(lo + d) * na + ia]) * x;
      }
      block_sum<kKryChunk>(acc, red);
      area = partial_area(P.partials, epoch);
      if (threadIdx.x == 0) {
#pragma unroll
        for (int d = 0; d < kKryChunk; ++d)
          if (d < nd) put_partial(my_partial(area, d), acc[d]);
      }
      grid_allreduce(gs, epoch, area, nd, tot);
      if (blockIdx.x == 0 && (int)threadIdx.x < nd) K.H[(size_t)(lo + threadIdx.x) * K.m + j] = tot[threadIdx.x];
      // (2) x -= sum_d h_d V_{lo+d} in order of d; ||x||^2
      double s2[1] = {0.0};
      for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const long i = (long)NC * p + c;
          double x = dst[i];
          for (int d = 0; d < nd; ++d) x = x - tot[d] * K.V[(size_t)(lo + d) * na + i];
          store_shared(dst + i, x);
          s2[0] += x * x;
        }
      if (aux) {
        double x = dst[ia];
        for (int d = 0; d < nd; ++d) x = x - tot[d] * K.V[(size_t)(lo + d) * na + ia];
        store_shared(dst + ia, x);
        s2[0] += x * x;
      }
      block_sum<1>(s2, red);
      area = partial_area(P.partials, epoch);
      if (threadIdx.x == 0) put_partial(my_partial(area, 0), s2[0]);
      grid_allreduce(gs, epoch, area, 1, tot);
      const double hn = sqrt(tot[0]);
      const bool broke = !(hn > 1e-300);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        K.H[(size_t)(j + 1) * K.m + j] = hn;
        if (broke) K.scalars[1] = (double)(j + 1);
      }
      if (broke) break;
      src = dst;
      hs = hn;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) K.scalars[2] = grid_aborted(P.barrier) != 0u ? 1.0 : 0.0;
  grid_exit(P.barrier);
}

}  // namespace

const void* kry_arnoldi_ptr(int kind) {
  switch (kind) {
    case OP_DIAG: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_DIAG, 1>);
    case OP_ADVDIFF: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_ADVDIFF, 1>);
    case OP_ALLENCAHN: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_ALLENCAHN, 1>);
    case OP_BRUSSELATOR: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_BRUSSELATOR, 2>);
    case OP_BURGERS: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_BURGERS, 1>);
    case OP_GRAYSCOTT: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_GRAYSCOTT, 2>);
    case OP_ADR: return reinterpret_cast<const void*>(&kry_arnoldi_kernel<OP_ADR, 1>);
    default: return nullptr;
  }
}

int kry_grid(long n) {
  long g = (n + kKryBlock - 1) / kKryBlock;
  if (g > kKryBlocksMax) g = kKryBlocksMax;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_kry_start(const KryDev& K, const double* w, hipStream_t s) {
  const int G = kry_grid(K.na);
  hipLaunchKernelGGL(kry_norm_partial_kernel, dim3(G), dim3(kKryBlock), 0, s, K, w);
  hipLaunchKernelGGL(kry_start_scale_kernel, dim3(G), dim3(kKryBlock), 0, s, K, w);
  return hipGetLastError();
}

hipError_t launch_kry_tail_dots(const KryDev& K, int j, int lo, int d0, int nd, bool tail, hipStream_t s) {
  hipLaunchKernelGGL(kry_tail_dots_kernel, dim3(kry_grid(K.na)), dim3(kKryBlock), 0, s, K, j, lo, d0, nd,
                     tail ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_kry_update(const KryDev& K, int j, int lo, int nd_total, hipStream_t s) {
  hipLaunchKernelGGL(kry_update_kernel, dim3(kry_grid(K.na)), dim3(kKryBlock), 0, s, K, j, lo, nd_total);
  return hipGetLastError();
}

hipError_t launch_kry_scale(const KryDev& K, int j, hipStream_t s) {
  hipLaunchKernelGGL(kry_scale_kernel, dim3(kry_grid(K.na)), dim3(kKryBlock), 0, s, K, j);
  return hipGetLastError();
}

hipError_t launch_kry_combine(const KryDev& K, int m, double beta, const KryCoef& F, double* out, hipStream_t s) {
  hipLaunchKernelGGL(kry_combine_kernel, dim3(kry_grid(K.na)), dim3(kKryBlock), 0, s, K, m, beta, F, out);
  return hipGetLastError();
}

hipError_t launch_kry_init(double* w, const double* b0, long N, int p, hipStream_t s) {
  hipLaunchKernelGGL(kry_init_kernel, dim3(kry_grid(N + p)), dim3(kKryBlock), 0, s, w, b0, N, p);
  return hipGetLastError();
}

}  // namespace lj
