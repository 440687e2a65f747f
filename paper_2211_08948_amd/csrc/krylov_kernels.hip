// Arnoldi's process on the augmented matrix of Sec. 2.1 (see
// krylov_kernels.hpp).  Every sum is formed per block in a fixed order and
// combined in block order -- by each block redundantly where the next pass
// needs the value -- so results do not depend on timing.  Once the basis
// breaks down (a zero new vector) the remaining kernels of the basis return
// at once.
#include <hip/hip_runtime.h>

#include <algorithm>

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

// The sum runs over c in order; the basis entries are loaded eight at a time
// before they are used, so eight loads per thread are in flight.
__global__ __launch_bounds__(kKryBlock) void kry_combine_kernel(KryDev K, int m, double beta, KryCoef F,
                                                               double* __restrict__ out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < K.na; i += (long)gridDim.x * blockDim.x) {
    double a = 0.0;
    int c = 0;
    for (; c + 8 <= m; c += 8) {
      double v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) v[q] = K.V[(size_t)(c + q) * K.na + i];
#pragma unroll
      for (int q = 0; q < 8; ++q) a += v[q] * F.f[c + q];
    }
    for (; c < m; ++c) a += K.V[(size_t)c * K.na + i] * F.f[c];
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

// One phase per column, one grid all-reduce per phase.  With u_j the
// orthogonalised, not yet normalised vector of column j (u_0 = w) and
// eta_j = ||u_j||, V_j = u_j / eta_j, the product is applied to u_j, and
// A~ V_j = z_j / eta_j with z_j = A~ u_j (A~ is linear).  Phase k (0 <= k <= m):
//   u_k = z_{k-1} / eta_{k-1} - h_{k-2,k-1} V_{k-2} - h_{k-1,k-1} V_{k-1}
//   (the window's terms in that order; u_0 = w), formed at the point and,
//   for the stencil, at its neighbours from z_{k-1}, u_{k-1} (V_{k-1} =
//   u_{k-1} / eta_{k-1}) and the stored V_{k-2}, all written before the last
//   barrier; V_{k-1} is stored; ||u_k||^2 partials; for k < m: z_k = A~ u_k
//   and the window's dot partials <V_{k-1}, z_k> and <u_k, z_k>.
// After the all-reduce: eta_k, H[k][k-1] = eta_k (k >= 1, breakdown below
// 1e-300 ends the basis), H[k-1][k] = <V_{k-1}, z_k> / eta_k and
// H[k][k] = <u_k, z_k> / eta_k / eta_k.  u and z alternate between two
// buffers each, so a phase's gathers never race the next phase's writes.
// Every load of a phase is unconditional (absent terms read a valid
// stand-in and are multiplied by nothing), so all of a point's loads are in
// flight at once: the phase costs one memory round trip, not one per term.
template <int KIND, int NC>
__global__ __launch_bounds__(kKryPBlock) void kry_arnoldi_kernel(KryArnoldi P) {
  const GridSync gs{P.barrier, P.spin_limit};
  constexpr int kSlots = 3;  // <V_{k-1}, z_k>, <u_k, z_k>, ||u_k||^2
  __shared__ double red[kSlots * (kKryPBlock / 64 + 1)];
  __shared__ double tot[kSlots];
  const KryDev& K = P.K;
  const OpDev& op = P.op;
  const long N = K.N, na = K.na;
  const int np = K.p;
  const int m = K.m;
  int p0, p1;
  kry_point_range(op.npts, p0, p1);
  // the auxiliary entries N .. N + np - 1 belong to block 0, one per thread
  const bool aux = blockIdx.x == 0 && (int)threadIdx.x < np;
  const long ia = N + threadIdx.x;
  unsigned int epoch = 0;
  double eta_prev = 1.0;    // eta_{k-1}
  double h_a = 0.0;         // h_{k-2,k-1} (0 when outside the window)
  double h_b = 0.0;         // h_{k-1,k-1}
  bool two_prev = false;    // the window of column k-1 held V_{k-2}
  for (int k = 0; k <= m; ++k) {
    const double* Zp = P.Z[(k + 1) & 1];  // z_{k-1}
    const double* Up = P.U[(k + 1) & 1];  // u_{k-1}
    // V_{k-2}, or a valid stand-in whose term is not used
    const double* Va = two_prev ? K.V + (size_t)(k - 2) * na : Up;
    double* Uk = P.U[k & 1];
    double* Zk = P.Z[k & 1];
    double* Vprev = K.V + (size_t)(k > 0 ? k - 1 : 0) * na;
    const bool prod = k < m;
    const bool two = P.window >= 2 && k >= 1;  // column k's window holds V_{k-1}
    // u_k from the loaded values at one element
    auto u_from = [&](double z, double u1, double va) -> double {
      double x = z / eta_prev;
      if (two_prev) x = x - h_a * va;
      return x - h_b * (u1 / eta_prev);
    };
    // tail of u_k (the same in every thread)
    double y[kKryMaxP];
    {
      double zt[kKryMaxP], ut[kKryMaxP], vt[kKryMaxP];
#pragma unroll
      for (int t = 0; t < kKryMaxP; ++t) {
        const long e = N + min(t, max(np - 1, 0));
        const bool ok = np > 0;
        zt[t] = (k > 0 && ok) ? Zp[e] : 0.0;
        ut[t] = (k > 0 && ok) ? Up[e] : 0.0;
        vt[t] = (k > 0 && ok) ? Va[e] : 0.0;
        if (k == 0) zt[t] = ok ? P.w[e] : 0.0;
      }
#pragma unroll
      for (int t = 0; t < kKryMaxP; ++t) y[t] = (t < np) ? (k == 0 ? zt[t] : u_from(zt[t], ut[t], vt[t])) : 0.0;
    }
    double acc[kSlots] = {0.0, 0.0, 0.0};
    for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
      double xv[5][2], uv[5][2], out[2], ucen[2];
#pragma unroll
      for (int t = 0; t < 5; ++t) {
        xv[t][0] = xv[t][1] = 0.0;
        uv[t][0] = uv[t][1] = 0.0;
      }
      int idx[5];
      if constexpr (KIND == OP_DIAG) {
        idx[0] = idx[1] = idx[2] = idx[3] = idx[4] = p;
      } else {
        const Nbr q = neighbours<KIND>(op, p);
        idx[0] = q.c;
        idx[1] = q.w;
        idx[2] = q.e;
        idx[3] = q.s;
        idx[4] = q.n;
      }
      constexpr int nt = (KIND == OP_DIAG) ? 1 : 5;
      double zl[5][2], ul[5][2], vl[5][2];
#pragma unroll
      for (int t = 0; t < nt; ++t)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const long e = (long)NC * idx[t] + c;
          if (k == 0) {
            zl[t][c] = P.w[e];
            ul[t][c] = vl[t][c] = 0.0;
          } else {
            zl[t][c] = Zp[e];
            ul[t][c] = Up[e];
            vl[t][c] = Va[e];
          }
        }
#pragma unroll
      for (int t = 0; t < nt; ++t)
#pragma unroll
        for (int c = 0; c < NC; ++c) xv[t][c] = (k == 0) ? zl[t][c] : u_from(zl[t][c], ul[t][c], vl[t][c]);
#pragma unroll
      for (int c = 0; c < NC; ++c) ucen[c] = ul[0][c];
      if (prod) {
        if constexpr (KIND == OP_DIAG) {
          uv[0][0] = op.state[p];
        } else {
          constexpr int su = StateUse<KIND>::value;
#pragma unroll
          for (int t = 0; t < su; ++t)
#pragma unroll
            for (int c = 0; c < NC; ++c) uv[t][c] = op.state[NC * idx[t] + c];
        }
        stencil_jv<KIND>(op, xv, uv, out);
      }
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const long e = (long)NC * p + c;
        const double u = xv[0][c];
        double vk1 = 0.0;
        if (k > 0) {
          vk1 = ucen[c] / eta_prev;
          store_shared(Vprev + e, vk1);
        }
        store_shared(Uk + e, u);
        acc[2] += u * u;
        if (prod) {
          double z = out[c];
          for (int t = 0; t < np; ++t)
            if (K.B[t] != nullptr) z = z + y[t] * K.B[t][e];
          store_shared(Zk + e, z);
          if (two) acc[0] += vk1 * z;
          acc[1] += u * z;
        }
      }
    }
    if (aux) {
      const int t = threadIdx.x;
      const double u = y[t];
      double vk1 = 0.0;
      if (k > 0) {
        vk1 = Up[ia] / eta_prev;
        store_shared(Vprev + ia, vk1);
      }
      store_shared(Uk + ia, u);
      acc[2] += u * u;
      if (prod) {
        const double z = (t + 1 < np) ? y[t + 1] : 0.0;
        store_shared(Zk + ia, z);
        if (two) acc[0] += vk1 * z;
        acc[1] += u * z;
      }
    }
    block_sum<kSlots>(acc, red);
    double* area = partial_area(P.partials, epoch);
    if (threadIdx.x == 0) {
      put_partial(my_partial(area, 0), acc[0]);
      put_partial(my_partial(area, 1), acc[1]);
      put_partial(my_partial(area, 2), acc[2]);
    }
    grid_allreduce(gs, epoch, area, kSlots, tot);
    const double eta = sqrt(tot[2]);
    if (k == 0) {
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        K.scalars[0] = eta;
        K.scalars[1] = 0.0;
      }
      if (!(eta > 0.0)) break;  // w = 0
    } else {
      const bool broke = !(eta > 1e-300);
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        K.H[(size_t)k * m + (k - 1)] = eta;
        if (broke) K.scalars[1] = (double)k;
      }
      if (broke) break;
    }
    if (!prod) break;
    const double hk1 = tot[0] / eta;         // h_{k-1,k}
    const double hkk = tot[1] / eta / eta;   // h_{k,k}
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (two) K.H[(size_t)(k - 1) * m + k] = hk1;
      K.H[(size_t)k * m + k] = hkk;
    }
    h_a = two ? hk1 : 0.0;
    h_b = hkk;
    two_prev = two;
    eta_prev = eta;
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
  // one entry per thread up to 4096 blocks: the pass reads m vectors
  const long g = std::min<long>(std::max<long>((K.na + kKryBlock - 1) / kKryBlock, 1), 4096);
  hipLaunchKernelGGL(kry_combine_kernel, dim3((int)g), dim3(kKryBlock), 0, s, K, m, beta, F, out);
  return hipGetLastError();
}

hipError_t launch_kry_init(double* w, const double* b0, long N, int p, hipStream_t s) {
  hipLaunchKernelGGL(kry_init_kernel, dim3(kry_grid(N + p)), dim3(kKryBlock), 0, s, w, b0, N, p);
  return hipGetLastError();
}

}  // namespace lj
