// Kernels of the Leja phi-action library for gfx950 (CDNA4, wave64).
//
//  * lj_power_kernel   -- persistent power iteration (Sec. 2.2 spectral estimate)
//  * lj_divdiff_kernel -- phi_l at the scaled Leja nodes + Newton divided
//                         differences (Sec. 2.2), one workgroup per accumulator
//  * lj_leja_kernel    -- persistent fused Newton recurrence (Sec. 2.2 display,
//                         vertical form of Sec. 4): stencil J y, basis update,
//                         K accumulator axpys, norm partials, grid barrier,
//                         stop/reject decision -- all iterations in one launch
//  * small streaming kernels for f(u), remainders and linear combinations
//
// All arithmetic is FP64 (vector ALU); the path is bandwidth/latency bound and
// has no dense contraction, so no MFMA is used.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "kernels.hpp"

namespace lj {

constexpr int kBlock = 1024;    // threads per block of the persistent kernels (one block per CU)
constexpr int kWaves = kBlock / 64;
constexpr int kNV = kMaxK + 1;  // reduced values per iteration: ||y||^2 and K ||p_k||^2

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a run of
// consecutive chunks so that halo rows shared by neighbouring chunks mostly
// stay inside one XCD's L2.
__device__ __forceinline__ int xcd_chunk(int b, int G) {
  if (G % 8 != 0) return b;
  return (b % 8) * (G / 8) + (b / 8);
}

__device__ __forceinline__ void point_range(int npts, int& p0, int& p1) {
  const int G = gridDim.x;
  const int chunk = (((npts + G - 1) / G) + 63) & ~63;
  const int cb = xcd_chunk(blockIdx.x, G);
  p0 = min(npts, cb * chunk);
  p1 = min(npts, p0 + chunk);
}

// Every block sums the per-block partials of one slot in the same fixed order;
// totals land in tot[0..nq) for all threads.
__device__ __forceinline__ void grid_totals(const double* __restrict__ part, int nq, double* red,
                                            double (&tot)[kNV]) {
  const int G = gridDim.x;
#pragma unroll
  for (int q = 0; q < kNV; ++q) tot[q] = 0.0;
  for (int b = threadIdx.x; b < G; b += blockDim.x) {
#pragma unroll
    for (int q = 0; q < kNV; ++q)
      if (q < nq) tot[q] += part[b * kNV + q];
  }
  block_sum<kNV>(tot, red);
}

// ---------------------------------------------------------------------------
// Power iteration: x_{k+1} = J x_k / ||J x_k||, lambda = ||J x_{K-1}|| / ||x_{K-1}||.
// The normalisation of x_k is folded into the next product (J(s y) = s J y).
// ---------------------------------------------------------------------------
template <int KIND, int NC>
__global__ __launch_bounds__(kBlock) void lj_power_kernel(PowerParams P) {
  __shared__ double red[kNV * kWaves + kNV];
  const OpDev& op = P.op;
  const int npts = op.npts;
  const int G = gridDim.x;
  int p0, p1;
  point_range(npts, p0, p1);
  unsigned int epoch = 0;
  const double* x0 = P.start;
  if (x0 == nullptr) {
    for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int idx = NC * p + cc;
        P.buf1[idx] = 0.5 + splitmix_uniform(P.seed, (uint64_t)idx);
      }
    }
    x0 = P.buf1;
    grid_barrier(P.barrier, epoch);
  }
  double scale = 1.0;
  double lam = 0.0;
  for (int k = 0; k < P.iters; ++k) {
    const double* src = (k == 0) ? x0 : ((k & 1) ? P.buf0 : P.buf1);
    double* dst = (k & 1) ? P.buf1 : P.buf0;
    double acc[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
      double out[2], xc[2];
      jv_point<KIND>(op, src, p, out, xc);
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const double x = scale * xc[cc];
        const double y = scale * out[cc];
        dst[NC * p + cc] = y;
        acc[0] += x * x;
        acc[1] += y * y;
      }
    }
    block_sum<kNV>(acc, red);
    double* part = P.partials + (size_t)(k & 1) * G * kNV;
    if (threadIdx.x == 0) {
      part[blockIdx.x * kNV + 0] = acc[0];
      part[blockIdx.x * kNV + 1] = acc[1];
    }
    grid_barrier(P.barrier, epoch);
    double tot[kNV];
    grid_totals(part, 2, red, tot);
    const double nx = sqrt(tot[0]);
    const double ny = sqrt(tot[1]);
    lam = ny / nx;
    if (ny == 0.0) {
      lam = 0.0;
      break;
    }
    scale = 1.0 / ny;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) P.scal->lam = lam;
}

// ---------------------------------------------------------------------------
// Divided differences of phi_l(s (c + gamma xi_j)), j < npts, one block per
// accumulator.  Also fixes the interval: alpha = -safety*lambda, beta = 0,
// c = (alpha+beta)/2, gamma = (beta-alpha)/4 (Sec. 2.2).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(128) void lj_divdiff_kernel(DDParams P) {
#pragma clang fp contract(off)
  __shared__ double d[kTable + 1];
  __shared__ double xs[kTable + 1];
  __shared__ double fm[2];
  const int k = blockIdx.x;
  const int j = threadIdx.x;
  const double lam = P.use_cg ? 0.0 : ((P.lam_host > 0.0) ? P.lam_host : P.scal->lam);
  const double alpha = -P.safety * lam;
  const double beta = 0.0;
  const double c = P.use_cg ? P.c_in : 0.5 * (alpha + beta);
  const double gamma = P.use_cg ? P.gamma_in : 0.25 * (beta - alpha);
  const int n = P.npts;
  const double s = P.s[k];
  double f = 0.0;
  if (j < n) {
    const double x = P.xi[j];
    xs[j] = x;
    const double z = s * (c + gamma * x);
    f = phi_dev(P.l[k], z);
    d[j] = f;
  }
  // max |f_j| over the block (two waves)
  double a = fabs(f);
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) a = fmax(a, __shfl_down(a, off, 64));
  if ((j & 63) == 0) fm[j >> 6] = a;
  __syncthreads();
  for (int order = 1; order < n; ++order) {
    double t = 0.0;
    if (j < n && j >= order) t = (d[j] - d[j - 1]) / (xs[j] - xs[j - order]);
    __syncthreads();
    if (j < n && j >= order) d[j] = t;
    __syncthreads();
  }
  if (j < n) P.coef[k * kTable + j] = d[j];
  if (j == 0) {
    P.fmax[k] = fmax(fm[0], fm[1]);
    if (k == 0 && !P.use_cg) {
      P.scal->lam = lam;
      P.scal->c = c;
      P.scal->gamma = gamma;
    }
  }
}

// ---------------------------------------------------------------------------
// Fused Leja recurrence.  One launch runs every iteration m = 1..max_points:
//   y_m = ((J - c) / gamma - xi_{m-1}) y_{m-1},  p_k += d_{k,m} y_m (active k),
// with ||y_m||^2 and ||p_k||^2 reduced per block, published to a slot of the
// partials array, summed by every block after the grid barrier in one fixed
// order, and the stop/reject decision taken identically by every block.
// ---------------------------------------------------------------------------
template <int KIND, int NC>
__global__ __launch_bounds__(kBlock) void lj_leja_kernel(LejaParams P) {
  __shared__ double s_coef[kMaxK * kTable];
  __shared__ double red[kNV * kWaves + kNV];
  const OpDev& op = P.op;
  const int npts = op.npts;
  const int K = P.K;
  const int G = gridDim.x;
  int p0, p1;
  point_range(npts, p0, p1);
  for (int i = threadIdx.x; i < K * kTable; i += blockDim.x) s_coef[i] = P.coef[i];
  const double c = P.scal->c;
  const double gamma = P.scal->gamma;
  __syncthreads();
  unsigned int epoch = 0;

  // m = 0: p_k = d_{k,0} v, and ||v||^2
  {
    double acc[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int idx = NC * p + cc;
        const double vv = P.v[idx];
        acc[0] += vv * vv;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k)
          if (k < K) P.p[k][idx] = s_coef[k * kTable] * vv;
      }
    }
    block_sum<kNV>(acc, red);
    if (threadIdx.x == 0) P.partials[blockIdx.x * kNV] = acc[0];
  }
  grid_barrier(P.barrier, epoch);
  double tot[kNV];
  grid_totals(P.partials, 1, red, tot);
  const double nv = sqrt(tot[0]);

  int st[kMaxK], mst[kMaxK];
  double err[kMaxK], hump[kMaxK];
  int n_active = 0;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    st[k] = (k < K) ? ACC_RUNNING : ACC_CONVERGED;
    mst[k] = -1;
    err[k] = 0.0;
    hump[k] = (k < K) ? P.hump * nv * P.fmax[k] : 0.0;
    if (k < K) ++n_active;
  }
  int iters = 0, accum_iters = 0;
  if (nv == 0.0) {
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      st[k] = ACC_CONVERGED;
      mst[k] = (k < K) ? 0 : -1;
    }
    n_active = 0;
  }

  for (int m = 1; m <= P.max_points && n_active > 0; ++m) {
    const double* __restrict__ src = (m == 1) ? P.v : ((m & 1) ? P.ybuf0 : P.ybuf1);
    double* __restrict__ dst = (m & 1) ? P.ybuf1 : P.ybuf0;
    const double xim = P.xi[m - 1];
    double dk[kMaxK];
    bool act[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      act[k] = (k < K) && (st[k] == ACC_RUNNING);
      dk[k] = act[k] ? s_coef[k * kTable + m] : 0.0;
    }
    double acc[kNV] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
      double out[2], xc[2];
      jv_point<KIND>(op, src, p, out, xc);
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int idx = NC * p + cc;
        const double y = (out[cc] - c * xc[cc]) / gamma - xim * xc[cc];
        dst[idx] = y;
        acc[0] += y * y;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
          if (act[k]) {
            const double pk = P.p[k][idx] + dk[k] * y;
            P.p[k][idx] = pk;
            acc[1 + k] += pk * pk;
          }
        }
      }
    }
    block_sum<kNV>(acc, red);
    double* part = P.partials + (size_t)(m & 1) * G * kNV;
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < kNV; ++q) part[blockIdx.x * kNV + q] = acc[q];
    }
    grid_barrier(P.barrier, epoch);
    grid_totals(part, 1 + K, red, tot);
    ++iters;
    accum_iters += n_active;
    const double ny = sqrt(tot[0]);
    n_active = 0;
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      if (!act[k]) continue;
      const double e = fabs(dk[k]) * ny;
      const double np = sqrt(tot[1 + k]);
      if (!(isfinite(e) && isfinite(np))) {
        st[k] = ACC_NONFINITE;
      } else if (e > hump[k]) {
        st[k] = ACC_HUMP;
      } else if (e <= (P.relative ? P.tol * np : P.tol)) {
        st[k] = ACC_CONVERGED;
        mst[k] = m;
        err[k] = e;
      } else if (m == P.max_points) {
        st[k] = ACC_MAXPTS;
      } else {
        ++n_active;
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      P.status->state[k] = st[k];
      P.status->m_star[k] = mst[k];
      P.status->err[k] = err[k];
    }
    P.status->iters = iters;
    P.status->accum_iters = accum_iters;
    P.status->vnorm = nv;
  }
}

// ---------------------------------------------------------------------------
// Streaming helpers.
// ---------------------------------------------------------------------------
__global__ void lj_fill_u32_kernel(unsigned int* p, int n, unsigned int value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = value;
}

template <int KIND, int NC>
__global__ __launch_bounds__(256) void lj_rhs_kernel(OpDev op, const double* __restrict__ u,
                                                     double* __restrict__ f) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < op.npts; p += gridDim.x * blockDim.x) {
    double out[2];
    rhs_point<KIND>(op, u, p, out);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) f[NC * p + cc] = out[cc];
  }
}

// R = f(x) - fu - J(state) d with d = x - state precomputed (Sec. 1 remainder)
template <int KIND, int NC>
__global__ __launch_bounds__(256) void lj_remainder_kernel(OpDev op, const double* __restrict__ x,
                                                           const double* __restrict__ d,
                                                           const double* __restrict__ fu,
                                                           double* __restrict__ r) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < op.npts; p += gridDim.x * blockDim.x) {
    double fx[2], jd[2], dc[2];
    rhs_point<KIND>(op, x, p, fx);
    jv_point<KIND>(op, d, p, jd, dc);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) r[NC * p + cc] = (fx[cc] - fu[NC * p + cc]) - jd[cc];
  }
}

__global__ __launch_bounds__(256) void lj_lincomb_kernel(LinComb L) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < L.n; i += (long)gridDim.x * blockDim.x) {
    double s = L.alpha[0] * L.x[0][i];
    for (int q = 1; q < L.nin; ++q) s += L.alpha[q] * L.x[q][i];
    L.out[i] = s;
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers (host side).
// ---------------------------------------------------------------------------
template <int KIND, int NC>
static void* leja_fn() { return reinterpret_cast<void*>(&lj_leja_kernel<KIND, NC>); }
template <int KIND, int NC>
static void* power_fn() { return reinterpret_cast<void*>(&lj_power_kernel<KIND, NC>); }

void* leja_kernel_ptr(int kind) {
  switch (kind) {
    case OP_DIAG: return leja_fn<OP_DIAG, 1>();
    case OP_ADVDIFF: return leja_fn<OP_ADVDIFF, 1>();
    case OP_ALLENCAHN: return leja_fn<OP_ALLENCAHN, 1>();
    case OP_BRUSSELATOR: return leja_fn<OP_BRUSSELATOR, 2>();
    case OP_BURGERS: return leja_fn<OP_BURGERS, 1>();
  }
  return nullptr;
}

void* power_kernel_ptr(int kind) {
  switch (kind) {
    case OP_DIAG: return power_fn<OP_DIAG, 1>();
    case OP_ADVDIFF: return power_fn<OP_ADVDIFF, 1>();
    case OP_ALLENCAHN: return power_fn<OP_ALLENCAHN, 1>();
    case OP_BRUSSELATOR: return power_fn<OP_BRUSSELATOR, 2>();
    case OP_BURGERS: return power_fn<OP_BURGERS, 1>();
  }
  return nullptr;
}

int persistent_block() { return kBlock; }

hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int value, hipStream_t s) {
  hipLaunchKernelGGL(lj_fill_u32_kernel, dim3((n + 255) / 256), dim3(256), 0, s, p, n, value);
  return hipGetLastError();
}

hipError_t launch_divdiff(const DDParams& P, hipStream_t s) {
  hipLaunchKernelGGL(lj_divdiff_kernel, dim3(P.K), dim3(128), 0, s, P);
  return hipGetLastError();
}

static int stream_grid(long n) {
  long g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

template <int KIND, int NC>
static void rhs_t(const OpDev& op, const double* u, double* f, hipStream_t s) {
  hipLaunchKernelGGL((lj_rhs_kernel<KIND, NC>), dim3(stream_grid(op.npts)), dim3(256), 0, s, op, u, f);
}
template <int KIND, int NC>
static void rem_t(const OpDev& op, const double* x, const double* d, const double* fu, double* r,
                  hipStream_t s) {
  hipLaunchKernelGGL((lj_remainder_kernel<KIND, NC>), dim3(stream_grid(op.npts)), dim3(256), 0, s, op,
                     x, d, fu, r);
}

hipError_t launch_rhs(const OpDev& op, const double* u, double* f, hipStream_t s) {
  switch (op.kind) {
    case OP_DIAG: rhs_t<OP_DIAG, 1>(op, u, f, s); break;
    case OP_ADVDIFF: rhs_t<OP_ADVDIFF, 1>(op, u, f, s); break;
    case OP_ALLENCAHN: rhs_t<OP_ALLENCAHN, 1>(op, u, f, s); break;
    case OP_BRUSSELATOR: rhs_t<OP_BRUSSELATOR, 2>(op, u, f, s); break;
    case OP_BURGERS: rhs_t<OP_BURGERS, 1>(op, u, f, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_remainder(const OpDev& op, const double* x, const double* d, const double* fu,
                            double* r, hipStream_t s) {
  switch (op.kind) {
    case OP_DIAG: rem_t<OP_DIAG, 1>(op, x, d, fu, r, s); break;
    case OP_ADVDIFF: rem_t<OP_ADVDIFF, 1>(op, x, d, fu, r, s); break;
    case OP_ALLENCAHN: rem_t<OP_ALLENCAHN, 1>(op, x, d, fu, r, s); break;
    case OP_BRUSSELATOR: rem_t<OP_BRUSSELATOR, 2>(op, x, d, fu, r, s); break;
    case OP_BURGERS: rem_t<OP_BURGERS, 1>(op, x, d, fu, r, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lincomb(const LinComb& L, hipStream_t s) {
  hipLaunchKernelGGL(lj_lincomb_kernel, dim3(stream_grid(L.n)), dim3(256), 0, s, L);
  return hipGetLastError();
}

}  // namespace lj
