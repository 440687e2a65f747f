// User-operator path: the Newton recurrence (Sec. 2.2) and the power
// iteration for an operator known only through host callbacks.  Each step is
// a few short kernels around the user's product; sums are formed per block in
// a fixed order and combined by one block in block order, so results do not
// depend on timing.  The stop / reject decisions are taken by that one block
// and written to device memory (read by the next step's kernels) and to a
// pinned status the host polls.
#include <hip/hip_runtime.h>

#include <cmath>

#include "device.hpp"
#include "user_kernels.hpp"

namespace lj {

namespace {

constexpr double kSqrtEpsMach = 1.4901161193847656e-08;  // sqrt(2^-52)

// Sum over the block of one value per thread, fixed order: wave sums, then
// thread 0 adds the wave sums in wave order.  Result valid in thread 0.
__device__ __forceinline__ double block_total(double v, double* red) {
  const double w = wave_sum(v);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = w;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  __syncthreads();
  return t;
}

// Sum of part[b * stride + q] over b < G in block order (thread 0's result);
// each thread first adds its own blocks b = t, t + 256, ... in order.
__device__ __forceinline__ double grid_total(const double* part, int G, int stride, int q, double* red) {
  double a = 0.0;
  for (int b = threadIdx.x; b < G; b += blockDim.x) a += part[(size_t)b * stride + q];
  return block_total(a, red);
}

template <int KIND, int NC>
__global__ __launch_bounds__(256) void lj_family_jv_kernel(OpDev op, const double* __restrict__ x,
                                                           double* __restrict__ y) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < op.npts; p += gridDim.x * blockDim.x) {
    double out[2], xc[2];
    jv_point<KIND, NC>(op, x, p, out, xc);
#pragma unroll
    for (int c = 0; c < NC; ++c) y[NC * p + c] = out[c];
  }
}

__global__ __launch_bounds__(kUserBlock) void lj_user_start_vector_kernel(double* x, long n, uint64_t seed) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    x[i] = 0.5 + splitmix_uniform(seed, (uint64_t)i);
}

__global__ __launch_bounds__(kUserBlock) void lj_user_sumsq_kernel(const double* __restrict__ x, long n,
                                                                  double* part) {
  __shared__ double red[kUserBlock / 64];
  double a = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    a += x[i] * x[i];
  const double t = block_total(a, red);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// what = 0: st->nu = ||x||; what = 1: st->eps from ||x||
__global__ __launch_bounds__(kUserBlock) void lj_user_norm_final_kernel(UserState* st, const double* part, int G,
                                                                       int what) {
  __shared__ double red[kUserBlock / 64];
  const double t = grid_total(part, G, 1, 0, red);
  if (threadIdx.x == 0) {
    const double nx = sqrt(t);
    if (what == 0) {
      st->nu = nx;
    } else {
      st->eps = nx > 0.0 ? kSqrtEpsMach * (1.0 + st->nu) / nx : 0.0;
    }
  }
}

__global__ __launch_bounds__(kUserBlock) void lj_user_fd_point_kernel(const UserState* st,
                                                                     const double* __restrict__ u,
                                                                     const double* __restrict__ x, long n,
                                                                     double* __restrict__ out) {
  const double eps = st->eps;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = u[i] + eps * x[i];
}

__device__ __forceinline__ double fd_quotient(double fx, double fu, double eps) {
  return eps != 0.0 ? (fx - fu) / eps : 0.0;
}

__global__ __launch_bounds__(kUserBlock) void lj_user_fd_quotient_kernel(const UserState* st,
                                                                        const double* __restrict__ fx,
                                                                        const double* __restrict__ fu, long n,
                                                                        double* __restrict__ out) {
  const double eps = st->eps;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    out[i] = fd_quotient(fx[i], fu[i], eps);
}

// ---- Newton recurrence -------------------------------------------------------

__device__ void copy_status(const UserState* st, UserStatus* h, int iters) {
  h->done = st->done;
  h->iters = iters;
  for (int k = 0; k < kMaxK; ++k) {
    h->state[k] = st->state[k];
    h->m_star[k] = st->m_star[k];
    h->err[k] = st->err[k];
  }
  h->nv = st->nv;
  h->lam = st->lam;
}

// p_k = d_{k,0} v; partial sums of v^2
__global__ __launch_bounds__(kUserBlock) void lj_user_rec_start_kernel(UserRec R, const double* __restrict__ v) {
  __shared__ double red[kUserBlock / 64];
  double a = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < R.n; i += (long)gridDim.x * blockDim.x) {
    const double x = v[i];
    a += x * x;
    for (int k = 0; k < R.K; ++k) R.p[k][i] = R.coef[k * kTable] * x;
  }
  const double t = block_total(a, red);
  if (threadIdx.x == 0) R.part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kUserBlock) void lj_user_rec_init_kernel(UserRec R, int G, int M, double tol,
                                                                     int relative, double hump, int fd) {
  __shared__ double red[kUserBlock / 64];
  const double t = grid_total(R.part, G, 1, 0, red);
  if (threadIdx.x == 0) {
    UserState* st = R.st;
    st->K = R.K;
    st->M = M;
    st->relative = relative;
    st->fd = fd;
    st->m = 0;
    st->tol = tol;
    st->hump = hump;
    st->nv = sqrt(t);
    // v = 0: every accumulator is exactly d_0 v = 0 with no Newton term
    const bool zero = !(st->nv > 0.0);
    for (int k = 0; k < kMaxK; ++k) {
      st->state[k] = (k < R.K) ? (zero ? ACC_CONVERGED : ACC_RUNNING) : ACC_CONVERGED;
      st->m_star[k] = (k < R.K && zero) ? 0 : -1;
      st->err[k] = 0.0;
    }
    st->done = zero ? 1 : 0;
    if (fd) st->eps = zero ? 0.0 : kSqrtEpsMach * (1.0 + st->nu) / st->nv;
    copy_status(st, R.host, 0);
  }
}

__global__ __launch_bounds__(kUserBlock) void lj_user_rec_step_kernel(UserRec R, int m, const double* __restrict__ jy,
                                                                     const double* __restrict__ fu,
                                                                     const double* __restrict__ yp,
                                                                     double* __restrict__ y, double c, double gamma,
                                                                     double rgamma, double xim) {
  __shared__ double red[kUserBlock / 64];
  const UserState* st = R.st;
  if (st->done) return;
  bool act[kMaxK];
  double d[kMaxK];
  for (int k = 0; k < kMaxK; ++k) {
    act[k] = k < R.K && st->state[k] == ACC_RUNNING;
    d[k] = act[k] ? R.coef[k * kTable + m] : 0.0;
  }
  const double eps = st->eps;
  double acc[1 + kMaxK] = {};
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < R.n; i += (long)gridDim.x * blockDim.x) {
    const double x = yp[i];
    const double jx = (fu != nullptr) ? fd_quotient(jy[i], fu[i], eps) : jy[i];
    const double yi = div_rn(jx - c * x, gamma, rgamma) - xim * x;
    y[i] = yi;
    acc[0] += yi * yi;
    for (int k = 0; k < R.K; ++k) {
      if (!act[k]) continue;
      const double pk = R.p[k][i] + d[k] * yi;
      R.p[k][i] = pk;
      acc[1 + k] += pk * pk;
    }
  }
  for (int q = 0; q <= R.K; ++q) {
    const double t = block_total(acc[q], red);
    if (threadIdx.x == 0) R.part[(size_t)blockIdx.x * (1 + kMaxK) + q] = t;
  }
}

// The Sec. 2.2 stop test and the rejection rules, in the order of the CPU
// reference: a non-finite term or norm, a term above hump ||v|| max|f|, then
// |d_m| ||y_m|| <= tol ||p|| (or <= tol, absolute).
__global__ __launch_bounds__(kUserBlock) void lj_user_rec_decide_kernel(UserRec R, int G, int m) {
  __shared__ double red[kUserBlock / 64];
  UserState* st = R.st;
  if (st->done) return;
  double tot[1 + kMaxK];
  for (int q = 0; q <= R.K; ++q) tot[q] = grid_total(R.part, G, 1 + kMaxK, q, red);
  if (threadIdx.x != 0) return;
  const double ny = sqrt(tot[0]);
  int running = 0;
  for (int k = 0; k < R.K; ++k) {
    if (st->state[k] != ACC_RUNNING) continue;
    const double e = fabs(R.coef[k * kTable + m]) * ny;
    const double np = sqrt(tot[1 + k]);
    if (!(isfinite(e) && isfinite(np))) {
      st->state[k] = ACC_NONFINITE;
    } else if (e > st->hump * st->nv * R.fmax[k]) {
      st->state[k] = ACC_HUMP;
    } else if (e <= (st->relative ? st->tol * np : st->tol)) {
      st->state[k] = ACC_CONVERGED;
      st->m_star[k] = m;
      st->err[k] = e;
    } else {
      st->err[k] = e;
      if (m >= st->M) {
        st->state[k] = ACC_MAXPTS;
      } else {
        ++running;
      }
    }
  }
  st->m = m;
  st->done = running == 0;
  if (st->fd) st->eps = ny > 0.0 ? kSqrtEpsMach * (1.0 + st->nu) / ny : 0.0;
  copy_status(st, R.host, m);
}

// ---- power iteration ---------------------------------------------------------

__global__ void lj_user_power_init_kernel(UserState* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st->done = 0;
    st->lam = 0.0;
    st->ny = 0.0;
  }
}

__global__ __launch_bounds__(kUserBlock) void lj_user_power_kernel(const UserState* st,
                                                                  const double* __restrict__ x,
                                                                  const double* __restrict__ src,
                                                                  const double* __restrict__ fu,
                                                                  double* __restrict__ y, long n, double* part) {
  __shared__ double red[kUserBlock / 64];
  if (st->done) return;
  const double eps = st->eps;
  double ax = 0.0, ay = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double xi = x[i];
    double yi;
    if (fu != nullptr) {
      yi = fd_quotient(src[i], fu[i], eps);
      y[i] = yi;
    } else {
      yi = src[i];
    }
    ax += xi * xi;
    ay += yi * yi;
  }
  const double tx = block_total(ax, red);
  const double ty = block_total(ay, red);
  if (threadIdx.x == 0) {
    part[2 * (size_t)blockIdx.x] = tx;
    part[2 * (size_t)blockIdx.x + 1] = ty;
  }
}

__global__ __launch_bounds__(kUserBlock) void lj_user_power_final_kernel(UserState* st, const double* part, int G,
                                                                        UserStatus* host) {
  __shared__ double red[kUserBlock / 64];
  if (st->done) return;
  const double tx = grid_total(part, G, 2, 0, red);
  const double ty = grid_total(part, G, 2, 1, red);
  if (threadIdx.x == 0) {
    const double nx = sqrt(tx), ny = sqrt(ty);
    st->ny = ny;
    if (ny == 0.0) {
      st->lam = 0.0;
      st->done = 1;
    } else {
      st->lam = ny / nx;
    }
    host->lam = st->lam;
  }
}

__global__ __launch_bounds__(kUserBlock) void lj_user_power_scale_kernel(const UserState* st,
                                                                        const double* __restrict__ y,
                                                                        double* __restrict__ xn, long n) {
  if (st->done) return;
  const double ny = st->ny;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    xn[i] = y[i] / ny;
}

}  // namespace

int user_grid(long n) {
  long g = (n + kUserBlock - 1) / kUserBlock;
  if (g > kUserBlocksMax) g = kUserBlocksMax;
  if (g < 1) g = 1;
  return (int)g;
}

hipError_t launch_family_jv(const OpDev& op, const double* x, double* y, hipStream_t s) {
  const int G = user_grid(op.npts);
  switch (op.kind) {
#define LJ_JV_CASE(K_, NC_)                                                                           \
  case K_:                                                                                            \
    hipLaunchKernelGGL((lj_family_jv_kernel<K_, NC_>), dim3(G), dim3(256), 0, s, op, x, y);          \
    break;
    LJ_JV_CASE(OP_DIAG, 1)
    LJ_JV_CASE(OP_ADVDIFF, 1)
    LJ_JV_CASE(OP_ALLENCAHN, 1)
    LJ_JV_CASE(OP_BRUSSELATOR, 2)
    LJ_JV_CASE(OP_BURGERS, 1)
    LJ_JV_CASE(OP_GRAYSCOTT, 2)
    LJ_JV_CASE(OP_ADR, 1)
#undef LJ_JV_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_user_start_vector(double* x, long n, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(lj_user_start_vector_kernel, dim3(user_grid(n)), dim3(kUserBlock), 0, s, x, n, seed);
  return hipGetLastError();
}

hipError_t launch_user_norm_u(UserState* st, const double* u, long n, double* part, hipStream_t s) {
  const int G = user_grid(n);
  hipLaunchKernelGGL(lj_user_sumsq_kernel, dim3(G), dim3(kUserBlock), 0, s, u, n, part);
  hipLaunchKernelGGL(lj_user_norm_final_kernel, dim3(1), dim3(kUserBlock), 0, s, st, part, G, 0);
  return hipGetLastError();
}

hipError_t launch_user_fd_step(UserState* st, const double* x, long n, double* part, hipStream_t s) {
  const int G = user_grid(n);
  hipLaunchKernelGGL(lj_user_sumsq_kernel, dim3(G), dim3(kUserBlock), 0, s, x, n, part);
  hipLaunchKernelGGL(lj_user_norm_final_kernel, dim3(1), dim3(kUserBlock), 0, s, st, part, G, 1);
  return hipGetLastError();
}

hipError_t launch_user_fd_point(const UserState* st, const double* u, const double* x, long n, double* out,
                                hipStream_t s) {
  hipLaunchKernelGGL(lj_user_fd_point_kernel, dim3(user_grid(n)), dim3(kUserBlock), 0, s, st, u, x, n, out);
  return hipGetLastError();
}

hipError_t launch_user_fd_quotient(const UserState* st, const double* fx, const double* fu, long n, double* out,
                                   hipStream_t s) {
  hipLaunchKernelGGL(lj_user_fd_quotient_kernel, dim3(user_grid(n)), dim3(kUserBlock), 0, s, st, fx, fu, n, out);
  return hipGetLastError();
}

hipError_t launch_user_rec_start(const UserRec& R, const double* v, int M, double tol, int relative, double hump,
                                 int fd, hipStream_t s) {
  const int G = user_grid(R.n);
  hipLaunchKernelGGL(lj_user_rec_start_kernel, dim3(G), dim3(kUserBlock), 0, s, R, v);
  hipLaunchKernelGGL(lj_user_rec_init_kernel, dim3(1), dim3(kUserBlock), 0, s, R, G, M, tol, relative, hump, fd);
  return hipGetLastError();
}

hipError_t launch_user_rec_step(const UserRec& R, int m, const double* jy, const double* fu, const double* y_prev,
                                double* y, double c, double gamma, double rgamma, double xim, hipStream_t s) {
  hipLaunchKernelGGL(lj_user_rec_step_kernel, dim3(user_grid(R.n)), dim3(kUserBlock), 0, s, R, m, jy, fu, y_prev,
                     y, c, gamma, rgamma, xim);
  return hipGetLastError();
}

hipError_t launch_user_rec_decide(const UserRec& R, int m, hipStream_t s) {
  hipLaunchKernelGGL(lj_user_rec_decide_kernel, dim3(1), dim3(kUserBlock), 0, s, R, user_grid(R.n), m);
  return hipGetLastError();
}

hipError_t launch_user_power_init(UserState* st, hipStream_t s) {
  hipLaunchKernelGGL(lj_user_power_init_kernel, dim3(1), dim3(64), 0, s, st);
  return hipGetLastError();
}

hipError_t launch_user_power(UserState* st, const double* x, const double* jy, const double* fu, double* y,
                             double* x_next, long n, double* part, UserStatus* host, hipStream_t s) {
  const int G = user_grid(n);
  hipLaunchKernelGGL(lj_user_power_kernel, dim3(G), dim3(kUserBlock), 0, s, st, x, jy, fu, y, n, part);
  hipLaunchKernelGGL(lj_user_power_final_kernel, dim3(1), dim3(kUserBlock), 0, s, st, part, G, host);
  hipLaunchKernelGGL(lj_user_power_scale_kernel, dim3(G), dim3(kUserBlock), 0, s, st, fu != nullptr ? y : jy,
                     x_next, n);
  return hipGetLastError();
}

}  // namespace lj
