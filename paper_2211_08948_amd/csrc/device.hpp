// Device-side building blocks of the Leja phi-action library (gfx950, wave64):
// operator stencils J(u)v and f(u), the scalar phi_l(z), wave/block
// reductions in a fixed order, and the grid-wide barrier of the persistent
// kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.hpp"

namespace lj {

// ---------------------------------------------------------------------------
// Stencils.  Sec. 3: centred second-order differences; the grids are periodic.
// Point p = j*nx + i; components of a two-component state are interleaved.
// jv_point returns (J x)(p) for every component in out[] and the centre values
// x(p) in xc[] (the Newton recurrence needs both).
// ---------------------------------------------------------------------------
struct Nbr {
  int c, w, e, s, n;  // flat point indices of centre and the four neighbours
};

__device__ __forceinline__ Nbr neighbours(const OpDev& op, int p) {
  const int nx = op.nx, ny = op.ny;
  const int j = p / nx;
  const int i = p - j * nx;
  Nbr r;
  r.c = p;
  r.w = (i == 0) ? p + nx - 1 : p - 1;
  r.e = (i == nx - 1) ? p - nx + 1 : p + 1;
  r.s = (j == 0) ? p + (ny - 1) * nx : p - nx;
  r.n = (j == ny - 1) ? p - (ny - 1) * nx : p + nx;
  return r;
}

// (Lap x)(p) from centre/neighbour values
__device__ __forceinline__ double lap5(const OpDev& op, double xc, double xw, double xe, double xs,
                                       double xn) {
  return (xw - 2.0 * xc + xe) * op.idx2 + (xs - 2.0 * xc + xn) * op.idy2;
}

template <int KIND>
__device__ __forceinline__ void jv_point(const OpDev& op, const double* __restrict__ x, int p,
                                         double out[2], double xc[2]) {
  if constexpr (KIND == OP_DIAG) {
    xc[0] = x[p];
    out[0] = op.state[p] * xc[0];
  } else if constexpr (KIND == OP_BRUSSELATOR) {
    const Nbr q = neighbours(op, p);
    const double2 C = *reinterpret_cast<const double2*>(x + 2 * q.c);
    const double2 W = *reinterpret_cast<const double2*>(x + 2 * q.w);
    const double2 E = *reinterpret_cast<const double2*>(x + 2 * q.e);
    const double2 S = *reinterpret_cast<const double2*>(x + 2 * q.s);
    const double2 N = *reinterpret_cast<const double2*>(x + 2 * q.n);
    const double2 st = *reinterpret_cast<const double2*>(op.state + 2 * q.c);
    const double U = st.x, V = st.y;
    const double Du = op.c0, Dv = op.c1, b = op.c3;
    xc[0] = C.x;
    xc[1] = C.y;
    // d/du (a - (b+1)u + u^2 v) = -(b+1) + 2uv,  d/dv = u^2
    out[0] = Du * lap5(op, C.x, W.x, E.x, S.x, N.x) + (-(b + 1.0) + 2.0 * U * V) * C.x + U * U * C.y;
    // d/du (b u - u^2 v) = b - 2uv,  d/dv = -u^2
    out[1] = Dv * lap5(op, C.y, W.y, E.y, S.y, N.y) + (b - 2.0 * U * V) * C.x - U * U * C.y;
  } else {
    const Nbr q = neighbours(op, p);
    const double c = x[q.c], w = x[q.w], e = x[q.e], s = x[q.s], n = x[q.n];
    xc[0] = c;
    if constexpr (KIND == OP_ADVDIFF) {
      out[0] = op.c0 * lap5(op, c, w, e, s, n) - op.c1 * ((e - w) * op.i2dx) - op.c2 * ((n - s) * op.i2dy);
    } else if constexpr (KIND == OP_ALLENCAHN) {
      const double u = op.state[q.c];
      out[0] = op.c0 * lap5(op, c, w, e, s, n) + (1.0 - 3.0 * u * u) * c;
    } else {  // OP_BURGERS: nu Lap x - (d/dx + d/dy)(u x)
      const double* __restrict__ u = op.state;
      const double qe = u[q.e] * e, qw = u[q.w] * w, qn = u[q.n] * n, qs = u[q.s] * s;
      out[0] = op.c0 * lap5(op, c, w, e, s, n) - ((qe - qw) * op.i2dx + (qn - qs) * op.i2dy);
    }
  }
}

// Right-hand side f(x)(p) of each family.
template <int KIND>
__device__ __forceinline__ void rhs_point(const OpDev& op, const double* __restrict__ x, int p,
                                          double out[2]) {
  if constexpr (KIND == OP_DIAG) {
    out[0] = op.state[p] * x[p];
  } else if constexpr (KIND == OP_BRUSSELATOR) {
    const Nbr q = neighbours(op, p);
    const double2 C = *reinterpret_cast<const double2*>(x + 2 * q.c);
    const double2 W = *reinterpret_cast<const double2*>(x + 2 * q.w);
    const double2 E = *reinterpret_cast<const double2*>(x + 2 * q.e);
    const double2 S = *reinterpret_cast<const double2*>(x + 2 * q.s);
    const double2 N = *reinterpret_cast<const double2*>(x + 2 * q.n);
    const double Du = op.c0, Dv = op.c1, a = op.c2, b = op.c3;
    const double uuv = C.x * C.x * C.y;
    out[0] = Du * lap5(op, C.x, W.x, E.x, S.x, N.x) + a - (b + 1.0) * C.x + uuv;
    out[1] = Dv * lap5(op, C.y, W.y, E.y, S.y, N.y) + b * C.x - uuv;
  } else {
    const Nbr q = neighbours(op, p);
    const double c = x[q.c], w = x[q.w], e = x[q.e], s = x[q.s], n = x[q.n];
    if constexpr (KIND == OP_ADVDIFF) {
      out[0] = op.c0 * lap5(op, c, w, e, s, n) - op.c1 * ((e - w) * op.i2dx) - op.c2 * ((n - s) * op.i2dy);
    } else if constexpr (KIND == OP_ALLENCAHN) {
      out[0] = op.c0 * lap5(op, c, w, e, s, n) + c - c * c * c;
    } else {  // OP_BURGERS: nu Lap u - (1/2)(d/dx + d/dy)(u^2)
      out[0] = op.c0 * lap5(op, c, w, e, s, n) - 0.5 * ((e * e - w * w) * op.i2dx + (n * n - s * s) * op.i2dy);
    }
  }
}

// ---------------------------------------------------------------------------
// phi_l(z) in FP64 (Sec. 1 definition).  |z| <= 2: Taylor series
// sum_{k<=40} z^k/(k+l)! by Horner (2^41/41! < 1e-37, far below one ulp);
// |z| > 2: the defining recurrence from exp(z), phi_{k+1} = (phi_k - 1/k!)/z,
// which only mildly amplifies rounding once |z| > 2.
// ---------------------------------------------------------------------------
__device__ inline double phi_dev(int l, double z) {
  if (fabs(z) <= 2.0) {
    // 1/(l+k)! for k = 0..40 via successive division from 1/l!
    double inv[41];
    double f = 1.0;
    for (int k = 2; k <= l; ++k) f /= (double)k;
    inv[0] = f;
    for (int k = 1; k <= 40; ++k) inv[k] = inv[k - 1] / (double)(l + k);
    double s = inv[40];
    for (int k = 39; k >= 0; --k) s = s * z + inv[k];
    return s;
  }
  double p = exp(z);
  double invfact = 1.0;  // 1/k!
  for (int k = 0; k < l; ++k) {
    p = (p - invfact) / z;
    invfact /= (double)(k + 1);
  }
  return p;
}

// ---------------------------------------------------------------------------
// Reductions.  Fixed association order for a given launch shape, so every
// block that reduces the same data gets bit-identical totals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
  // butterfly over the 64 lanes; lane 0's value is the canonical result
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Sum NV values per thread over the block; result valid in red[0..NV) (LDS)
// after the call for all threads.  red must hold NV * (blockDim.x/64) doubles.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    const double s = wave_sum(v[q]);
    if (lane == 0) red[q * nw + wid] = s;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t += red[threadIdx.x * nw + w];
    red[NV * nw + threadIdx.x] = t;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = red[NV * nw + q];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Grid barrier of a cooperatively launched (co-resident) grid, two-level to
// match the chip: workgroups are dispatched round-robin over the XCDs, so
// block b belongs to group b % 8 (one group per XCD).  Each block first drains
// its own memory operations (its stores are then in its XCD's L2), arrives on
// its group counter, and only the group's last arrival publishes the whole
// XCD's L2 with one agent-scope release, arrives on the global counter and
// waits for all groups.  Every block ends with an agent-scope acquire.  A
// per-block release on a flat counter costs one L2 write-back per block,
// serialised per XCD, which dominated at hundreds of blocks.
//
// Counters are monotonic (barrier e completes at e arrivals per member), so no
// reset is needed inside a launch; the layout (128-byte spaced words) is
//   base[0]            global counter
//   base[32*(1+g)]     group g arrival counter
//   base[32*(9+g)]     group g release flag (holds the last completed epoch)
// and everything must be zero at launch (kBarrierWords words).
// ---------------------------------------------------------------------------

__device__ __forceinline__ void grid_barrier(unsigned int* base, unsigned int& epoch) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's loads and stores have completed
  __syncthreads();
  if (threadIdx.x == 0) {
    epoch += 1u;
    const unsigned int G = gridDim.x;
    const unsigned int ng = G < 8u ? G : 8u;
    const unsigned int g = blockIdx.x % ng;
    const unsigned int gsize = (G - g + ng - 1u) / ng;
    unsigned int* gc = base + 32 * (1 + g);
    unsigned int* gf = base + 32 * (9 + g);
    const unsigned int old = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == epoch * gsize - 1u) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(base, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (__hip_atomic_load(base, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch * ng) {
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(gf, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      while (__hip_atomic_load(gf, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
  }
  __syncthreads();
}

// SplitMix64 (Steele, Lea, Flood 2014): output number i of the stream seeded
// with `seed`, mapped to [0, 1) with 53 bits.
__device__ __host__ __forceinline__ double splitmix_uniform(uint64_t seed, uint64_t i) {
  uint64_t z = seed + (i + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * 0x1.0p-53;
}

}  // namespace lj
