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
// Stencils.  Sec. 3: centred second-order differences; the grids are periodic
// except for the Neumann families (family_neumann), whose boundary cells are
// their own ghost neighbours.
// Point p = j*nx + i; components of a two-component state are interleaved.
//
// stencil_jv evaluates (J x) at one point from values: x at the centre and the
// four neighbours (index 0 centre, 1 west, 2 east, 3 south, 4 north; NC
// components each) and the linearisation state at the same five places.  The
// global-memory kernels and the LDS-tiled kernel both call it, so both perform
// exactly the same arithmetic per point.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double lap5(const OpDev& op, double xc, double xw, double xe, double xs,
                                       double xn) {
  return (xw - 2.0 * xc + xe) * op.idx2 + (xs - 2.0 * xc + xn) * op.idy2;
}

template <int KIND>
__device__ __forceinline__ void stencil_jv(const OpDev& op, const double (&x)[5][2], const double (&u)[5][2],
                                           double out[2]) {
  if constexpr (KIND == OP_DIAG) {
    out[0] = u[0][0] * x[0][0];
  } else if constexpr (KIND == OP_ADVDIFF) {
    out[0] = op.c0 * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) -
             op.c1 * ((x[2][0] - x[1][0]) * op.i2dx) - op.c2 * ((x[4][0] - x[3][0]) * op.i2dy);
  } else if constexpr (KIND == OP_ALLENCAHN) {
    const double uc = u[0][0];
    out[0] = op.c0 * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) + (1.0 - 3.0 * uc * uc) * x[0][0];
  } else if constexpr (KIND == OP_BRUSSELATOR) {
    const double U = u[0][0], V = u[0][1];
    const double Du = op.c0, Dv = op.c1, b = op.c3;
    // d/du (a - (b+1)u + u^2 v) = -(b+1) + 2uv,  d/dv = u^2
    out[0] = Du * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) + (-(b + 1.0) + 2.0 * U * V) * x[0][0] +
             U * U * x[0][1];
    // d/du (b u - u^2 v) = b - 2uv,  d/dv = -u^2
    out[1] = Dv * lap5(op, x[0][1], x[1][1], x[2][1], x[3][1], x[4][1]) + (b - 2.0 * U * V) * x[0][0] -
             U * U * x[0][1];
  } else if constexpr (KIND == OP_GRAYSCOTT) {
    const double U = u[0][0], V = u[0][1];
    const double a1 = op.c0, a2 = op.c1, a = op.c2, b = op.c3;
    // d/du (-u v^2 + a(1 - u)) = -v^2 - a,  d/dv = -2uv
    out[0] = a1 * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) + (-(V * V) - a) * x[0][0] -
             2.0 * U * V * x[0][1];
    // d/du (u v^2 - (a + b) v) = v^2,  d/dv = 2uv - (a + b)
    out[1] = a2 * lap5(op, x[0][1], x[1][1], x[2][1], x[3][1], x[4][1]) + V * V * x[0][0] +
             (2.0 * U * V - (a + b)) * x[0][1];
  } else if constexpr (KIND == OP_ADR) {
    // alpha Lap x + beta (d_x + d_y) x + rate (-3u^2 + 3u - 1/2) x
    const double uc = u[0][0];
    out[0] = op.c0 * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) +
             op.c1 * ((x[2][0] - x[1][0]) * op.i2dx + (x[4][0] - x[3][0]) * op.i2dy) +
             op.c2 * (uc * (3.0 - 3.0 * uc) - 0.5) * x[0][0];
  } else {  // OP_BURGERS: nu Lap x - (d/dx + d/dy)(u x)
    const double qe = u[2][0] * x[2][0], qw = u[1][0] * x[1][0];
    const double qn = u[4][0] * x[4][0], qs = u[3][0] * x[3][0];
    out[0] = op.c0 * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) -
             ((qe - qw) * op.i2dx + (qn - qs) * op.i2dy);
  }
}

// which state values a family's Jacobian reads: none, the centre, or all five
template <int KIND>
struct StateUse {
  static constexpr int value = (KIND == OP_ADVDIFF) ? 0 : (KIND == OP_BURGERS ? 5 : 1);
};

struct Nbr {
  int c, w, e, s, n;  // flat point indices of centre and the four neighbours
};

template <int KIND>
__device__ __forceinline__ Nbr neighbours(const OpDev& op, int p) {
  const int nx = op.nx, ny = op.ny;
  const int j = p / nx;
  const int i = p - j * nx;
  constexpr bool neu = family_neumann(KIND);
  Nbr r;
  r.c = p;
  r.w = (i == 0) ? (neu ? p : p + nx - 1) : p - 1;
  r.e = (i == nx - 1) ? (neu ? p : p - nx + 1) : p + 1;
  r.s = (j == 0) ? (neu ? p : p + (ny - 1) * nx) : p - nx;
  r.n = (j == ny - 1) ? (neu ? p : p - (ny - 1) * nx) : p + nx;
  return r;
}

// Gathers what (J x)(p) needs from global memory: x at p and its four
// neighbours, and the state values the family reads (unused entries zero).
template <int KIND, int NC>
__device__ __forceinline__ void gather_point(const OpDev& op, const double* __restrict__ x, int p,
                                             double (&xv)[5][2], double (&uv)[5][2]) {
#pragma unroll
  for (int t = 0; t < 5; ++t) {
    xv[t][0] = xv[t][1] = 0.0;
    uv[t][0] = uv[t][1] = 0.0;
  }
  if constexpr (KIND == OP_DIAG) {
    xv[0][0] = x[p];
    uv[0][0] = op.state[p];
  } else {
    const Nbr q = neighbours<KIND>(op, p);
    const int idx[5] = {q.c, q.w, q.e, q.s, q.n};
#pragma unroll
    for (int t = 0; t < 5; ++t) {
#pragma unroll
      for (int c = 0; c < NC; ++c) xv[t][c] = x[NC * idx[t] + c];
    }
    constexpr int su = StateUse<KIND>::value;
#pragma unroll
    for (int t = 0; t < su; ++t) {
#pragma unroll
      for (int c = 0; c < NC; ++c) uv[t][c] = op.state[NC * idx[t] + c];
    }
  }
}

// (J x)(p) from global memory; xc[] receives x(p) (the recurrence needs it)
template <int KIND, int NC>
__device__ __forceinline__ void jv_point(const OpDev& op, const double* __restrict__ x, int p, double out[2],
                                         double xc[2]) {
  double xv[5][2], uv[5][2];
  gather_point<KIND, NC>(op, x, p, xv, uv);
  stencil_jv<KIND>(op, xv, uv, out);
#pragma unroll
  for (int c = 0; c < NC; ++c) xc[c] = xv[0][c];
}

// Right-hand side f(x) at one point from x at the centre and its four
// neighbours (index 0 centre, 1 west, 2 east, 3 south, 4 north), and for the
// diagonal family the diagonal entry there.
template <int KIND>
__device__ __forceinline__ void rhs_values(const OpDev& op, const double (&x)[5][2], double diag, double out[2]) {
  if constexpr (KIND == OP_DIAG) {
    out[0] = diag * x[0][0];
  } else if constexpr (KIND == OP_BRUSSELATOR) {
    const double Du = op.c0, Dv = op.c1, a = op.c2, b = op.c3;
    const double uuv = x[0][0] * x[0][0] * x[0][1];
    out[0] = Du * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) + a - (b + 1.0) * x[0][0] + uuv;
    out[1] = Dv * lap5(op, x[0][1], x[1][1], x[2][1], x[3][1], x[4][1]) + b * x[0][0] - uuv;
  } else if constexpr (KIND == OP_GRAYSCOTT) {
    const double a1 = op.c0, a2 = op.c1, a = op.c2, b = op.c3;
    const double uvv = x[0][0] * x[0][1] * x[0][1];
    out[0] = a1 * lap5(op, x[0][0], x[1][0], x[2][0], x[3][0], x[4][0]) - uvv + a * (1.0 - x[0][0]);
    out[1] = a2 * lap5(op, x[0][1], x[1][1], x[2][1], x[3][1], x[4][1]) + uvv - (a + b) * x[0][1];
  } else {
    const double c = x[0][0], w = x[1][0], e = x[2][0], s = x[3][0], n = x[4][0];
    if constexpr (KIND == OP_ADVDIFF) {
      out[0] = op.c0 * lap5(op, c, w, e, s, n) - op.c1 * ((e - w) * op.i2dx) - op.c2 * ((n - s) * op.i2dy);
    } else if constexpr (KIND == OP_ALLENCAHN) {
      out[0] = op.c0 * lap5(op, c, w, e, s, n) + c - c * c * c;
    } else if constexpr (KIND == OP_ADR) {
      out[0] = op.c0 * lap5(op, c, w, e, s, n) + op.c1 * ((e - w) * op.i2dx + (n - s) * op.i2dy) +
               op.c2 * (c * (1.0 - c) * (c - 0.5));
    } else {  // OP_BURGERS: nu Lap u - (1/2)(d/dx + d/dy)(u^2)
      out[0] = op.c0 * lap5(op, c, w, e, s, n) - 0.5 * ((e * e - w * w) * op.i2dx + (n * n - s * s) * op.i2dy);
    }
  }
}

// x at a point and its four neighbours (the diagonal family: the point only)
template <int KIND, int NC>
__device__ __forceinline__ void gather_x(const OpDev& op, const double* __restrict__ x, int p, double (&xv)[5][2]) {
#pragma unroll
  for (int t = 0; t < 5; ++t) xv[t][0] = xv[t][1] = 0.0;
  if constexpr (KIND == OP_DIAG) {
    xv[0][0] = x[p];
  } else {
    const Nbr q = neighbours<KIND>(op, p);
    const int idx[5] = {q.c, q.w, q.e, q.s, q.n};
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c) xv[t][c] = x[NC * idx[t] + c];
  }
}

// Right-hand side f(x)(p) of each family.
template <int KIND>
__device__ __forceinline__ void rhs_point(const OpDev& op, const double* __restrict__ x, int p,
                                          double out[2]) {
  constexpr int NC = family_ncomp(KIND);
  double xv[5][2];
  gather_x<KIND, NC>(op, x, p, xv);
  rhs_values<KIND>(op, xv, (KIND == OP_DIAG) ? op.state[p] : 0.0, out);
}

// ---------------------------------------------------------------------------
// t / den from r = 1/den (correctly rounded, formed once by a division):
// q = t r, then one correction by the exact FMA residual t - q den
// (Markstein 1990).  The result is the correctly rounded quotient, the value
// an IEEE division returns, at three FMA-unit instructions instead of the
// division's scaled Newton sequence; the CPU tests check the identity on
// random and near-boundary operands.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double div_rn(double t, double den, double r) {
  const double q = t * r;
  return fma(fma(-q, den, t), r, q);
}

// ---------------------------------------------------------------------------
// phi_l(z) in FP64 (Sec. 1 definition).  |z| <= 2: the Taylor series
// sum_{k<=40} z^k/(k+l)! by Horner (2^41/41! < 1e-37, far below one ulp), with
// the coefficients 1/(l+k)! formed at compile time by successive division;
// |z| > 2: the defining recurrence from exp(z), phi_{k+1} = (phi_k - 1/k!)/z,
// which only mildly amplifies rounding once |z| > 2.
// ---------------------------------------------------------------------------
template <int L>
struct InvFactorials {
  double v[41];  // v[k] = 1/(L+k)!
  constexpr InvFactorials() : v() {
    double f = 1.0;
    for (int k = 2; k <= L; ++k) f /= (double)k;
    v[0] = f;
    for (int k = 1; k <= 40; ++k) v[k] = v[k - 1] / (double)(L + k);
  }
};

template <int L>
__device__ __forceinline__ double phi_series(double z) {
  constexpr InvFactorials<L> c{};
  double s = c.v[40];
#pragma unroll
  for (int k = 39; k >= 0; --k) s = s * z + c.v[k];
  return s;
}

// l in [0, kMaxL]; the callers validate it.  phi_eval is the inline form:
// a call waits at its entry for every memory operation its caller has in
// flight, so a kernel that issued its input loads first and evaluates phi
// while they arrive takes this one; the others call phi_dev, out of line.
__device__ __forceinline__ double phi_eval(int l, double z) {
  if (fabs(z) <= 2.0) {
    switch (l) {
      case 0: return phi_series<0>(z);
      case 1: return phi_series<1>(z);
      case 2: return phi_series<2>(z);
      case 3: return phi_series<3>(z);
      default: return phi_series<4>(z);
    }
  }
  double p = exp(z);
  double invfact = 1.0;  // 1/k!
  for (int k = 0; k < l; ++k) {
    p = (p - invfact) / z;
    invfact /= (double)(k + 1);
  }
  return p;
}
__device__ __noinline__ double phi_dev(int l, double z) { return phi_eval(l, z); }

// ---------------------------------------------------------------------------
// Cross-lane moves and reductions on DPP (data-parallel primitives: lane
// permutations applied on the ALU's operand path, a few cycles each, instead
// of the LDS crossbar behind ds_bpermute).  All lanes of the wave must be
// active.  Fixed association order for a given launch shape, so every block
// that reduces the same data gets bit-identical totals.
// ---------------------------------------------------------------------------
template <int CTRL, int ROW_MASK = 0xf>
__device__ __forceinline__ double dpp_move(double v) {
  const int2 x = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_update_dpp(0, x.x, CTRL, ROW_MASK, 0xf, true);
  r.y = __builtin_amdgcn_update_dpp(0, x.y, CTRL, ROW_MASK, 0xf, true);
  return __builtin_bit_cast(double, r);  // lanes outside ROW_MASK or without a source: 0
}

__device__ __forceinline__ double read_lane(double v, int lane) {
  const int2 x = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readlane(x.x, lane);
  r.y = __builtin_amdgcn_readlane(x.y, lane);
  return __builtin_bit_cast(double, r);
}

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
  const int2 x = __builtin_bit_cast(int2, v);
  int2 r;
  r.x = __builtin_amdgcn_readfirstlane(x.x);
  r.y = __builtin_amdgcn_readfirstlane(x.y);
  return __builtin_bit_cast(double, r);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// the value held by lane (i - 1), for lane i > 0; lane 0 receives 0
__device__ __forceinline__ double wave_shift_up(double v) { return dpp_move<0x138>(v); }  // wave_shr:1

// Sum over the 64 lanes, returned in every lane: inclusive scans within each
// row of 16 lanes (row_shr 1, 2, 4, 8), then row 0 added into row 1 and row 2
// into row 3 (row_bcast:15), then rows 0-1 into rows 2-3 (row_bcast:31); lane
// 63 then holds the total.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<0x111>(v);
  v += dpp_move<0x112>(v);
  v += dpp_move<0x114>(v);
  v += dpp_move<0x118>(v);
  v += dpp_move<0x142, 0xa>(v);
  v += dpp_move<0x143, 0xc>(v);
  return read_lane(v, 63);
}

// Inclusive sums within each row of 16 lanes (row_shr 1, 2, 4, 8): lane 15 of
// a row then holds the sum of the row's 16 values.
__device__ __forceinline__ double row_sum(double v) {
  v += dpp_move<0x111>(v);
  v += dpp_move<0x112>(v);
  v += dpp_move<0x114>(v);
  v += dpp_move<0x118>(v);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Sum NV values per thread over the block; every thread's v[] holds the block
// totals after the call.  red (LDS) must hold NV * (blockDim.x/64 + 1)
// doubles: the wave sums, then the totals.
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
// Grid barrier with an all-reduce of per-block partial sums, for a
// cooperatively launched (co-resident) grid.
//
// Everything one block writes for another block to read inside a launch (the
// Newton basis vectors, halo rows, partial sums) is stored with device-scope
// stores (store_shared), which write through the XCD's L2 to the device's
// coherence point.  So a barrier needs no L2 write-back: each block drains its
// stores (s_waitcnt), and an acquire after the barrier drops the CU's and the
// L2's stale lines before the block reads what the others wrote.  (A release
// per block would write back the whole L2 of its XCD, serialised per XCD.)
// Arrival is two-level to spread the atomic traffic: block b belongs to group
// g = b % 8 (workgroups are dispatched round-robin over the 8 XCDs, so a group
// is one XCD); the group's last arrival arrives on the global counter, waits
// for all groups and raises the group's flag, on which the others wait.
//
// Counters are monotonic (barrier e completes at e arrivals per member), so no
// reset is needed inside a launch; the layout (128-byte spaced words) is
//   base[0]            global counter
//   base[32*(1+g)]     group g arrival counter
//   base[32*(9+g)]     group g release flag (holds the last completed epoch)
//   base[32*17]        exit counter (grid_exit)
//   base[32*18]        abort word (see wait_at_least)
// Everything must be zero at launch; grid_exit leaves it zero again.
//
// Partial sums: two areas alternate by epoch parity, each kPartStride x
// gridDim.x doubles, slot-major (slot q of block b at [q * gridDim.x + b]).
// After the barrier every block adds slot q over the blocks in the same fixed
// order (lane t takes blocks t, t + 64, ..., then the wave sums its lanes), so
// all blocks obtain bit-identical totals.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_shared(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double* partial_area(double* partials, unsigned int epoch) {
  return partials + (size_t)(epoch & 1u) * kPartStride * gridDim.x;
}

// where this block stores slot q of a partial-sum area
__device__ __forceinline__ double* my_partial(double* area, int q) { return area + (size_t)q * gridDim.x + blockIdx.x; }

__device__ __forceinline__ void put_partial(double* p, double v) { store_shared(p, v); }

struct NoOverlap {
  __device__ void operator()() const {}
};

// Waits until *word >= target.  The wait is bounded: the host launches a grid
// without the cooperative guarantee only when all its blocks fit on the
// device at once, but should some block never arrive, the waiter raises the
// abort word after kGridSpinLimit polls, every later wait returns at once, the
// launch runs to its end, and the host sees the abort in the status and
// relaunches cooperatively.  Returns false on abort.

__device__ __forceinline__ bool wait_at_least(unsigned int* word, unsigned int target, unsigned int* abort_word,
                                              unsigned int spin_limit) {
  unsigned int spins = 0;
  while (__hip_atomic_load(word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
    if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return false;
    if (++spins > spin_limit) {
      __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

__device__ __forceinline__ unsigned int grid_aborted(unsigned int* base) {
  return __hip_atomic_load(base + 32 * 18, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// `epoch` counts the barriers this block has passed; every thread of the block
// advances its copy (callers pick the partial-sum area with it before the
// call).  nq slots (nq <= kPartStride) of `area` are reduced into tot[0..nq)
// (LDS); nq = 0 makes it a plain barrier.  The barrier itself is run by the
// first lane of the block's last wave; meanwhile the other waves run `overlap`
// (work that touches no global memory another block writes before this
// barrier).  Right after the barrier every thread runs `prefetch`, which may
// issue loads of data the other blocks wrote before it (their latency then
// overlaps that of the partial sums').  Each wave issues the loads of all its
// rows of partials before summing any, so the reduction costs one memory
// round trip.
// The barrier state and the bound on each wait (kGridSpinLimit; a host may
// pass a smaller one to force the abort path).
struct GridSync {
  unsigned int* base;
  unsigned int spin_limit;
};

template <class Overlap = NoOverlap, class Prefetch = NoOverlap>
__device__ __forceinline__ void grid_allreduce(const GridSync& gs, unsigned int& epoch, double* area, int nq,
                                               double* tot, Overlap&& overlap = Overlap{},
                                               Prefetch&& prefetch = Prefetch{}) {
  unsigned int* base = gs.base;
  __builtin_amdgcn_s_waitcnt(0);  // this thread's loads and stores have completed
  __syncthreads();
  epoch += 1u;
  const unsigned int agent = blockDim.x - 64u;
  if (threadIdx.x == agent) {
    const unsigned int G = gridDim.x;
    const unsigned int ng = G < 8u ? G : 8u;
    const unsigned int g = blockIdx.x % ng;
    const unsigned int gsize = (G - g + ng - 1u) / ng;
    unsigned int* gc = base + 32 * (1 + g);
    unsigned int* gf = base + 32 * (9 + g);
    unsigned int* abort_word = base + 32 * 18;
    const unsigned int old = __hip_atomic_fetch_add(gc, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == epoch * gsize - 1u) {
      __hip_atomic_fetch_add(base, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      (void)wait_at_least(base, epoch * ng, abort_word, gs.spin_limit);
      __hip_atomic_store(gf, epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      (void)wait_at_least(gf, epoch, abort_word, gs.spin_limit);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  } else if (threadIdx.x < agent) {
    overlap();
  }
  __syncthreads();
  prefetch();
  if (nq > 0) {
    // slot q: lane t adds blocks t, t + 64, t + 128, ... in that order, then
    // the wave sums its lanes (zeros stand in for absent blocks; the sums are
    // of squares, never -0, so adding +0 changes nothing)
    const int G = gridDim.x;
    const int lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    const int w = threadIdx.x >> 6;
    if (G <= 256 && nq <= 3 * nw) {
      double v[3][4];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int q = w + r * nw;
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int b = lane + 64 * c;
          v[r][c] = (q < nq && b < G) ? area[(size_t)q * G + b] : 0.0;
        }
      }
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int q = w + r * nw;
        if (q >= nq) break;
        double a = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c) a += v[r][c];
        const double t = wave_sum(a);
        if (lane == 0) tot[q] = t;
      }
    } else {
      for (int q = w; q < nq; q += nw) {
        const double* __restrict__ row = area + (size_t)q * G;
        double a = 0.0;
        for (int b = lane; b < G; b += 64) a += row[b];
        const double t = wave_sum(a);
        if (lane == 0) tot[q] = t;
      }
    }
    __syncthreads();
  }
}

__device__ __forceinline__ void grid_barrier(const GridSync& gs, unsigned int& epoch) {
  grid_allreduce(gs, epoch, nullptr, 0, nullptr);
}

// Call once per block after its last grid_barrier.  The last block to arrive
// here knows every block has left every barrier wait, so it can zero the
// barrier words for the next launch on the stream.
__device__ __forceinline__ void grid_exit(unsigned int* base) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned int old = __hip_atomic_fetch_add(base + 32 * 17, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old == gridDim.x - 1u) {
      for (int i = 0; i < 19; ++i) __hip_atomic_store(base + 32 * i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
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
