// Kernels of the Leja phi-action library for gfx950 (CDNA4, wave64).
//
// One phi-action is one persistent, cooperatively launched kernel that runs
//   (1) the power-iteration spectral bound (Sec. 2.2), unless a bound is given,
//   (2) phi_l at the scaled Leja nodes and the Newton divided differences
//       (Sec. 2.2), redundantly in every block, one wave per accumulator,
//   (3) the Newton recurrence y_m = ((J - c)/gamma - xi_{m-1}) y_{m-1},
//       p_k += d_{k,m} y_m for K accumulators sharing y_m (Sec. 2.2 display,
//       vertical form of Sec. 4), with the stop/reject test on FP64 norms.
// Two shapes of the same computation:
//   * lj_action_stream: every Newton step is a pass over the vectors in HBM
//     (any grid size); one grid barrier per step carries the norm partials;
//   * lj_action_tile: each block keeps one tile of the grid plus an S-wide
//     halo in LDS and runs S steps between grid barriers (temporal blocking):
//     step j recomputes the halo ring that step j+1 needs, so the only global
//     traffic per S steps is one halo exchange and the norm partials.  The
//     S basis values of the block's own points stay in registers; after the
//     barrier every block replays the stop decisions of those S steps from the
//     reduced norms and commits each accumulator's terms up to its own stop
//     index, so the result is the untiled recurrence's, term for term.
// All arithmetic is FP64 on the vector ALU: the path is bandwidth/latency
// bound and has no dense contraction, so no MFMA is used.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "kernels.hpp"

namespace lj {

constexpr int kBlock = 1024;  // threads per block of the persistent kernels (one block per CU)
constexpr int kWaves = kBlock / 64;
constexpr int kQ = 1 + kMaxK;  // reduced values per Newton step: ||y||^2 and K ||p_k||^2

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a run of
// consecutive chunks / tiles so that neighbouring work shares an L2.
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

// ---------------------------------------------------------------------------
// Divided differences of phi_{l_k}(s_k (c + gamma xi_j)), j < n, for K
// accumulators: wave k computes accumulator k, lane t holding nodes t and t+64.
// Order by order, d_j <- (d_j - d_{j-1}) / (xi_j - xi_{j-order}) for j >= order
// (the standard table, Sec. 2.2), with d_{j-1} taken from the neighbouring
// lane by a DPP wave shift.  The quotient is div_rn (reciprocal + one
// Markstein correction), the same value a division gives.  The reciprocals do
// not depend on d, so those of the next order are formed while the current
// order's chain runs.
//
// After `order` orders the entries d_0..d_order are final, so the table can be
// advanced lazily: the Newton step m needs d_m only, and the action kernels
// advance it a few orders at a time while their blocks wait at a grid
// barrier.  The state lives in the registers of waves 0..K-1.  The nodes
// 64..100 are needed only by recurrences longer than 64 terms, so their half
// of the column lags: it catches up (same operations, same values) once an
// entry there is asked for, taking node 63's value after each order from h63.
// ---------------------------------------------------------------------------
struct DivDiff {
  double d0, d1;  // current column at nodes j0 = lane (after `order` orders), j1 = lane + 64 (after `order1`)
  double h63;     // lane k (k <= 63): d_63 after order k
  int order;      // orders done
  int order1;     // orders done on the nodes j1
  int n;          // nodes
};

// phi values at the nodes, fmax[k] = max_j |f_j|, coef[k * kTable] = d_0.
// Called by every thread; waves >= K do nothing.
__device__ void dd_init(DivDiff& D, int K, const int* l, const double* s, int n, double c, double gamma,
                        const double* xi, double* coef, double* fmax_out) {
#pragma clang fp contract(off)
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  D.order = 0;
  D.order1 = 0;
  D.n = n;
  D.d0 = 0.0;
  D.d1 = 0.0;
  D.h63 = 0.0;
  if (wid >= K) return;
  const int lk = l[wid];
  const double sk = s[wid];
  const int j0 = lane, j1 = lane + 64;
  const double x0 = xi[j0];
  const double x1 = (j1 < kTable) ? xi[j1] : 0.0;
  if (j0 < n) D.d0 = phi_dev(lk, sk * (c + gamma * x0));
  if (j1 < n) D.d1 = phi_dev(lk, sk * (c + gamma * x1));
  D.h63 = read_lane(D.d0, 63);
  const double m = wave_max(fmax(fabs(D.d0), fabs(D.d1)));
  if (lane == 0) {
    fmax_out[wid] = m;
    coef[wid * kTable] = D.d0;
  }
}

// dd_init with the phi values computed by every thread of the block (one
// (accumulator, node) pair per thread and round, staged in coef), then taken
// by the wave that owns the accumulator's table: the same values, in a
// fraction of the time one wave needs for all of them.  Called by every
// thread; ends with a block barrier.  phi is inline here: the register-tiled
// kernels' loads of v, issued at launch, stay in flight meanwhile.
__device__ void dd_init_par(DivDiff& D, int K, const int* l, const double* s, int n, double c, double gamma,
                            const double* xi, double* coef, double* fmax_out) {
#pragma clang fp contract(off)
  for (int t = threadIdx.x; t < K * kTable; t += blockDim.x) {
    const int k = t / kTable, j = t - k * kTable;
    if (j < n) coef[t] = phi_eval(l[k], s[k] * (c + gamma * xi[j]));
  }
  __syncthreads();
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  D.order = 0;
  D.order1 = 0;
  D.n = n;
  D.d0 = 0.0;
  D.d1 = 0.0;
  D.h63 = 0.0;
  if (wid < K) {
    const int j0 = lane, j1 = lane + 64;
    if (j0 < n) D.d0 = coef[wid * kTable + j0];
    if (j1 < n && j1 < kTable) D.d1 = coef[wid * kTable + j1];
    D.h63 = read_lane(D.d0, 63);
    const double m = wave_max(fmax(fabs(D.d0), fabs(D.d1)));
    if (lane == 0) fmax_out[wid] = m;
  }
  __syncthreads();
}

// Orders up to min(upto, n - 1); writes the entries that became final.
__device__ void dd_advance(DivDiff& D, int K, int upto, const double* xi, double* coef) {
#pragma clang fp contract(off)
  const int wid = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  if (wid >= K) return;
  const int n = D.n;
  const int last = min(upto, n - 1);
  if (last <= D.order) return;
  const int j0 = lane, j1 = lane + 64;
  // nodes 0..63: an order k changes the entries j >= k only, so orders up to
  // min(last, 63).  The next order's denominator comes from the nodes moved
  // up one lane (DPP), and its reciprocal forms while this order's chain runs.
  const int first = D.order + 1;
  const int last0 = min(last, 63);
  if (first <= last0) {
    const double x0 = xi[j0];
    double d0 = D.d0, h63 = D.h63;
    double xs0 = xi[max(j0 - first, 0)];  // node j0 - order (lanes j0 >= order)
    double den0 = (j0 >= first && j0 < n) ? x0 - xs0 : 1.0;
    double r0 = 1.0 / den0;
    for (int order = first; order <= last0; ++order) {
      xs0 = wave_shift_up(xs0);
      const double nden0 = (j0 >= order + 1 && j0 < n) ? x0 - xs0 : 1.0;
      const double nr0 = 1.0 / nden0;
      const double p0 = wave_shift_up(d0);
      const double q0 = div_rn(d0 - p0, den0, r0);
      if (j0 >= order && j0 < n) d0 = q0;
      const double t63 = read_lane(d0, 63);
      if (lane == order) h63 = t63;
      den0 = nden0;
      r0 = nr0;
    }
    D.d0 = d0;
    D.h63 = h63;
    if (j0 >= first && j0 <= last0) coef[wid * kTable + j0] = d0;
  }
  // nodes 64..100, once an entry there is asked for: the orders they missed,
  // with node 63's value after order k - 1 (constant from order 63 on)
  if (last >= 64) {
    const int f1 = D.order1 + 1;
    const double x1 = (j1 < kTable) ? xi[j1] : 0.0;
    double d1 = D.d1;
    for (int order = f1; order <= last; ++order) {
      const double xb = xi[min(max(j1 - order, 0), kTable - 1)];
      const double den1 = (j1 >= order && j1 < n) ? x1 - xb : 1.0;
      double p1 = wave_shift_up(d1);
      const double left = read_lane(D.h63, min(order - 1, 63));
      if (lane == 0) p1 = left;
      const double q1 = div_rn(d1 - p1, den1, 1.0 / den1);
      if (j1 >= order && j1 < n) d1 = q1;
    }
    D.d1 = d1;
    D.order1 = last;
    if (j1 >= f1 && j1 <= last) coef[wid * kTable + j1] = d1;
  }
  D.order = last;
}

// The interval of Sec. 2.2: alpha = -safety * lambda, beta = 0, c the midpoint,
// gamma a quarter of the length.
__device__ __forceinline__ void interval(double lam, double safety, double& c, double& gamma) {
#pragma clang fp contract(off)
  const double alpha = -safety * lam;
  const double beta = 0.0;
  c = 0.5 * (alpha + beta);
  gamma = 0.25 * (beta - alpha);
}

// ---------------------------------------------------------------------------
// Stop / reject decision of one Newton step m (identical in every block):
// accumulator k freezes at the first m with |d_{k,m}| ||y_m|| <= tol ||p_k||
// (or <= tol in the absolute form); it is rejected when that term exceeds
// hump_max ||v|| max|f_k|, when a value is not finite, or at max_points.
// ---------------------------------------------------------------------------
struct Decision {
  int st[kMaxK];
  int mst[kMaxK];
  double err[kMaxK];
  double hump[kMaxK];
  int n_active;
  int iters;
  int accum_iters;
  int next;  // predicted steps to the last stop (a length for the next super-step)
  int next_local;  // the same from the decay over the super-step's last four steps
};

__device__ __forceinline__ void decision_init(Decision& D, int K, double nv, double hump_max, const double* fmaxk) {
  D.n_active = 0;
  D.iters = 0;
  D.accum_iters = 0;
  D.next = kMaxPoints;
  D.next_local = kMaxPoints;
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    D.st[k] = (k < K) ? ACC_RUNNING : ACC_CONVERGED;
    D.mst[k] = -1;
    D.err[k] = 0.0;
    D.hump[k] = (k < K) ? hump_max * nv * fmaxk[k] : 0.0;
    if (k < K) ++D.n_active;
  }
  if (nv == 0.0) {  // v = 0: every phi_l(hJ) v is 0, no term is needed
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      D.st[k] = ACC_CONVERGED;
      D.mst[k] = (k < K) ? 0 : -1;
    }
    D.n_active = 0;
  }
}

// Stop decisions of the steps m0+1 .. m0+steps of one super-step, from the
// reduced totals tot[(j-1)*Q + q] of step m0+j (Q = 1 + K: ||y||^2, then
// ||p_k||^2 after the term), taken by the lanes of one
// wave in parallel over (step, accumulator).  An accumulator's test at a step
// depends only on its own state, which does not change until it stops, so its
// stopping step is the lowest one whose test does not continue, exactly as if
// the steps were decided one after another.  D is in LDS; commit[k]
// (LDS) receives how many of the super-step's terms accumulator k adds; trace
// (optional) receives the totals of the steps that were decided.  Called by
// all 64 lanes of one wave, with steps <= 16.
__device__ void replay_decisions(Decision& D, int K, int m0, int steps, int Q, const double* tot, const double* coef,
                                 double tol, int relative, int max_points, int* commit,
                                 double (*trace)[1 + kMaxK]) {
  const int lane = threadIdx.x & 63;
  const int j = lane >> 2, k = lane & 3;  // step m0 + j + 1, accumulator k
  const int m = m0 + j + 1;
  const bool run0 = (k < K) && (D.st[k] == ACC_RUNNING);
  int oc = ACC_RUNNING;
  double e = 0.0;
  if (run0 && j < steps) {
    const double ny = sqrt(tot[j * Q]);
    e = fabs(coef[k * kTable + m]) * ny;
    const double np = sqrt(tot[j * Q + 1 + k]);
    if (!(isfinite(e) && isfinite(np))) {
      oc = ACC_NONFINITE;
    } else if (e > D.hump[k]) {
      oc = ACC_HUMP;
    } else if (e <= (relative ? tol * np : tol)) {
      oc = ACC_CONVERGED;
    } else if (m == max_points) {
      oc = ACC_MAXPTS;
    }
  }
  const unsigned long long stop = __ballot(oc != ACC_RUNNING);
  const unsigned long long mine = stop & (0x1111111111111111ull << k);
  const int first = mine ? (int)__builtin_ctzll(mine) : -1;  // lane of the stopping step
  const int src = first >= 0 ? first : lane;
  const int oc_f = __shfl(oc, src, 64);
  const double e_f = __shfl(e, src, 64);
  const int cm = run0 ? (first >= 0 ? (first >> 2) + 1 : steps) : 0;
  const bool still = run0 && first < 0;
  const unsigned long long alive = __ballot(lane < kMaxK && still);
  const int c0 = __builtin_amdgcn_readlane(cm, 0), c1 = __builtin_amdgcn_readlane(cm, 1);
  const int c2 = __builtin_amdgcn_readlane(cm, 2), c3 = __builtin_amdgcn_readlane(cm, 3);
  const int cmax = max(max(c0, c1), max(c2, c3));
  if (lane < kMaxK) {
    commit[k] = cm;
    if (run0 && first >= 0) {
      D.st[k] = oc_f;
      if (oc_f == ACC_CONVERGED) {
        D.mst[k] = m0 + (first >> 2) + 1;
        D.err[k] = e_f;
      }
    }
  }
  // How many more steps the accumulators still running are likely to need:
  // each extrapolates the decay of its ratio e / (stop threshold) over this
  // batch of steps geometrically, plus one step of margin.  Only the length
  // of the next batch of speculative steps depends on it, never a decision.
  // (single precision suffices for a length; the same inputs give the same
  // length in every block)
  // The decay usually steepens as the expansion converges, so the rate over
  // the last four steps alone often predicts a shorter (and closer)
  // remainder; the register-tiled kernels take the smaller of the two (on
  // the 512^2 bench step it saves more overshooting steps than the extra
  // super-steps it causes cost), the LDS-tiled one the whole-batch rate.
  int need = 0, need_loc = 0;
  {
    float lq = 0.0f;
    if (run0 && j < steps && oc == ACC_RUNNING) {
      const double thr = relative ? tol * sqrt(tot[j * Q + 1 + k]) : tol;
      lq = __log2f((float)e) - __log2f((float)thr);
    }
    const float l_first = lq;  // lanes k < 4 hold step m0 + 1 of accumulator k themselves
    const float l_last = __shfl(lq, 4 * max(steps - 1, 0) + k, 64);
    const int w = min(4, steps - 1);
    const float l_mid = __shfl(lq, 4 * max(steps - 1 - w, 0) + k, 64);
    auto extrapolate = [&](float rate) {
      const int n = (rate > 0.0f && l_last < 64.0f * rate) ? (int)ceilf(l_last / rate) + 1 : kMaxPoints;
      return max(n, 1);
    };
    if (lane < kMaxK && still) {
      need = extrapolate((steps > 1) ? (l_first - l_last) / (float)(steps - 1) : 0.0f);
      need_loc = extrapolate((w > 0) ? (l_mid - l_last) / (float)w : 0.0f);
    }
  }
  const int need_all = max(max(__builtin_amdgcn_readlane(need, 0), __builtin_amdgcn_readlane(need, 1)),
                           max(__builtin_amdgcn_readlane(need, 2), __builtin_amdgcn_readlane(need, 3)));
  const int need_loc_all =
      max(max(__builtin_amdgcn_readlane(need_loc, 0), __builtin_amdgcn_readlane(need_loc, 1)),
          max(__builtin_amdgcn_readlane(need_loc, 2), __builtin_amdgcn_readlane(need_loc, 3)));
  if (lane == 0) {
    D.n_active = __builtin_popcountll(alive);
    if (cmax > 0) D.iters = m0 + cmax;
    D.accum_iters += c0 + c1 + c2 + c3;
    D.next = need_all;
    D.next_local = need_loc_all;
  }
  if (trace != nullptr) {
    for (int t = lane; t < cmax * kQ; t += 64) {
      const int jj = t / kQ, q = t % kQ;
      trace[m0 + jj][q] = (q < Q) ? tot[jj * Q + q] : 0.0;
    }
  }
}

__device__ __forceinline__ void write_status(LejaStatus* S, const Decision& D, int pit, int barriers, double nv,
                                             double lam, double c, double gamma, unsigned int* barrier_base,
                                             int skipped) {
#pragma unroll
  for (int k = 0; k < kMaxK; ++k) {
    S->state[k] = D.st[k];
    S->m_star[k] = D.mst[k];
    S->err[k] = D.err[k];
  }
  S->iters = D.iters;
  S->accum_iters = D.accum_iters;
  S->power_iters = pit;
  S->barriers = barriers;
  S->aborted = grid_aborted(barrier_base) != 0u ? 1 : 0;
  S->skipped = skipped;
  S->vnorm = nv;
  S->lam = lam;
  S->c = c;
  S->gamma = gamma;
}

// The launch's status, written by one thread: the device status block and,
// when the caller passed a host slot (pinned host memory), the same header
// there, so that the host needs no copy after the launch.
__device__ __forceinline__ void store_status(const ActionParams& P, const Decision& D, int pit, int barriers,
                                             double nv, double lam, double c, double gamma,
                                             const unsigned long long (&prof)[8], int skipped = 0) {
  write_status(P.status, D, pit, barriers, nv, lam, c, gamma, P.barrier, skipped);
  for (int q = 0; q < 8; ++q) P.status->prof[q] = prof[q];
  if (P.status_host != nullptr) {
    write_status(P.status_host, D, pit, barriers, nv, lam, c, gamma, P.barrier, skipped);
    for (int q = 0; q < 8; ++q) P.status_host->prof[q] = prof[q];
  }
}

// The learned proposal's attempt at one expansion (skip_src set) does no work
// when the proposal's decision, made on the device before the launch, asked
// for substeps or found no usable bound (*skip_src != 1): block 0 records the
// request and the bound in the status, every block leaves.  Returns true
// then; called by every thread with the same arguments.
__device__ __forceinline__ bool skip_launch(const ActionParams& P, double lam, const unsigned long long (&prof)[8]) {
  if (P.skip_src == nullptr) return false;
  const int sk = __builtin_amdgcn_readfirstlane(*P.skip_src);
  if (sk == 1) return false;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    Decision D;
    decision_init(D, 0, 1.0, 0.0, nullptr);
    store_status(P, D, 0, 0, 0.0, lam, 0.0, 0.0, prof, sk);
  }
  grid_exit(P.barrier);
  return true;
}

// ---------------------------------------------------------------------------
// Streaming passes over points p = pbeg, pbeg + stride, ... < pend, U points
// per thread at a time: every load of those points (stencil values, state,
// accumulators) is issued before any arithmetic or store, so a thread keeps
// all of them in flight at once.  The points are visited, and the per-thread
// sums accumulated, in the same order as a one-point loop, for every U.
// ---------------------------------------------------------------------------

// y(p) = scale * J x(p); sums of (scale x)^2 and y^2 (power iteration, Sec. 2.2)
template <int KIND, int NC, bool SHARED, int U>
__device__ __forceinline__ void power_pass(const OpDev& op, const double* __restrict__ src, double* __restrict__ dst,
                                           double scale, int pbeg, int pend, int stride, double& a0, double& a1) {
  for (int p0 = pbeg; p0 < pend; p0 += stride * U) {
    double xv[U][5][2], uv[U][5][2];
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (p0 + u * stride < pend) gather_point<KIND, NC>(op, src, p0 + u * stride, xv[u], uv[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * stride;
      if (p >= pend) continue;
      double out[2];
      stencil_jv<KIND>(op, xv[u], uv[u], out);
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const double x = scale * xv[u][0][cc];
        const double y = scale * out[cc];
        if constexpr (SHARED) {
          store_shared(dst + NC * p + cc, y);
        } else {
          dst[NC * p + cc] = y;
        }
        a0 += x * x;
        a1 += y * y;
      }
    }
  }
}

// One Newton step (Sec. 2.2 display): y = ((J - c) x)/gamma - xi x, and for
// every active accumulator p_k += d_k y; acc[0] += y^2, acc[1+k] += p_k^2.
// rgamma = 1/gamma (the quotient is div_rn).
template <int KIND, int NC, bool SHARED, int U, int KM = kMaxK>
__device__ __forceinline__ void newton_pass(const OpDev& op, const double* __restrict__ src,
                                            double* __restrict__ dst, double* const (&pp)[kMaxK],
                                            const bool (&act)[kMaxK], const double (&dk)[kMaxK], double c,
                                            double gamma, double rgamma, double xim, int pbeg, int pend,
                                            int stride, double (&acc)[1 + KM]) {
  for (int p0 = pbeg; p0 < pend; p0 += stride * U) {
    double xv[U][5][2], uv[U][5][2], pv[U][KM][2];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * stride;
      if (p >= pend) continue;
      gather_point<KIND, NC>(op, src, p, xv[u], uv[u]);
#pragma unroll
      for (int k = 0; k < KM; ++k)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) pv[u][k][cc] = act[k] ? pp[k][NC * p + cc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int p = p0 + u * stride;
      if (p >= pend) continue;
      double out[2];
      stencil_jv<KIND>(op, xv[u], uv[u], out);
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int idx = NC * p + cc;
        const double xc = xv[u][0][cc];
        const double y = div_rn(out[cc] - c * xc, gamma, rgamma) - xim * xc;
        if constexpr (SHARED) {
          store_shared(dst + idx, y);
        } else {
          dst[idx] = y;
        }
        acc[0] += y * y;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (act[k]) {
            const double pk = pv[u][k][cc] + dk[k] * y;
            pp[k][idx] = pk;
            acc[1 + k] += pk * pk;
          }
        }
      }
    }
  }
}

// per-block shared state of both action kernels
struct ActionShared {
  double xi[kTable];
  double coef[kMaxK * kTable];
  double fmax[kMaxK];
  double tot[64];
  double red[kQ * (kWaves + 1)];  // block_sum: wave sums, then totals
};

// ===========================================================================
// Streaming action kernel (any grid size): one pass over HBM per Newton step.
// ===========================================================================
template <int KIND, int NC, int KM>
__global__ __launch_bounds__(kBlock) void lj_action_stream(ActionParams P) {
  const GridSync gsync{P.barrier, P.spin_limit};
  __shared__ ActionShared sh;
  const OpDev& op = P.op;
  const int npts = op.npts;
  const int K = P.K;
  for (int i = threadIdx.x; i < kTable; i += blockDim.x) sh.xi[i] = P.xi[i];
  int p0, p1;
  point_range(npts, p0, p1);
  unsigned int epoch = 0;
  double wred[kQ];
  unsigned long long prof[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long t_last = wall_clock64();
  auto tick = [&](int phase) {
    const unsigned long long t = wall_clock64();
    prof[phase] += t - t_last;
    t_last = t;
  };

  // (1) spectral bound
  double lam = (P.lam_src != nullptr && !P.do_power) ? *P.lam_src : P.lam_in;
  if (skip_launch(P, lam, prof)) return;
  int pit = 0;
  if (P.do_power) {
    const double* x0 = P.start;
    if (x0 == nullptr) {
      for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
          store_shared(P.ybuf1 + NC * p + cc, 0.5 + splitmix_uniform(P.seed, (uint64_t)(NC * p + cc)));
      x0 = P.ybuf1;
      grid_barrier(gsync, epoch);
    }
    double scale = 1.0;
    for (int k = 0; k < P.power_iters; ++k) {
      const double* src = (k == 0) ? x0 : ((k & 1) ? P.ybuf0 : P.ybuf1);
      double* dst = (k & 1) ? P.ybuf1 : P.ybuf0;
      double a0 = 0.0, a1 = 0.0;
      power_pass<KIND, NC, true, 1>(op, src, dst, scale, p0 + (int)threadIdx.x, p1, blockDim.x, a0, a1);
#pragma unroll
      for (int q = 0; q < kQ; ++q) wred[q] = 0.0;
      wred[0] = a0;
      wred[1] = a1;
      block_sum<kQ>(wred, sh.red);
      double* area = partial_area(P.partials, epoch);
      if (threadIdx.x == 0) {
        put_partial(my_partial(area, 0), wred[0]);
        put_partial(my_partial(area, 1), wred[1]);
      }
      grid_allreduce(gsync, epoch, area, 2, sh.tot);
      const double nx = sqrt(sh.tot[0]);
      const double ny = sqrt(sh.tot[1]);
      lam = ny / nx;
      pit = k + 1;
      if (ny == 0.0) {
        lam = 0.0;
        break;
      }
      scale = 1.0 / ny;
    }
  }
  lam = uniform(lam);
  if (P.lam_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *P.lam_out = lam;
  double c, gamma;
  interval(lam, P.safety, c, gamma);
  const double rgamma = uniform(1.0 / gamma);
  tick(kProfPower);
  if (K == 0) {  // bound only
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Decision D;
      decision_init(D, 0, 1.0, 0.0, sh.fmax);
      store_status(P, D, pit, (int)epoch, 0.0, lam, c, gamma, prof);
    }
    grid_exit(P.barrier);
    return;
  }

  // (2) divided differences, every block for itself: d_0, d_1 now, then one
  // order more while each step's barrier is pending
  __syncthreads();
  DivDiff dd;
  dd_init(dd, K, P.l, P.s, P.max_points + 1, c, gamma, sh.xi, sh.coef, sh.fmax);
  dd_advance(dd, K, 1, sh.xi, sh.coef);
  __syncthreads();
  tick(kProfDivdiff);

  // (3) m = 0: p_k = d_{k,0} v and ||v||^2
  {
    double a0 = 0.0;
    for (int p = p0 + (int)threadIdx.x; p < p1; p += blockDim.x) {
#pragma unroll
      for (int cc = 0; cc < NC; ++cc) {
        const int idx = NC * p + cc;
        const double vv = P.v[idx];
        a0 += vv * vv;
#pragma unroll
        for (int k = 0; k < KM; ++k)
          if (k < K) P.p[k][idx] = sh.coef[k * kTable] * vv;
      }
    }
#pragma unroll
    for (int q = 0; q < kQ; ++q) wred[q] = 0.0;
    wred[0] = a0;
    block_sum<kQ>(wred, sh.red);
    if (threadIdx.x == 0) put_partial(my_partial(partial_area(P.partials, epoch), 0), wred[0]);
  }
  grid_allreduce(gsync, epoch, partial_area(P.partials, epoch), 1, sh.tot,
                 [&] { dd_advance(dd, K, 2, sh.xi, sh.coef); });
  const double nv = sqrt(sh.tot[0]);
  // The decision state is the same in every thread, so it lives once per block
  // in LDS: wave 0 takes the decisions, everyone reads the outcome.
  __shared__ Decision sD;
  __shared__ int s_commit[kMaxK];
  if (threadIdx.x < 64) decision_init(sD, K, nv, P.hump, sh.fmax);
  __syncthreads();

  for (int m = 1; m <= P.max_points && uniform(sD.n_active) > 0; ++m) {
    const double* __restrict__ src = (m == 1) ? P.v : ((m & 1) ? P.ybuf0 : P.ybuf1);
    double* __restrict__ dst = (m & 1) ? P.ybuf1 : P.ybuf0;
    const double xim = uniform(sh.xi[m - 1]);
    double dk[kMaxK];
    bool act[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) {
      act[k] = (k < KM) && (k < K) && (uniform(sD.st[k]) == ACC_RUNNING);
      dk[k] = act[k] ? uniform(sh.coef[k * kTable + m]) : 0.0;
    }
    double acc[1 + KM];
#pragma unroll
    for (int q = 0; q < 1 + KM; ++q) acc[q] = 0.0;
    // one point per thread at a time: two in flight measured no faster on
    // HBM-bound grids and spill at the 128-VGPR limit of 1024-thread blocks
    newton_pass<KIND, NC, true, 1, KM>(op, src, dst, P.p, act, dk, c, gamma, rgamma, xim, p0 + (int)threadIdx.x,
                                       p1, blockDim.x, acc);
    tick(kProfSteps);
    block_sum(acc, sh.red);
    double* area = partial_area(P.partials, epoch);
    if (threadIdx.x == 0) {
#pragma unroll
      for (int q = 0; q < 1 + KM; ++q)
        if (q <= K) put_partial(my_partial(area, q), acc[q]);
    }
    tick(kProfPublish);
    grid_allreduce(gsync, epoch, area, 1 + K, sh.tot, [&] { dd_advance(dd, K, m + 2, sh.xi, sh.coef); });
    tick(kProfBarrier);
    if (threadIdx.x < 64)
      replay_decisions(sD, K, m - 1, 1, 1 + K, sh.tot, sh.coef, P.tol, P.relative, P.max_points, s_commit,
                       blockIdx.x == 0 ? P.status->trace : nullptr);
    __syncthreads();
    tick(kProfDecide);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_status(P, sD, pit, (int)epoch, nv, lam, c, gamma, prof);
  }
  grid_exit(P.barrier);
}

// ===========================================================================
// LDS-tiled action kernel with temporal blocking: one tile per block, one
// owned point per thread, scalar families whose Jacobian reads the state at
// the centre only.  EPT: extended (tile + halo) points per thread; KM: the
// most accumulators the instance carries (1 for single actions and bounds,
// which frees the registers of the other three).
// Neumann families: extended points outside the domain are ghosts held at
// zero in both buffers, and a boundary cell's coefficient towards its ghost
// is folded into its diagonal (the ghost equals the cell itself), so every
// in-domain point stays exact through the super-step.
// ===========================================================================
template <int KIND, int S, int EPT, int KM>
__global__ __launch_bounds__(kBlock) void lj_action_tile(ActionParams P) {
  const GridSync gsync{P.barrier, P.spin_limit};
  static_assert(KIND == OP_ADVDIFF || KIND == OP_ALLENCAHN || KIND == OP_ADR,
                "tiled kernel: scalar centre-state families");
  constexpr bool kNeumann = family_neumann(KIND);
  extern __shared__ double lds[];
  __shared__ ActionShared sh;
  const OpDev& op = P.op;
  const int K = P.K;
  const int Q = 1 + K;  // reduced values per Newton step: ||y||^2, then K ||p_k||^2
  const int nx = op.nx, ny = op.ny;
  for (int i = threadIdx.x; i < kTable; i += blockDim.x) sh.xi[i] = P.xi[i];

  // ---- tile geometry: owned w x h points at (x0, y0), extended by S per side
  const int tb = xcd_chunk(blockIdx.x, gridDim.x);
  const int x0 = (tb % P.ntx) * P.tx, y0 = (tb / P.ntx) * P.ty;
  const int w = min(P.tx, nx - x0), h = min(P.ty, ny - y0);
  const int EW = w + 2 * S, EH = h + 2 * S, NE = EW * EH;
  // dynamic LDS: two buffers of the extended tile, then the owned point's
  // basis values of the current super-step, H[(j-1) * kBlock + thread].
  // Buffers are addressed by offsets from `lds` (never through a pointer
  // table) so that the accesses compile to LDS instructions, not flat ones.
  auto Y = [&](int b) { return lds + b * NE; };
  double* H = lds + P.lds_h;
  // extended points of this thread: e = threadIdx.x + k * kBlock (valid if < NE),
  // tile coordinates packed as ex | ey << 16.
  // The stencil is folded into five coefficients: (J x)(p) = fw x_W + fe x_E +
  // fs x_S + fn x_N + e_d(p) x_C, e_d(p) the diagonal of J at the point (for
  // Allen-Cahn the Laplacian's centre plus 1 - 3u^2).  Once the bound is known
  // all five are divided by gamma and c / gamma is taken off the diagonal, so
  // a Newton step is y = fw x_W + ... + (e_d(p) - xi) x_C: six FP64 operations
  // instead of thirteen -- the same polynomial in J, rounded in another order.
  int e_xy[EPT];
  double e_d[EPT];
  bool ghost[EPT];  // outside the domain (Neumann families only)
  double fw, fe, fs, fn;
  if constexpr (KIND == OP_ALLENCAHN) {
    fw = fe = op.c0 * op.idx2;
    fs = fn = op.c0 * op.idy2;
  } else if constexpr (KIND == OP_ADR) {  // alpha Lap x + beta (d_x + d_y) x (centred)
    fw = op.c0 * op.idx2 - op.c1 * op.i2dx;
    fe = op.c0 * op.idx2 + op.c1 * op.i2dx;
    fs = op.c0 * op.idy2 - op.c1 * op.i2dy;
    fn = op.c0 * op.idy2 + op.c1 * op.i2dy;
  } else {  // advection-diffusion: nu Lap x - a_x d_x x - a_y d_y x (centred)
    fw = op.c0 * op.idx2 + op.c1 * op.i2dx;
    fe = op.c0 * op.idx2 - op.c1 * op.i2dx;
    fs = op.c0 * op.idy2 + op.c2 * op.i2dy;
    fn = op.c0 * op.idy2 - op.c2 * op.i2dy;
  }
  const double d_lap = -2.0 * op.c0 * (op.idx2 + op.idy2);
  auto gidx = [&](int k) {
    const int ex = e_xy[k] & 0xffff, ey = e_xy[k] >> 16;
    int gx = (x0 - S + ex) % nx;
    if (gx < 0) gx += nx;
    int gy = (y0 - S + ey) % ny;
    if (gy < 0) gy += ny;
    return gy * nx + gx;
  };
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const int e = threadIdx.x + k * kBlock;
    const int ey = e / EW;
    const int ex = e - ey * EW;
    e_xy[k] = ex | (ey << 16);
    const int ux = x0 - S + ex, uy = y0 - S + ey;  // unwrapped grid coordinates
    ghost[k] = kNeumann && (ux < 0 || ux >= nx || uy < 0 || uy >= ny);
    if constexpr (KIND == OP_ALLENCAHN) {
      const double u = (e < NE) ? op.state[gidx(k)] : 0.0;
      e_d[k] = d_lap + (1.0 - 3.0 * u * u);
    } else if constexpr (KIND == OP_ADR) {
      const double u = (e < NE && !ghost[k]) ? op.state[gidx(k)] : 0.0;
      double d = d_lap + op.c2 * (u * (3.0 - 3.0 * u) - 0.5);
      if (ux == 0) d += fw;
      if (ux == nx - 1) d += fe;
      if (uy == 0) d += fs;
      if (uy == ny - 1) d += fn;
      e_d[k] = d;
    } else {
      e_d[k] = d_lap;
    }
  }
  const int o = threadIdx.x;
  const bool own = o < w * h;
  const int lx = own ? o % w : 0, ly = own ? o / w : 0;
  const int eo = (ly + S) * EW + lx + S;
  const int go = (y0 + ly) * nx + x0 + lx;

  unsigned int epoch = 0;
  int cur = 0, par = 0;
  unsigned long long prof[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long t_last = wall_clock64();
  auto tick = [&](int phase) {
    const unsigned long long t = wall_clock64();
    prof[phase] += t - t_last;
    t_last = t;
  };

  // one step on the region still exact after j steps: a power product (the
  // coefficients of J, xim = 0) or a Newton step (the coefficients divided
  // by gamma, xim = xi_{m-1})
  auto step = [&](int j, double xim) {
    const double* src = Y(cur);
    double* dst = Y(cur ^ 1);
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e >= NE) continue;
      if (kNeumann && ghost[k]) {
        dst[e] = 0.0;
        continue;
      }
      const int ex = e_xy[k] & 0xffff, ey = e_xy[k] >> 16;
      if (ex < j || ex >= EW - j || ey < j || ey >= EH - j) continue;
      const double xc = src[e], xw = src[e - 1], xe = src[e + 1], xs = src[e - EW], xn = src[e + EW];
      double y;
      if constexpr (KIND == OP_ALLENCAHN) {
        y = fw * (xw + xe) + fs * (xs + xn);
      } else {
        y = fw * xw + fe * xe + fs * xs + fn * xn;
      }
      dst[e] = fma(e_d[k] - xim, xc, y);
    }
    __syncthreads();
    cur ^= 1;
  };
  // halo ring of the extended tile: fetched from a global vector into
  // registers right after a barrier (its loads overlap the partial sums'),
  // written into the current buffer once the stop decisions are taken, the
  // owned points scaled alongside (scale 1: halo only)
  auto inner = [&](int k) {
    const int ex = e_xy[k] & 0xffff, ey = e_xy[k] >> 16;
    return ex >= S && ex < S + w && ey >= S && ey < S + h;
  };
  double hv[EPT];
  auto fetch_halo = [&](const double* g) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * kBlock;
      hv[k] = (e < NE && !inner(k) && !ghost[k]) ? g[gidx(k)] : 0.0;
    }
  };
  auto put_halo = [&](double scale) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e >= NE) continue;
      if (inner(k)) {
        if (scale != 1.0) Y(cur)[e] *= scale;
      } else {
        Y(cur)[e] = scale * hv[k];
      }
    }
    __syncthreads();
  };
  // Block sums of one value per thread for each step of a super-step: per
  // step only the 16-lane row sums are formed (four DPP adds) and staged,
  // rowred[slot * 64 + 4 * wave + row]; the block totals of all the
  // super-step's slots are formed at once before the barrier, one wave per
  // slot summing its 64 row sums.
  static_assert(4 * kWaves == 64, "one lane per row sum of a slot");
  __shared__ double rowred[kPartStride * 4 * kWaves];
  auto stage = [&](int slot, double v) {
    const double s = row_sum(v);
    if ((threadIdx.x & 15) == 15) rowred[slot * 4 * kWaves + (threadIdx.x >> 4)] = s;
  };
  // block totals of staged slots [0, nslots) -> this barrier's partials
  auto publish = [&](int nslots) {
    __syncthreads();
    double* area = partial_area(P.partials, epoch);
    const int lane = threadIdx.x & 63;
    for (int q = threadIdx.x >> 6; q < nslots; q += kWaves) {
      const double t = wave_sum(rowred[q * 4 * kWaves + lane]);
      if (lane == 0) put_partial(my_partial(area, q), t);
    }
    __syncthreads();
    return area;
  };

  // ---- (1) spectral bound: S products between barriers, normalised per barrier
  double lam = (P.lam_src != nullptr && !P.do_power) ? *P.lam_src : P.lam_in;
  if (skip_launch(P, lam, prof)) return;
  int pit = 0;
  if (P.do_power) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = threadIdx.x + k * kBlock;
      if (e >= NE) continue;
      const int g = gidx(k);
      Y(0)[e] = ghost[k] ? 0.0 : (P.start ? P.start[g] : 0.5 + splitmix_uniform(P.seed, (uint64_t)g));
    }
    __syncthreads();
    int done = 0;
    while (done < P.power_iters) {
      const int steps = min(S, P.power_iters - done);
      {
        const double x = own ? Y(cur)[eo] : 0.0;
        stage(0, x * x);
      }
      for (int j = 1; j <= steps; ++j) {
        step(j, 0.0);
        const double y = own ? Y(cur)[eo] : 0.0;
        stage(j, y * y);
      }
      double* area = publish(steps + 1);
      double* yb = (par == 0) ? P.ybuf0 : P.ybuf1;
      if (own) store_shared(yb + go, Y(cur)[eo]);
      const bool more = done + steps < P.power_iters;
      grid_allreduce(gsync, epoch, area, steps + 1, sh.tot, NoOverlap{}, [&] {
        if (more) fetch_halo(yb);
      });
      const double nprev = sh.tot[steps - 1], nlast = sh.tot[steps];
      done += steps;
      pit = done;
      lam = sqrt(nlast) / sqrt(nprev);
      if (nlast == 0.0) {
        lam = 0.0;
        break;
      }
      if (more) {
        put_halo(1.0 / sqrt(nlast));
        par ^= 1;
      }
    }
  }
  lam = uniform(lam);
  if (P.lam_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *P.lam_out = lam;
  double c, gamma;
  interval(lam, P.safety, c, gamma);
  const double rgamma = uniform(1.0 / gamma);
  tick(kProfPower);
  if (K == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Decision D;
      decision_init(D, 0, 1.0, 0.0, sh.fmax);
      store_status(P, D, pit, (int)epoch, 0.0, lam, c, gamma, prof);
    }
    grid_exit(P.barrier);
    return;
  }

  // the Newton steps' coefficients: (J - c) / gamma
  fw *= rgamma;
  fe *= rgamma;
  fs *= rgamma;
  fn *= rgamma;
#pragma unroll
  for (int k = 0; k < EPT; ++k) e_d[k] = (e_d[k] - c) * rgamma;

  // ---- (2) divided differences up to the first super-step's last term (the
  // rest while barriers are pending), and y_0 = v on the extended tile
  // (v's loads are issued after the node values -- whose function calls
  // would wait for them -- and are in flight while the table advances)
  __syncthreads();
  DivDiff dd;
  dd_init(dd, K, P.l, P.s, P.max_points + 1, c, gamma, sh.xi, sh.coef, sh.fmax);
  double v_in[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) v_in[k] = ((int)threadIdx.x + k * kBlock < NE && !ghost[k]) ? P.v[gidx(k)] : 0.0;
  dd_advance(dd, K, S, sh.xi, sh.coef);
  cur = 0;
#pragma unroll
  for (int k = 0; k < EPT; ++k)
    if ((int)threadIdx.x + k * kBlock < NE) Y(0)[threadIdx.x + k * kBlock] = v_in[k];
  __syncthreads();
  tick(kProfDivdiff);

  // ---- (3) Newton recurrence in super-steps of S.  The decision state is the
  // same in every thread, so it lives once per block in LDS: wave 0 replays
  // the decisions, everyone reads the outcome.
  __shared__ Decision sD;
  __shared__ int s_commit[kMaxK];
  double pk[KM];
  const double v_own = own ? Y(0)[eo] : 0.0;
#pragma unroll
  for (int k = 0; k < KM; ++k) pk[k] = sh.coef[k * kTable] * v_own;
  if (threadIdx.x == 0) decision_init(sD, K, 1.0, 0.0, sh.fmax);  // redone once ||v|| is known
  __syncthreads();
  double nv = 0.0;
  bool first = true;
  int m0 = 0;
  while (true) {
    const int steps = min(min(S, P.max_points - m0), uniform(sD.next));
    bool act0[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) act0[k] = (k < K) && (uniform(sD.st[k]) == ACC_RUNNING);
    double ps[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) ps[k] = pk[k];
#pragma unroll
    for (int j = 1; j <= S; ++j) {
      if (j > steps) break;
      const int m = m0 + j;
      step(j, uniform(sh.xi[m - 1]));
      const double y = own ? Y(cur)[eo] : 0.0;
      H[(j - 1) * kBlock + threadIdx.x] = y;
      stage((j - 1) * Q, y * y);
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (!act0[k]) continue;
        ps[k] = ps[k] + uniform(sh.coef[k * kTable + m]) * y;
        stage((j - 1) * Q + 1 + k, ps[k] * ps[k]);
      }
    }
    tick(kProfSteps);
    if (first) stage(steps * Q, v_own * v_own);  // ||v||^2 rides on the first barrier
    const int nq = steps * Q + (first ? 1 : 0);
    double* area = publish(nq);
    double* yb = (par == 0) ? P.ybuf0 : P.ybuf1;
    if (own) store_shared(yb + go, Y(cur)[eo]);
    tick(kProfPublish);
    grid_allreduce(
        gsync, epoch, area, nq, sh.tot, [&] { dd_advance(dd, K, m0 + steps + S, sh.xi, sh.coef); },
        [&] { fetch_halo(yb); });
    tick(kProfBarrier);
    if (threadIdx.x < 64) {
      if (first) {
        nv = sqrt(sh.tot[steps * Q]);
        decision_init(sD, K, nv, P.hump, sh.fmax);
      }
      replay_decisions(sD, K, m0, steps, Q, sh.tot, sh.coef, P.tol, P.relative, P.max_points, s_commit,
                       blockIdx.x == 0 ? P.status->trace : nullptr);
    }
    first = false;
    __syncthreads();
    tick(kProfDecide);
    // commit each accumulator's terms up to its stop index
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const int ck = uniform(s_commit[k]);
#pragma unroll
      for (int j = 1; j <= S; ++j)
        if (j <= ck) pk[k] = pk[k] + uniform(sh.coef[k * kTable + m0 + j]) * H[(j - 1) * kBlock + threadIdx.x];
    }
    m0 += steps;
    tick(kProfCommit);
    if (sD.n_active == 0 || m0 >= P.max_points) break;
    put_halo(1.0);
    par ^= 1;
    tick(kProfHalo);
  }
  if (own) {
#pragma unroll
    for (int k = 0; k < KM; ++k)
      if (k < K) P.p[k][go] = pk[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_status(P, sD, pit, (int)epoch, nv, lam, c, gamma, prof);
  }
  grid_exit(P.barrier);
}

// ===========================================================================
// Register-tiled action kernel with temporal blocking, for the periodic
// scalar families whose Jacobian reads the state at the centre only
// (Allen-Cahn, advection-diffusion).  One block of 8 waves per CU owns a
// 32 x 32 tile; the tile extended by kRegS = 16 points on every side is
// 64 x 64 and lives in registers: lane c of every wave holds column c, wave w
// rows 8w .. 8w+7.  A step takes the west and east neighbours from the
// adjacent lanes (DPP wave shifts), north and south from the lane's own
// registers, and the outer neighbours of a wave's first and last rows from
// the adjacent waves through LDS (one workgroup barrier per step).  Values at
// the borders of the extended tile go stale by one column / row per step, so
// after 16 steps exactly the owned 32 x 32 points are exact: up to 16 Newton
// steps run between grid barriers, with the halo recomputed in registers.
// The owned points' basis values of the super-step go to LDS (the history
// the commit replays when an accumulator stops inside a super-step); the
// accumulators run speculatively in registers, and the committed values are
// kept in the output vectors between super-steps.  Per point and step the
// arithmetic is that of lj_action_tile (the same folded stencil), so the
// results are term for term those of the untiled recurrence up to that
// stencil's rounding.
// ===========================================================================
constexpr int kRegS = 16;                        // steps per super-step = halo width
constexpr int kRegTile = 32;                     // owned tile edge
constexpr int kRegWaves = 8;
constexpr int kRegRows = 8;                      // extended rows per wave
constexpr int kRegBlock = 64 * kRegWaves;
constexpr int kRegSlots = kRegS * (1 + kMaxK) + 1;  // reduced values per super-step, at most
static_assert(kRegWaves * kRegRows == kRegTile + 2 * kRegS && kRegTile + 2 * kRegS == 64, "64 x 64 extended tile");
static_assert(kRegSlots <= kRegPartStride, "partial-sum slots");

struct RegShared {
  double xi[kTable];
  double coef[kMaxK * kTable];
  double fmax[kMaxK];
  double tot[kRegSlots];
  double stg[kRegSlots][4];            // per step and value: the sums of the owned waves 2..5 (lanes 16-47)
  double xrow[2][2 * kRegWaves][64];   // [parity][2 w: first row of wave w, 2 w + 1: its last row][lane]
  Decision D;
  int commit[kMaxK];
  int lk[kMaxK];     // l_k and s_k of the launch (read from LDS by the divided differences)
  double sk[kMaxK];
};

// Compile-time tag of a tile's shape in the several-tile kernel: full (every
// point of lanes 16-47 in the owned waves is owned) or ragged (masked).
template <bool B>
struct TileTag {
  static constexpr bool full = B;
};

// Partial sums of one super-step: slot q of block b at area[q * G + b].
__device__ __forceinline__ double* reg_area(double* partials, unsigned int epoch) {
  return partials + (size_t)(epoch & 1u) * kRegPartStride * gridDim.x;
}

// After a grid barrier: totals of slots [0, nq) of `area` into tot (LDS);
// wave w adds the slots w, w + 8, ..., CH of them per round, lane t the blocks
// t, t + 64, t + 128, t + 192 (G <= 256) in that order, then the wave sums
// its lanes -- the same fixed order in every block.  All loads of a round are
// issued before any sum.
template <int CH>
__device__ __forceinline__ void reg_reduce(const double* area, int nq, double* tot) {
  const int G = gridDim.x;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int r0 = 0; r0 * kRegWaves < nq; r0 += CH) {
    double v[CH][4];
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int q = w + kRegWaves * (r0 + r);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int b = lane + 64 * c;
        v[r][c] = (q < nq && b < G) ? area[(size_t)q * G + b] : 0.0;
      }
    }
#pragma unroll
    for (int r = 0; r < CH; ++r) {
      const int q = w + kRegWaves * (r0 + r);
      const double a = ((v[r][0] + v[r][1]) + v[r][2]) + v[r][3];
      const double t = wave_sum(a);
      if (q < nq && lane == 0) tot[q] = t;
    }
  }
  __syncthreads();
}

template <int KIND, int KM, bool FULL>
__global__ __launch_bounds__(kRegBlock) void lj_action_reg(ActionParams P) {
  static_assert(KIND == OP_ADVDIFF || KIND == OP_ALLENCAHN, "register-tiled kernel: periodic scalar families");
  constexpr int CH = (KM == 1) ? 5 : 3;  // rows of partial sums per wave and load round
  const GridSync gsync{P.barrier, P.spin_limit};
  extern __shared__ double Hist[];  // kRegS x 1024: basis values of the owned points per step
  __shared__ RegShared sh;
  const OpDev& op = P.op;
  const int K = P.K;
  const int Q = 1 + K;
  const int nx = op.nx, ny = op.ny;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  static_assert(kTable <= kRegBlock, "one Leja node per thread");
  // the nodes, l_k and s_k go to LDS just before the divided differences;
  // their loads are issued here with the state's and the bound's (indices
  // clamped in range: no branch, so no load waits for another)
  const double xi_t = P.xi[min((int)threadIdx.x, kTable - 1)];
  const int l_t = P.l[min((int)threadIdx.x, kMaxK - 1)];
  const double s_t = P.s[min((int)threadIdx.x, kMaxK - 1)];

  // ---- tile geometry: owned w x h points at (x0, y0); lane = extended column,
  // rows 8 wv + i of the extended tile (extended origin at x0 - 16, y0 - 16)
  const int tb = xcd_chunk(blockIdx.x, gridDim.x);
  const int x0 = (tb % P.ntx) * kRegTile, y0 = (tb / P.ntx) * kRegTile;
  const int w = min(kRegTile, nx - x0), h = min(kRegTile, ny - y0);
  int gxc = (x0 - kRegS + lane) % nx;  // this lane's global column (periodic)
  if (gxc < 0) gxc += nx;
  auto grow = [&](int i) {  // global row of extended row 8 wv + i
    int gy = (y0 - kRegS + kRegRows * wv + i) % ny;
    if (gy < 0) gy += ny;
    return gy;
  };
  const bool lane_own = lane >= kRegS && lane < kRegS + w;
  const bool owned_wave = wv >= 2 && wv < 6;  // rows 16 .. 47
  auto row_own = [&](int i) {
    const int r = kRegRows * wv + i - kRegS;
    return r >= 0 && r < h;
  };
  auto own = [&](int i) { return FULL ? (owned_wave && lane_own) : (lane_own && row_own(i)); };
  // a value of an owned point, zero elsewhere (called by the owned waves only:
  // in a full tile the row sums taken there, lanes 16-31 and 32-47, see owned
  // points only, so no mask is needed)
  auto ownv = [&](int i, double v) { return FULL ? v : (own(i) ? v : 0.0); };
  auto hidx = [&](int i) { return (kRegRows * wv + i - kRegS) * kRegTile + (lane - kRegS); };
  auto gown = [&](int i) { return (y0 + kRegRows * wv + i - kRegS) * nx + x0 + lane - kRegS; };

  // folded stencil as in lj_action_tile: (J x)(p) = fw x_W + fe x_E + fs x_S +
  // fn x_N + e_d(p) x_C
  double fw, fe, fs, fn;
  if constexpr (KIND == OP_ALLENCAHN) {
    fw = fe = op.c0 * op.idx2;
    fs = fn = op.c0 * op.idy2;
  } else {
    fw = op.c0 * op.idx2 + op.c1 * op.i2dx;
    fe = op.c0 * op.idx2 - op.c1 * op.i2dx;
    fs = op.c0 * op.idy2 + op.c2 * op.i2dy;
    fn = op.c0 * op.idy2 - op.c2 * op.i2dy;
  }
  const double d_lap = -2.0 * op.c0 * (op.idx2 + op.idy2);
  double x[kRegRows], dg[kRegRows];
#pragma unroll
  for (int i = 0; i < kRegRows; ++i) {
    if constexpr (KIND == OP_ALLENCAHN) {
      const double u = op.state[(size_t)grow(i) * nx + gxc];
      dg[i] = d_lap + (1.0 - 3.0 * u * u);
    } else {
      dg[i] = d_lap;
    }
  }

  unsigned int epoch = 0;
  int par = 0;     // row-exchange buffer
  int ypar = 0;    // global exchange vector
  unsigned long long prof[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long t_last = wall_clock64();
  auto tick = [&](int phase) {
    const unsigned long long t = wall_clock64();
    prof[phase] += t - t_last;
    t_last = t;
  };

  // one step of x <- A x on the whole extended tile, A = the folded stencil
  // with diagonal dg - xim
  // (the interior rows 1..6 are formed while the neighbours' rows are read)
  auto point = [&](int i, double xs, double xn, double xim) {
    const double xc = x[i];
    const double xw = dpp_move<0x138>(xc);  // wave_shr:1 -- lane c - 1
    const double xe = dpp_move<0x130>(xc);  // wave_shl:1 -- lane c + 1
    double y;
    if constexpr (KIND == OP_ALLENCAHN) {
      y = fw * (xw + xe) + fs * (xs + xn);
    } else {
      y = fw * xw + fe * xe + fs * xs + fn * xn;
    }
    return fma(dg[i] - xim, xc, y);
  };
  auto step = [&](double xim) {
    double* xr = &sh.xrow[par][0][0];
    xr[(2 * wv) * 64 + lane] = x[0];
    xr[(2 * wv + 1) * 64 + lane] = x[kRegRows - 1];
    __syncthreads();
    const double above = xr[(2 * ((wv + kRegWaves - 1) % kRegWaves) + 1) * 64 + lane];
    const double below = xr[(2 * ((wv + 1) % kRegWaves)) * 64 + lane];
    par ^= 1;
    double y[kRegRows];
#pragma unroll
    for (int i = 1; i < kRegRows - 1; ++i) y[i] = point(i, x[i - 1], x[i + 1], xim);
    y[0] = point(0, above, x[1], xim);
    y[kRegRows - 1] = point(kRegRows - 1, x[kRegRows - 2], below, xim);
#pragma unroll
    for (int i = 0; i < kRegRows; ++i) x[i] = y[i];
  };
  // row sums of one value per owned point (owned waves only): lanes 31 and 47
  // hold the sums of lanes 16-31 and 32-47
  auto stage = [&](int slot, double a) {
    const double t = row_sum(a);
    const double u = read_lane(t, 31) + read_lane(t, 47);
    if (lane == 0) sh.stg[slot][wv - 2] = u;
  };
  // block totals of the staged slots -> this barrier's partial-sum area
  auto publish = [&](int nq) {
    __syncthreads();
    double* area = reg_area(P.partials, epoch);
    for (int q = threadIdx.x; q < nq; q += kRegBlock) {
      const double t = (sh.stg[q][0] + sh.stg[q][1]) + (sh.stg[q][2] + sh.stg[q][3]);
      store_shared(area + (size_t)q * gridDim.x + blockIdx.x, t);
    }
    return area;
  };
  // the owned points' current values to the exchange vector; after the
  // barrier the halo (every position outside the owned points) is reloaded
  // from it, scaled
  auto put_owned = [&]() {
    double* yb = ypar ? P.ybuf1 : P.ybuf0;
    if (owned_wave) {
#pragma unroll
      for (int i = 0; i < kRegRows; ++i)
        if (own(i)) store_shared(yb + gown(i), x[i]);
    }
  };
  auto fetch_halo = [&]() {
    const double* yb = ypar ? P.ybuf1 : P.ybuf0;
#pragma unroll
    for (int i = 0; i < kRegRows; ++i)
      if (!own(i)) x[i] = yb[(size_t)grow(i) * nx + gxc];
  };

  // sum of squares of the owned points' current values over this lane's rows
  // (two interleaved partial sums, then added)
  auto sumsq_own = [&]() {
    double a0 = 0.0, a1 = 0.0;
#pragma unroll
    for (int i = 0; i < kRegRows; i += 2) {
      const double t0 = ownv(i, x[i]), t1 = ownv(i + 1, x[i + 1]);
      a0 = fma(t0, t0, a0);
      a1 = fma(t1, t1, a1);
    }
    return a0 + a1;
  };

  // ---- (1) spectral bound: up to 16 products between barriers, normalised per barrier
  double lam = (P.lam_src != nullptr && !P.do_power) ? *P.lam_src : P.lam_in;
  if (skip_launch(P, lam, prof)) return;
  int pit = 0;
  if (P.do_power) {
#pragma unroll
    for (int i = 0; i < kRegRows; ++i) {
      const size_t g = (size_t)grow(i) * nx + gxc;
      x[i] = P.start ? P.start[g] : 0.5 + splitmix_uniform(P.seed, (uint64_t)g);
    }
    int done = 0;
    while (done < P.power_iters) {
      const int steps = min(kRegS, P.power_iters - done);
      // only the last two norms are read (the bound and the rescaling):
      // slot 0 holds ||x|| before the last product, slot 1 after it
      if (owned_wave && steps == 1) stage(0, sumsq_own());
      for (int j = 1; j <= steps; ++j) {
        step(0.0);
        if (owned_wave && j >= steps - 1) stage(j - (steps - 1), sumsq_own());
      }
      double* area = publish(2);
      put_owned();
      const bool more = done + steps < P.power_iters;
      grid_allreduce(gsync, epoch, nullptr, 0, nullptr, NoOverlap{}, [&] {
        if (more) fetch_halo();
      });
      reg_reduce<CH>(area, 2, sh.tot);
      const double nprev = sh.tot[0], nlast = sh.tot[1];
      done += steps;
      pit = done;
      lam = sqrt(nlast) / sqrt(nprev);
      if (nlast == 0.0) {
        lam = 0.0;
        break;
      }
      if (more) {
        const double sc = 1.0 / sqrt(nlast);
#pragma unroll
        for (int i = 0; i < kRegRows; ++i) x[i] *= sc;
        ypar ^= 1;
      }
    }
  }
  lam = uniform(lam);
  if (P.lam_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *P.lam_out = lam;
  double c, gamma;
  interval(lam, P.safety, c, gamma);
  const double rgamma = uniform(1.0 / gamma);
  tick(kProfPower);
  if (K == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Decision D;
      decision_init(D, 0, 1.0, 0.0, sh.fmax);
      store_status(P, D, pit, (int)epoch, 0.0, lam, c, gamma, prof);
    }
    grid_exit(P.barrier);
    return;
  }

  // the Newton steps' coefficients: (J - c) / gamma
  fw *= rgamma;
  fe *= rgamma;
  fs *= rgamma;
  fn *= rgamma;
#pragma unroll
  for (int i = 0; i < kRegRows; ++i) dg[i] = (dg[i] - c) * rgamma;

  // ---- (2) y_0 = v on the extended tile, and the divided differences up to
  // the first super-step's last term (the rest while barriers are pending).
  // v's loads are issued first and stay in flight while the table is formed:
  // it reads LDS only (the nodes, l_k and s_k), so nothing waits on them
  // before the first use of y_0
#pragma unroll
  for (int i = 0; i < kRegRows; ++i) x[i] = P.v[(size_t)grow(i) * nx + gxc];
  if (threadIdx.x < kTable) sh.xi[threadIdx.x] = xi_t;
  if (threadIdx.x < kMaxK) {
    sh.lk[threadIdx.x] = l_t;
    sh.sk[threadIdx.x] = s_t;
  }
  __syncthreads();
  DivDiff dd;
  dd_init_par(dd, K, sh.lk, sh.sk, P.max_points + 1, c, gamma, sh.xi, sh.coef, sh.fmax);
  dd_advance(dd, K, kRegS, sh.xi, sh.coef);
  __syncthreads();
  tick(kProfDivdiff);

  // ---- (3) Newton recurrence in super-steps of up to 16.  Committed
  // accumulator values live in the outputs between super-steps: p_k = d_{k,0} v.
  double ps[KM][kRegRows];
  double v_sq = 0.0;
  if (owned_wave) {
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const double d0 = sh.coef[k * kTable];
#pragma unroll
      for (int i = 0; i < kRegRows; ++i) {
        ps[k][i] = d0 * x[i];
        if (k < K && own(i)) P.p[k][gown(i)] = ps[k][i];
      }
    }
    v_sq = sumsq_own();
  }
  if (threadIdx.x == 0) decision_init(sh.D, K, 1.0, 0.0, sh.fmax);  // redone once ||v|| is known
  __syncthreads();
  double nv = 0.0;
  bool first = true;
  int m0 = 0;
  while (true) {
    const int steps = min(min(kRegS, P.max_points - m0), min(uniform(sh.D.next), uniform(sh.D.next_local)));
    bool act0[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) act0[k] = (k < K) && (uniform(sh.D.st[k]) == ACC_RUNNING);
    // the super-step's nodes and coefficients, lane j holding those of step
    // m0 + 1 + j (read per step with readlane: no LDS wait in the loop)
    const double xiv = (lane < steps) ? sh.xi[m0 + lane] : 0.0;
    double cfv[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) cfv[k] = (lane < steps && act0[k]) ? sh.coef[k * kTable + m0 + 1 + lane] : 0.0;
    for (int j = 1; j <= steps; ++j) {
      step(read_lane(xiv, j - 1));
      if (owned_wave) {
        if (FULL) {
          if (lane_own) {
#pragma unroll
            for (int i = 0; i < kRegRows; ++i) Hist[(j - 1) * (kRegTile * kRegTile) + hidx(i)] = x[i];
          }
        } else {
#pragma unroll
          for (int i = 0; i < kRegRows; ++i)
            if (own(i)) Hist[(j - 1) * (kRegTile * kRegTile) + hidx(i)] = x[i];
        }
        // ||y||^2 and, for every accumulator (a frozen one adds 0 * y, which
        // leaves its sum unchanged), the new p_k and ||p_k||^2; the row sums
        // of all 1 + KM values run side by side
        double t[1 + KM];
        t[0] = sumsq_own();
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const double dk = read_lane(cfv[k], j - 1);
          double b0 = 0.0, b1 = 0.0;
#pragma unroll
          for (int i = 0; i < kRegRows; i += 2) {
            ps[k][i] = ps[k][i] + dk * x[i];
            ps[k][i + 1] = ps[k][i + 1] + dk * x[i + 1];
            const double t0 = ownv(i, ps[k][i]), t1 = ownv(i + 1, ps[k][i + 1]);
            b0 = fma(t0, t0, b0);
            b1 = fma(t1, t1, b1);
          }
          t[1 + k] = b0 + b1;
        }
#pragma unroll
        for (int q = 0; q < 1 + KM; ++q) t[q] += dpp_move<0x111>(t[q]);
#pragma unroll
        for (int q = 0; q < 1 + KM; ++q) t[q] += dpp_move<0x112>(t[q]);
#pragma unroll
        for (int q = 0; q < 1 + KM; ++q) t[q] += dpp_move<0x114>(t[q]);
#pragma unroll
        for (int q = 0; q < 1 + KM; ++q) t[q] += dpp_move<0x118>(t[q]);
        double u[1 + KM];
#pragma unroll
        for (int q = 0; q < 1 + KM; ++q) u[q] = read_lane(t[q], 31) + read_lane(t[q], 47);
        if (lane == 0) {
          sh.stg[(j - 1) * Q][wv - 2] = u[0];
#pragma unroll
          for (int k = 0; k < KM; ++k)
            if (k < K) sh.stg[(j - 1) * Q + 1 + k][wv - 2] = u[1 + k];
        }
      }
    }
    tick(kProfSteps);
    if (first && owned_wave) stage(steps * Q, v_sq);  // ||v||^2 rides on the first barrier
    const int nq = steps * Q + (first ? 1 : 0);
    double* area = publish(nq);
    put_owned();
    tick(kProfPublish);
    grid_allreduce(
        gsync, epoch, nullptr, 0, nullptr, [&] { dd_advance(dd, K, m0 + steps + kRegS, sh.xi, sh.coef); },
        [&] { fetch_halo(); });
    reg_reduce<CH>(area, nq, sh.tot);
    tick(kProfBarrier);
    if (threadIdx.x < 64) {
      if (first) {
        nv = sqrt(sh.tot[steps * Q]);
        decision_init(sh.D, K, nv, P.hump, sh.fmax);
      }
      replay_decisions(sh.D, K, m0, steps, Q, sh.tot, sh.coef, P.tol, P.relative, P.max_points, sh.commit,
                       blockIdx.x == 0 ? P.status->trace : nullptr);
    }
    first = false;
    __syncthreads();
    tick(kProfDecide);
    // commit: an accumulator that ran through the super-step keeps its
    // speculative sum; one that stopped inside it adds its terms up to its
    // stop index to the committed value, from the history
    if (owned_wave) {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (k >= K) continue;
        const int ck = uniform(sh.commit[k]);
        if (ck == 0) continue;
        if (ck < steps) {
#pragma unroll
          for (int i = 0; i < kRegRows; ++i) {
            if (!own(i)) continue;
            double pk = P.p[k][gown(i)];
            for (int j = 1; j <= ck; ++j)
              pk = pk + uniform(sh.coef[k * kTable + m0 + j]) * Hist[(j - 1) * (kRegTile * kRegTile) + hidx(i)];
            ps[k][i] = pk;
          }
        }
#pragma unroll
        for (int i = 0; i < kRegRows; ++i)
          if (own(i)) P.p[k][gown(i)] = ps[k][i];
      }
    }
    m0 += steps;
    ypar ^= 1;
    tick(kProfCommit);
    if (sh.D.n_active == 0 || m0 >= P.max_points) break;
    __syncthreads();  // the commit's history reads precede the next super-step's writes
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_status(P, sh.D, pit, (int)epoch, nv, lam, c, gamma, prof);
  }
  grid_exit(P.barrier);
}

// ===========================================================================
// The register-tiled kernel on grids of more 32 x 32 tiles than CUs (tiles in
// the last column and row may be narrower, FULL = false: their points outside
// the grid are masked as in the one-tile kernel).  Each block owns a contiguous range
// of tiles and, per super-step, takes every one of them through the same up
// to 16 steps in turn: load the extended tile (from the previous super-step's
// exchange vector) and the state, step in registers exactly as the one-tile
// kernel does, store the owned points.  Because a block may still read the
// previous exchange vector while a faster one writes the next, three of them
// rotate.  The committed value of accumulator k lives in one of two buffers
// (the output, or its workspace) and each super-step writes the speculative
// value into the other: when k ran through the super-step the two swap
// roles.  When it stopped inside, the block runs the super-step again from
// its input (still intact: it is two vectors behind the next write) up to the
// last such stop and adds to the committed value the terms up to each
// accumulator's own stop index, in the forward order -- the same values the
// one-tile kernel takes from its LDS history, without writing a history.
// When the super-step's length comes from the predicted stop, the
// accumulators' values at its last kRegSnap steps but one are also stored:
// a stop there (the likely case) is a copy of the snapshot instead.
// Norm partials are summed over the block's tiles in tile order.
// ===========================================================================
template <int KIND, int KM, bool FULL>
__global__ __launch_bounds__(kRegBlock) void lj_action_regm(ActionParams P) {
  static_assert(KIND == OP_ADVDIFF || KIND == OP_ALLENCAHN, "register-tiled kernel: periodic scalar families");
  constexpr int CH = (KM == 1) ? 5 : 3;
  const GridSync gsync{P.barrier, P.spin_limit};
  __shared__ RegShared sh;
  const OpDev& op = P.op;
  const int K = P.K;
  const int Q = 1 + K;
  const int nx = op.nx, ny = op.ny;
  const size_t N = (size_t)nx * ny;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kTable; i += kRegBlock) sh.xi[i] = P.xi[i];
  const int T = P.ntx * P.nty;
  const int bb = xcd_chunk(blockIdx.x, gridDim.x);
  const int tb0 = (int)((long)bb * T / gridDim.x), tb1 = (int)((long)(bb + 1) * T / gridDim.x);
  const bool owned_wave = wv >= 2 && wv < 6;
  // the tile's owned w x h points at (x0, y0); this wave's owned rows are
  // its first nr (the same for the whole wave)
  int x0 = 0, y0 = 0, w = kRegTile, nr = owned_wave ? kRegRows : 0;
  bool tfull = true;  // the current tile is 32 x 32
  auto set_tile = [&](int t) {
    x0 = (t % P.ntx) * kRegTile;
    y0 = (t / P.ntx) * kRegTile;
    if constexpr (!FULL) {
      w = min(kRegTile, nx - x0);
      const int h = min(kRegTile, ny - y0);
      nr = uniform(owned_wave ? min(kRegRows, max(0, h - kRegRows * (wv - 2))) : 0);
      tfull = w == kRegTile && h == kRegTile;
    }
  };
  // runs body(tag) on the current tile: a ragged grid's full tiles take the
  // unmasked form too (the masks cost registers the steps need)
  auto per_tile = [&](auto&& body) {
    if constexpr (FULL) {
      body(TileTag<true>{});
    } else {
      if (tfull) {
        body(TileTag<true>{});
      } else {
        body(TileTag<false>{});
      }
    }
  };
  // lanes that may own points of the tile (in a full tile: own all 8 rows'),
  // and within them whether row i's point is owned
  const bool own_any = owned_wave && lane >= kRegS && lane < kRegS + kRegTile;
  auto own = [&](auto tg, int i) { return decltype(tg)::full || (lane < kRegS + w && i < nr); };
  // sum of squares of this lane's owned values t[0..7] (owned waves only;
  // the row sums taken there, lanes 16-31 and 32-47, see no other lanes, so
  // a full tile needs no mask)
  auto sq_own = [&](auto tg, const double (&t)[kRegRows]) {
    double a0 = 0.0, a1 = 0.0;
    if (decltype(tg)::full || nr == kRegRows) {
#pragma unroll
      for (int i = 0; i < kRegRows; i += 2) {
        a0 = fma(t[i], t[i], a0);
        a1 = fma(t[i + 1], t[i + 1], a1);
      }
    } else {
#pragma unroll
      for (int i = 0; i < kRegRows; i += 2) {
        const double u0 = i < nr ? t[i] : 0.0, u1 = i + 1 < nr ? t[i + 1] : 0.0;
        a0 = fma(u0, u0, a0);
        a1 = fma(u1, u1, a1);
      }
    }
    const double a = a0 + a1;
    return (decltype(tg)::full || lane < kRegS + w) ? a : 0.0;
  };
  auto gidx = [&](int i) {  // global index of extended point (lane, row 8 wv + i), periodic
    int gx = (x0 - kRegS + lane) % nx;
    if (gx < 0) gx += nx;
    int gy = (y0 - kRegS + kRegRows * wv + i) % ny;
    if (gy < 0) gy += ny;
    return (size_t)gy * nx + gx;
  };
  // owned point of row i (own(i) only; there the same as gidx(i), which a
  // ragged tile's lanes of own_any read from instead: in range everywhere,
  // their values at points not owned are left out of every sum and store)
  auto gown = [&](int i) { return (size_t)(y0 + kRegRows * wv + i - kRegS) * nx + x0 + lane - kRegS; };

  double fw, fe, fs, fn;
  if constexpr (KIND == OP_ALLENCAHN) {
    fw = fe = op.c0 * op.idx2;
    fs = fn = op.c0 * op.idy2;
  } else {
    fw = op.c0 * op.idx2 + op.c1 * op.i2dx;
    fe = op.c0 * op.idx2 - op.c1 * op.i2dx;
    fs = op.c0 * op.idy2 + op.c2 * op.i2dy;
    fn = op.c0 * op.idy2 - op.c2 * op.i2dy;
  }
  const double d_lap = -2.0 * op.c0 * (op.idx2 + op.idy2);
  double dshift = 0.0, dscale = 1.0;  // the diagonal as (e_d - dshift) * dscale
  double x[kRegRows], dg[kRegRows];
  auto load_state = [&]() {
#pragma unroll
    for (int i = 0; i < kRegRows; ++i) {
      double e;
      if constexpr (KIND == OP_ALLENCAHN) {
        const double u = op.state[gidx(i)];
        e = d_lap + (1.0 - 3.0 * u * u);
      } else {
        e = d_lap;
      }
      dg[i] = (dscale == 1.0 && dshift == 0.0) ? e : (e - dshift) * dscale;
    }
  };
  auto yb = [&](int i) { return i == 0 ? P.ybuf0 : (i == 1 ? P.ybuf1 : P.ybuf2); };

  unsigned int epoch = 0;
  int par = 0;
  unsigned long long prof[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long t_last = wall_clock64();
  auto tick = [&](int phase) {
    const unsigned long long t = wall_clock64();
    prof[phase] += t - t_last;
    t_last = t;
  };
  auto point = [&](int i, double xs, double xn, double xim) {
    const double xc = x[i];
    const double xw = dpp_move<0x138>(xc);
    const double xe = dpp_move<0x130>(xc);
    double y;
    if constexpr (KIND == OP_ALLENCAHN) {
      y = fw * (xw + xe) + fs * (xs + xn);
    } else {
      y = fw * xw + fe * xe + fs * xs + fn * xn;
    }
    return fma(dg[i] - xim, xc, y);
  };
  auto step = [&](double xim) {
    double* xr = &sh.xrow[par][0][0];
    xr[(2 * wv) * 64 + lane] = x[0];
    xr[(2 * wv + 1) * 64 + lane] = x[kRegRows - 1];
    __syncthreads();
    const double above = xr[(2 * ((wv + kRegWaves - 1) % kRegWaves) + 1) * 64 + lane];
    const double below = xr[(2 * ((wv + 1) % kRegWaves)) * 64 + lane];
    par ^= 1;
    double y[kRegRows];
#pragma unroll
    for (int i = 1; i < kRegRows - 1; ++i) y[i] = point(i, x[i - 1], x[i + 1], xim);
    y[0] = point(0, above, x[1], xim);
    y[kRegRows - 1] = point(kRegRows - 1, x[kRegRows - 2], below, xim);
#pragma unroll
    for (int i = 0; i < kRegRows; ++i) x[i] = y[i];
  };
  auto sumsq = [&](auto tg) { return sq_own(tg, x); };  // owned waves: this lane's owned points
  // add this tile's sums of slots (one value per owned wave) to the staging area
  auto stage_add = [&](int slot, double a) {
    const double t = row_sum(a);
    const double u = read_lane(t, 31) + read_lane(t, 47);
    if (lane == 0) sh.stg[slot][wv - 2] += u;
  };
  auto zero_stage = [&](int nq) {
    for (int q = threadIdx.x; q < nq * 4; q += kRegBlock) sh.stg[q >> 2][q & 3] = 0.0;
    __syncthreads();
  };
  auto publish = [&](int nq) {
    __syncthreads();
    double* area = reg_area(P.partials, epoch);
    for (int q = threadIdx.x; q < nq; q += kRegBlock) {
      const double t = (sh.stg[q][0] + sh.stg[q][1]) + (sh.stg[q][2] + sh.stg[q][3]);
      store_shared(area + (size_t)q * gridDim.x + blockIdx.x, t);
    }
    return area;
  };
  auto put_owned = [&](auto tg, double* dst) {
    if (own_any) {
#pragma unroll
      for (int i = 0; i < kRegRows; ++i)
        if (own(tg, i)) store_shared(dst + gown(i), x[i]);
    }
  };

  // ---- (1) spectral bound: up to 16 products per super-step over all tiles,
  // normalised per super-step
  double lam = (P.lam_src != nullptr && !P.do_power) ? *P.lam_src : P.lam_in;
  if (skip_launch(P, lam, prof)) return;
  int pit = 0;
  int r = 0;  // exchange vector read this super-step; the next one is written
  if (P.do_power) {
    int done = 0;
    double sc = 1.0;
    while (done < P.power_iters) {
      const int steps = min(kRegS, P.power_iters - done);
      zero_stage(2);  // the two norms read: before and after the last product
      for (int t = tb0; t < tb1; ++t) {
        set_tile(t);
        per_tile([&](auto tg) {
          load_state();
#pragma unroll
          for (int i = 0; i < kRegRows; ++i) {
            const size_t g = gidx(i);
            x[i] = (done == 0) ? (P.start ? P.start[g] : 0.5 + splitmix_uniform(P.seed, (uint64_t)g))
                               : sc * yb(r)[g];
          }
          if (owned_wave && steps == 1) stage_add(0, sumsq(tg));
          for (int j = 1; j <= steps; ++j) {
            step(0.0);
            if (owned_wave && j >= steps - 1) stage_add(j - (steps - 1), sumsq(tg));
          }
          put_owned(tg, yb((r + 1) % 3));
        });
      }
      double* area = publish(2);
      grid_allreduce(gsync, epoch, nullptr, 0, nullptr);
      reg_reduce<CH>(area, 2, sh.tot);
      const double nprev = sh.tot[0], nlast = sh.tot[1];
      done += steps;
      pit = done;
      lam = sqrt(nlast) / sqrt(nprev);
      if (nlast == 0.0) {
        lam = 0.0;
        break;
      }
      sc = 1.0 / sqrt(nlast);
      r = (r + 1) % 3;
    }
  }
  lam = uniform(lam);
  if (P.lam_out != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *P.lam_out = lam;
  double c, gamma;
  interval(lam, P.safety, c, gamma);
  const double rgamma = uniform(1.0 / gamma);
  tick(kProfPower);
  if (K == 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      Decision D;
      decision_init(D, 0, 1.0, 0.0, sh.fmax);
      store_status(P, D, pit, (int)epoch, 0.0, lam, c, gamma, prof);
    }
    grid_exit(P.barrier);
    return;
  }
  fw *= rgamma;
  fe *= rgamma;
  fs *= rgamma;
  fn *= rgamma;
  dshift = c;
  dscale = rgamma;

  // ---- (2) divided differences
  __syncthreads();
  DivDiff dd;
  dd_init_par(dd, K, P.l, P.s, P.max_points + 1, c, gamma, sh.xi, sh.coef, sh.fmax);
  dd_advance(dd, K, kRegS, sh.xi, sh.coef);
  __syncthreads();
  tick(kProfDivdiff);

  // ---- (3) Newton recurrence in super-steps of up to 16 over all tiles
  if (threadIdx.x == 0) decision_init(sh.D, K, 1.0, 0.0, sh.fmax);  // redone once ||v|| is known
  __syncthreads();
  double nv = 0.0;
  bool first = true;
  int m0 = 0;
  bool cpar[KM], fin[KM];  // committed value in the workspace / final value in the output
#pragma unroll
  for (int k = 0; k < KM; ++k) cpar[k] = fin[k] = false;
  const double* src = P.v;  // input of the current super-step
  // run the current super-step again from its input for the accumulators in
  // `sel`, adding to each committed value its terms up to its own stop index
  // ck[k] (<= cmax), and write the sums to the outputs
  auto replay = [&](const bool* sel, const int* ck, int cmax) {
    double cf[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) cf[k] = (sel[k] && lane < ck[k]) ? sh.coef[k * kTable + m0 + 1 + lane] : 0.0;
    const double xiv = (lane < cmax) ? sh.xi[m0 + lane] : 0.0;
    for (int t = tb0; t < tb1; ++t) {
      set_tile(t);
      per_tile([&](auto tg) {
        load_state();
#pragma unroll
        for (int i = 0; i < kRegRows; ++i) x[i] = src[gidx(i)];
        double ps[KM][kRegRows];
        if (own_any) {
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            if (!sel[k]) continue;
            const double* cb = cpar[k] ? P.pw[k] : P.p[k];
#pragma unroll
            for (int i = 0; i < kRegRows; ++i) ps[k][i] = cb[decltype(tg)::full ? gown(i) : gidx(i)];
          }
        }
        for (int j = 1; j <= cmax; ++j) {
          step(read_lane(xiv, j - 1));
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            if (!sel[k] || j > ck[k]) continue;
            const double dk = read_lane(cf[k], j - 1);
            if (own_any) {
#pragma unroll
              for (int i = 0; i < kRegRows; ++i) ps[k][i] = ps[k][i] + dk * x[i];
            }
          }
        }
        if (own_any) {
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            if (!sel[k]) continue;
#pragma unroll
            for (int i = 0; i < kRegRows; ++i)
              if (own(tg, i)) P.p[k][gown(i)] = ps[k][i];
          }
        }
      });
    }
  };
  while (true) {
    const int pred = min(uniform(sh.D.next), uniform(sh.D.next_local));  // predicted last stop (+1)
    const int steps = min(min(kRegS, P.max_points - m0), pred);
    bool act0[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) act0[k] = (k < K) && (uniform(sh.D.st[k]) == ACC_RUNNING);
    const double xiv = (lane < steps) ? sh.xi[m0 + lane] : 0.0;
    double cfv[KM];
#pragma unroll
    for (int k = 0; k < KM; ++k) cfv[k] = (lane < steps && act0[k]) ? sh.coef[k * kTable + m0 + 1 + lane] : 0.0;
    const int nq = steps * Q + (first ? 1 : 0);
    src = first ? P.v : yb(r);
    const bool snap = pred <= kRegS;  // the length is the predicted stop
    zero_stage(nq);
    for (int t = tb0; t < tb1; ++t) {
      set_tile(t);
      per_tile([&](auto tg) {
        load_state();
#pragma unroll
        for (int i = 0; i < kRegRows; ++i) x[i] = src[gidx(i)];
        double ps[KM][kRegRows];
        if (own_any) {
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            if (!act0[k]) continue;
            if (first) {
              const double d0 = sh.coef[k * kTable];
#pragma unroll
              for (int i = 0; i < kRegRows; ++i) {
                ps[k][i] = d0 * x[i];
                if (own(tg, i)) P.p[k][gown(i)] = ps[k][i];  // the committed value p_k = d_{k,0} v
              }
            } else {
              const double* cb = cpar[k] ? P.pw[k] : P.p[k];
#pragma unroll
              for (int i = 0; i < kRegRows; ++i) ps[k][i] = cb[decltype(tg)::full ? gown(i) : gidx(i)];
            }
          }
        }
        if (first && owned_wave) stage_add(steps * Q, sumsq(tg));
        for (int j = 1; j <= steps; ++j) {
          step(read_lane(xiv, j - 1));
          if (owned_wave) {
            double tq[1 + KM];
            tq[0] = sumsq(tg);
#pragma unroll
            for (int k = 0; k < KM; ++k) {
              const double dk = read_lane(cfv[k], j - 1);
#pragma unroll
              for (int i = 0; i < kRegRows; ++i) ps[k][i] = ps[k][i] + dk * x[i];
              tq[1 + k] = sq_own(tg, ps[k]);
            }
            const int d = steps - j;  // snapshot d - 1 holds the values after step m0 + j
            if (snap && d >= 1 && d <= kRegSnap && own_any) {
#pragma unroll
              for (int k = 0; k < KM; ++k) {
                if (!act0[k]) continue;
                double* sn = P.snap + (size_t)(k * kRegSnap + d - 1) * N;
#pragma unroll
                for (int i = 0; i < kRegRows; ++i)
                  if (own(tg, i)) sn[gown(i)] = ps[k][i];
              }
            }
#pragma unroll
            for (int q = 0; q < 1 + KM; ++q) tq[q] += dpp_move<0x111>(tq[q]);
#pragma unroll
            for (int q = 0; q < 1 + KM; ++q) tq[q] += dpp_move<0x112>(tq[q]);
#pragma unroll
            for (int q = 0; q < 1 + KM; ++q) tq[q] += dpp_move<0x114>(tq[q]);
#pragma unroll
            for (int q = 0; q < 1 + KM; ++q) tq[q] += dpp_move<0x118>(tq[q]);
            double uq[1 + KM];
#pragma unroll
            for (int q = 0; q < 1 + KM; ++q) uq[q] = read_lane(tq[q], 31) + read_lane(tq[q], 47);
            if (lane == 0) {
              sh.stg[(j - 1) * Q][wv - 2] += uq[0];
#pragma unroll
              for (int k = 0; k < KM; ++k)
                if (k < K) sh.stg[(j - 1) * Q + 1 + k][wv - 2] += uq[1 + k];
            }
          }
        }
        put_owned(tg, yb((r + 1) % 3));
        if (own_any) {  // the speculative values go to the buffer that is not the committed one
#pragma unroll
          for (int k = 0; k < KM; ++k) {
            if (!act0[k]) continue;
            double* sb = cpar[k] ? P.p[k] : P.pw[k];
#pragma unroll
            for (int i = 0; i < kRegRows; ++i)
              if (own(tg, i)) sb[gown(i)] = ps[k][i];
          }
        }
      });
    }
    tick(kProfSteps);
    double* area = publish(nq);
    tick(kProfPublish);
    grid_allreduce(gsync, epoch, nullptr, 0, nullptr,
                   [&] { dd_advance(dd, K, m0 + steps + kRegS, sh.xi, sh.coef); });
    reg_reduce<CH>(area, nq, sh.tot);
    tick(kProfBarrier);
    if (threadIdx.x < 64) {
      if (first) {
        nv = sqrt(sh.tot[steps * Q]);
        decision_init(sh.D, K, nv, P.hump, sh.fmax);
      }
      replay_decisions(sh.D, K, m0, steps, Q, sh.tot, sh.coef, P.tol, P.relative, P.max_points, sh.commit,
                       blockIdx.x == 0 ? P.status->trace : nullptr);
    }
    __syncthreads();
    tick(kProfDecide);
    // commit: a run-through accumulator's speculative buffer becomes the
    // committed one; those that stopped inside the super-step take the
    // committed value plus the terms up to their stop index (forward order),
    // formed by running the super-step again up to the last such stop
    bool redo[KM], fromsnap[KM];
    int ck[KM];
    int cmax = -1;
    bool anysnap = false;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      ck[k] = act0[k] ? uniform(sh.commit[k]) : 0;
      const bool in = act0[k] && ck[k] < steps;
      fromsnap[k] = in && snap && ck[k] >= 1 && steps - ck[k] <= kRegSnap;
      redo[k] = in && !fromsnap[k];
      anysnap = anysnap || fromsnap[k];
      if (redo[k]) cmax = max(cmax, ck[k]);
      if (act0[k] && !in) cpar[k] = !cpar[k];
    }
    if (anysnap) {
      for (int t = tb0; t < tb1; ++t) {
        set_tile(t);
        if (!own_any) continue;
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (!fromsnap[k]) continue;
          const double* sn = P.snap + (size_t)(k * kRegSnap + steps - ck[k] - 1) * N;
#pragma unroll
          for (int i = 0; i < kRegRows; ++i)
            if (own(TileTag<FULL>{}, i)) P.p[k][gown(i)] = sn[gown(i)];
        }
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (!fromsnap[k]) continue;
        fin[k] = true;
        cpar[k] = false;
      }
    }
    if (cmax >= 0) {
      if constexpr (KM == 1) {
        replay(redo, ck, cmax);
      } else {
        // one accumulator at a time keeps the register state of the
        // four-accumulator instance within the file
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (!redo[k]) continue;
          bool one[KM];
#pragma unroll
          for (int q = 0; q < KM; ++q) one[q] = (q == k);
          replay(one, ck, ck[k]);
        }
      }
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        if (!redo[k]) continue;
        fin[k] = true;
        cpar[k] = false;
      }
    }
    m0 += steps;
    r = (r + 1) % 3;
    first = false;
    tick(kProfCommit);
    if (sh.D.n_active == 0 || m0 >= P.max_points) break;
    __syncthreads();
  }
  // accumulators whose committed value sits in the workspace: to the output
#pragma unroll
  for (int k = 0; k < KM; ++k) {
    if (k >= K || fin[k] || !cpar[k]) continue;
    for (int t = tb0; t < tb1; ++t) {
      set_tile(t);
      if (!own_any) continue;
#pragma unroll
      for (int i = 0; i < kRegRows; ++i)
        if (own(TileTag<FULL>{}, i)) P.p[k][gown(i)] = P.pw[k][gown(i)];
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    store_status(P, sh.D, pit, (int)epoch, nv, lam, c, gamma, prof);
  }
  grid_exit(P.barrier);
}

// ---------------------------------------------------------------------------
// Stand-alone divided differences (the lj_divided_differences entry point);
// the same dd_init / dd_advance the action kernels run.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void lj_divdiff_kernel(DDParams P) {
  __shared__ double xi[kTable];
  __shared__ double coef[kMaxK * kTable];
  __shared__ double fm[kMaxK];
  for (int i = threadIdx.x; i < kTable; i += blockDim.x) xi[i] = P.xi[i];
  __syncthreads();
  DivDiff dd;
  dd_init(dd, P.K, P.l, P.s, P.npts, P.c, P.gamma, xi, coef, fm);
  dd_advance(dd, P.K, P.npts - 1, xi, coef);
  __syncthreads();
  for (int i = threadIdx.x; i < P.K * kTable; i += blockDim.x) P.coef[i] = coef[i];
  if ((int)threadIdx.x < P.K) P.fmax[threadIdx.x] = fm[threadIdx.x];
}

// ===========================================================================
// Batched actions (the batching form): many independent instances; each is
// run from start to end -- power iteration, divided differences and the whole
// Newton recurrence with its stop decisions -- by one team of blocks.  A team
// is `team` blocks that run on one XCD (blocks b, b + 8, b + 16, ... of a
// launch are dispatched to the same XCD, so they share its L2) and
// synchronise through a counter of their own: no grid-wide barrier.  Each member streams its chunk of the instance's
// points, team reductions sum the members' partials in rank order, and every
// member takes the same stop decisions.  Team leaders take instances from a
// work queue (one atomic counter) in the order the host gives (largest
// first), so the long instances start first and short ones fill the tail.
// The arithmetic of every step is that of lj_action_stream.
// ===========================================================================

// Team barrier: drain this block's stores, arrive on the team counter, wait
// for all members, then an agent-scope acquire drops stale cache lines.  The
// wait is bounded: the host launches only schedules whose blocks are all
// co-resident, but should a member never arrive, the waiting block raises the
// batch's abort word (and every later wait returns at once), so the launch
// ends and the host reports the failure instead of the device hanging.
constexpr unsigned int kTeamSpinLimit = 1u << 22;

__device__ __forceinline__ void team_barrier(unsigned int* ctr, unsigned int& epoch, int T,
                                             unsigned int* abort_word) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (T == 1) return;
  epoch += 1u;
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    unsigned int spins = 0;
    while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch * (unsigned int)T) {
      if (__hip_atomic_load(abort_word, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
      if (++spins > kTeamSpinLimit) {
        __hip_atomic_store(abort_word, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

template <int KIND, int NC, int BS>
__global__ __launch_bounds__(BS) void lj_batch_kernel(BatchParams B) {
  constexpr int NW = BS / 64;
  // two points in flight per thread where the register budget allows it
  constexpr int kBatchUnroll = (BS >= 1024) ? 1 : 2;
  __shared__ double xi[kTable];
  __shared__ double coef[kMaxK * kTable];
  __shared__ double fmaxk[kMaxK];
  __shared__ double red[kQ * NW + kQ];
  __shared__ double tot[kQ];
  __shared__ Decision sD;
  __shared__ int s_commit[kMaxK];
  __shared__ double s_s[kMaxK];   // (l, s) of the accumulators of the running recurrence
  __shared__ int s_l[kMaxK];
  __shared__ double s_s0[kMaxK];  // a_k h of the instance
  __shared__ int s_flag;
  __shared__ int s_iters, s_accum, s_vecs, s_rej;  // the instance's running counts
  __shared__ int f_state[kMaxK], f_mst[kMaxK], f_sub[kMaxK];
  __shared__ double f_err[kMaxK];
  for (int i = threadIdx.x; i < kTable; i += BS) xi[i] = B.xi[i];
  const int K = B.K;
  const int T = B.team;
  // team geometry: members share blockIdx.x % 8 (one XCD)
  const int grp = blockIdx.x & 7, q8 = blockIdx.x >> 3;
  const int rank = q8 % T;
  const int team = (q8 / T) * 8 + grp;
  unsigned int* tw = B.team_words + (size_t)team * kTeamWords;
  unsigned int* ctr = tw;
  unsigned int* mailbox = tw + 16;
  double* tpart = B.team_part + (size_t)team * 2 * kQ * T;
  unsigned int tepoch = 0;
  // team all-reduce of nq block totals (LDS, as block_sum leaves them) into
  // tot[0..nq): members' values added in rank order
  auto team_sum = [&](const double* btot, int nq) {
    if (T == 1) {
      if ((int)threadIdx.x < nq) tot[threadIdx.x] = btot[threadIdx.x];
      __syncthreads();
      return;
    }
    double* area = tpart + (size_t)(tepoch & 1u) * kQ * T;
    if ((int)threadIdx.x < nq) area[threadIdx.x * T + rank] = btot[threadIdx.x];
    team_barrier(ctr, tepoch, T, B.queue + 1);
    if ((int)threadIdx.x < nq) {
      double t = 0.0;
      for (int r = 0; r < T; ++r) t += area[threadIdx.x * T + r];
      tot[threadIdx.x] = t;
    }
    __syncthreads();
  };

  for (;;) {
    if (rank == 0 && threadIdx.x == 0) {
      const unsigned int job = atomicAdd(B.queue, 1u);
      __hip_atomic_store(mailbox, job, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_flag = (int)job;
    }
    team_barrier(ctr, tepoch, T, B.queue + 1);
    if (threadIdx.x == 0 && rank != 0) s_flag = (int)__hip_atomic_load(mailbox, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int job = uniform(s_flag);
    if (job >= B.n) break;
    const unsigned long long t_start = wall_clock64();
    const int inst = uniform(B.order[job]);
    const BatchItem* __restrict__ it = B.items + inst;
    const OpDev op = it->op;
    const int npts = op.npts;
    // this member's chunk of the points
    const int chunk = ((npts + T - 1) / T + 63) & ~63;
    const int pb = min(npts, rank * chunk), pe = min(npts, pb + chunk);
    double* y0 = it->y0;
    double* y1 = it->y1;
    const double* v = it->v;
    double* pp[kMaxK];
#pragma unroll
    for (int k = 0; k < kMaxK; ++k) pp[k] = (k < K) ? it->p[k] : nullptr;
    if (threadIdx.x < kMaxK) {
      s_s[threadIdx.x] = ((int)threadIdx.x < K) ? it->s[threadIdx.x] : 0.0;
      s_s0[threadIdx.x] = s_s[threadIdx.x];
    }

    // (1) spectral bound
    double lam = it->lam_in;
    int pit = 0;
    if (!(lam > 0.0)) {
      for (int p = pb + (int)threadIdx.x; p < pe; p += BS)
#pragma unroll
        for (int cc = 0; cc < NC; ++cc)
          store_shared(y1 + NC * p + cc, 0.5 + splitmix_uniform(B.seed, (uint64_t)(NC * p + cc)));
      team_barrier(ctr, tepoch, T, B.queue + 1);
      double scale = 1.0;
      for (int k = 0; k < B.power_iters; ++k) {
        const double* src = (k & 1) ? y0 : y1;
        double* dst = (k & 1) ? y1 : y0;
        double w2[2] = {0.0, 0.0};
        power_pass<KIND, NC, true, kBatchUnroll>(op, src, dst, scale, pb + (int)threadIdx.x, pe, BS, w2[0], w2[1]);
        block_sum<2>(w2, red);
        team_sum(red + 2 * NW, 2);
        const double nx = sqrt(tot[0]);
        const double ny = sqrt(tot[1]);
        lam = ny / nx;
        pit = k + 1;
        if (ny == 0.0) {
          lam = 0.0;
          break;
        }
        scale = 1.0 / ny;
      }
    }
    lam = uniform(lam);
    double c, gamma;
    interval(lam, B.safety, c, gamma);
    const double rgamma = uniform(1.0 / gamma);

    // out = sum_q alpha[q] x_q over this member's points (write-through
    // stores: the next recurrence reads out at the neighbours), then a team
    // barrier; the same rounding as the library's linear combinations
    auto combine = [&](double* out, int nin, const double* alpha, const double* const* xs) {
      for (int p = pb + (int)threadIdx.x; p < pe; p += BS) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const int idx = NC * p + cc;
          double t = alpha[0] * xs[0][idx];
          for (int q = 1; q < nin; ++q) t = fma(alpha[q], xs[q][idx], t);
          store_shared(out + idx, t);
        }
      }
      if (threadIdx.x == 0) s_vecs += nin + 1;
      team_barrier(ctr, tepoch, T, B.queue + 1);
    };

    // (2)-(5) the instance's Newton recurrences, one after another through
    // one recurrence body:
    //   phase 0: the shared basis, outputs w_k = phi_{l_k}(a_k h J) v;
    // then each accumulator the shared basis rejected is redone alone with
    // s = 2, 4, ... substeps of tau = a_k h / s, advancing
    // w(t) = t^l phi_l(t J) v by w(t + tau) = e^{tau J} w(t)
    //   + sum_j tau^j t^{l-j} / (l-j)! phi_j(tau J) v (the result scaled by (a_k h)^l):
    //   phase 1 (l > 0): phi_1..phi_l of tau J on v in one recurrence,
    //            then w = phi_l / s^l,
    //   phase 2: exponential number i of tau J (l > 0: on w, then w = e +
    //            the phi_j terms, i = 1 .. s-1; l = 0: the chain from v,
    //            i = 0 .. s-1).
    if (threadIdx.x < kMaxK) {
      s_l[threadIdx.x] = B.l[threadIdx.x];
      f_sub[threadIdx.x] = 1;
    }
    if (threadIdx.x == 0) {
      s_iters = 0;
      s_accum = 0;
      s_vecs = 0;
      s_rej = 0;
    }
    double nv = 0.0;
    int phase = 0, kk = -1, lk = 0, ns = 1, si = 0, used0 = 0;
    double tau = 0.0;
    double* const sub0 = it->sub;
    const size_t stride = it->nsub_stride;
#pragma unroll 1
    for (;;) {
      // ---- the recurrence of this phase: input, accumulators, outputs
      const double* vin = v;
      int Kr = K;
      double* outs[kMaxK];
#pragma unroll
      for (int k = 0; k < kMaxK; ++k) outs[k] = pp[k];
      if (phase == 1) {
        Kr = lk;
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) outs[k] = (k < lk) ? sub0 + (size_t)k * stride : nullptr;
        if (threadIdx.x < kMaxK) {
          s_l[threadIdx.x] = threadIdx.x + 1;
          s_s[threadIdx.x] = tau;
        }
      } else if (phase == 2) {
        Kr = 1;
        if (lk > 0) {
          vin = pp[kk];
          outs[0] = sub0 + (size_t)lk * stride;
        } else {
          vin = (si == 0) ? v : (((si - 1) & 1) ? sub0 + stride : sub0);
          outs[0] = (si == ns - 1) ? pp[kk] : ((si & 1) ? sub0 + stride : sub0);
        }
        if (threadIdx.x == 0) {
          s_l[0] = 0;
          s_s[0] = tau;
        }
      }
      __syncthreads();
      {
        DivDiff dd;
        dd_init(dd, Kr, s_l, s_s, B.max_points + 1, c, gamma, xi, coef, fmaxk);
        dd_advance(dd, Kr, B.max_points, xi, coef);
      }
      __syncthreads();
      // m = 0: p_k = d_{k,0} v and ||v||^2
      double a0[1] = {0.0};
      for (int p = pb + (int)threadIdx.x; p < pe; p += BS) {
#pragma unroll
        for (int cc = 0; cc < NC; ++cc) {
          const int idx = NC * p + cc;
          const double vv = vin[idx];
          a0[0] += vv * vv;
#pragma unroll
          for (int k = 0; k < kMaxK; ++k)
            if (k < Kr) outs[k][idx] = coef[k * kTable] * vv;
        }
      }
      block_sum<1>(a0, red);
      team_sum(red + NW, 1);
      if (phase == 0) nv = sqrt(tot[0]);
      if (threadIdx.x < 64) decision_init(sD, Kr, sqrt(tot[0]), B.hump, fmaxk);
      __syncthreads();
      // Newton steps
      const double* src = vin;
      for (int m = 1; m <= B.max_points && uniform(sD.n_active) > 0; ++m) {
        double* dst = (m & 1) ? y1 : y0;
        const double xim = uniform(xi[m - 1]);
        double dk[kMaxK];
        bool act[kMaxK];
#pragma unroll
        for (int k = 0; k < kMaxK; ++k) {
          act[k] = (k < Kr) && (uniform(sD.st[k]) == ACC_RUNNING);
          dk[k] = act[k] ? uniform(coef[k * kTable + m]) : 0.0;
        }
        double acc[kQ] = {0.0, 0.0, 0.0, 0.0, 0.0};
        newton_pass<KIND, NC, true, kBatchUnroll>(op, src, dst, outs, act, dk, c, gamma, rgamma, xim,
                                                  pb + (int)threadIdx.x, pe, BS, acc);
        block_sum<kQ>(acc, red);
        team_sum(red + kQ * NW, 1 + Kr);
        if (threadIdx.x < 64)
          replay_decisions(sD, Kr, m - 1, 1, 1 + Kr, tot, coef, B.tol, B.relative, B.max_points, s_commit, nullptr);
        __syncthreads();
        src = dst;
      }
      if (threadIdx.x == 0) {
        s_iters += sD.iters;
        s_accum += sD.accum_iters;
      }
      __syncthreads();

      // ---- what follows this recurrence
      bool next_acc = false;  // go on with the next rejected accumulator
      bool attempt_failed = false;
      if (phase == 0) {
        if (threadIdx.x < kMaxK) {
          const int k = threadIdx.x;
          f_state[k] = (k < K) ? sD.st[k] : ACC_CONVERGED;
          f_mst[k] = (k < K) ? sD.mst[k] : -1;
          f_err[k] = (k < K) ? sD.err[k] : 0.0;
        }
        __syncthreads();
        bool any = false;
#pragma unroll 1
        for (int k = 0; k < K; ++k) any = any || (uniform(f_state[k]) != ACC_CONVERGED);
        if (any && threadIdx.x == 0) s_rej = 1;
        next_acc = true;
      } else if (phase == 1) {
        bool ok = true;
#pragma unroll 1
        for (int j = 0; j < lk; ++j) ok = ok && (uniform(sD.st[j]) == ACC_CONVERGED);
        if (ok) {
          double sl = 1.0;  // s^l, exact
#pragma unroll 1
          for (int j = 0; j < lk; ++j) sl *= (double)ns;
          const double a1[1] = {1.0 / sl};
          const double* x1[1] = {sub0 + (size_t)(lk - 1) * stride};
          combine(pp[kk], 1, a1, x1);
          phase = 2;
          si = 1;
          if (si == ns) next_acc = true;  // (s >= 2 here, so never)
        } else {
          attempt_failed = true;
        }
      } else {
        if (uniform(sD.st[0]) != ACC_CONVERGED) {
          attempt_failed = true;
        } else {
          if (lk > 0) {
            double sl = 1.0;
#pragma unroll 1
            for (int j = 0; j < lk; ++j) sl *= (double)ns;
            double al[1 + kMaxK];
            const double* xs[1 + kMaxK];
            al[0] = 1.0;
            xs[0] = sub0 + (size_t)lk * stride;
            double fact = 1.0;  // (l - j)!
#pragma unroll 1
            for (int j = lk; j >= 1; --j) {
              if (j < lk) fact *= (double)(lk - j);
              double ip = 1.0;  // i^(l-j), exact
#pragma unroll 1
              for (int q = 0; q < lk - j; ++q) ip *= (double)si;
              al[j] = ip / (fact * sl);
              xs[j] = sub0 + (size_t)(j - 1) * stride;
            }
            combine(pp[kk], lk + 1, al, xs);
          }
          si += 1;
          if (si == ns) {  // the attempt succeeded
            if (threadIdx.x == 0) {
              f_state[kk] = ACC_CONVERGED;
              f_mst[kk] = s_iters - used0;
              f_err[kk] = 0.0;
              f_sub[kk] = ns;
            }
            next_acc = true;
          }
        }
      }
      if (attempt_failed) {
        if (threadIdx.x == 0) s_rej += 1;
        ns *= 2;
        if (ns > B.max_substeps) {
          if (threadIdx.x == 0) {
            f_mst[kk] = -1;
            f_sub[kk] = ns / 2;
          }
          next_acc = true;
        }
      }
      __syncthreads();
      if (next_acc) {  // the next accumulator the shared basis rejected, if any
        int k = kk + 1;
#pragma unroll 1
        for (;;) {
          while (k < K && uniform(f_state[k]) == ACC_CONVERGED) ++k;
          if (k >= K || B.max_substeps >= 2) break;
          ++k;  // no substeps allowed: it stays rejected (m* -1, s 1)
        }
        if (k >= K) break;
        kk = k;
        lk = B.l[k];
        ns = 2;
      }
      if (next_acc || attempt_failed) {  // start an attempt at ns substeps
        tau = uniform(s_s0[kk]) / (double)ns;
        phase = (lk > 0) ? 1 : 2;
        si = 0;
        used0 = uniform(s_iters);
      }
    }

    // (6) outcome of this instance
    if (rank == 0 && threadIdx.x == 0) {
      BatchStatus* S = B.status + inst;
#pragma unroll
      for (int k = 0; k < kMaxK; ++k) {
        S->state[k] = f_state[k];
        S->m_star[k] = f_mst[k];
        S->err[k] = f_err[k];
        S->substeps[k] = f_sub[k];
      }
      S->iters = s_iters;
      S->accum_iters = s_accum;
      S->vec_passes = s_vecs;
      S->rejections = s_rej;
      S->power_iters = pit;
      S->vnorm = nv;
      S->lam = lam;
      S->c = c;
      S->gamma = gamma;
      S->block = blockIdx.x;
      S->t0 = t_start;
      S->t1 = wall_clock64();
    }
  }
}

// zeroes n words (graph-capturable replacement of a memset node)
__global__ void lj_fill_u32(unsigned int* p, int n, unsigned int v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// Streaming helpers.
// ---------------------------------------------------------------------------
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

// out = alpha_0 x_0, then out = fma(alpha_q, x_q, out) for q = 1, 2, ...
__global__ __launch_bounds__(256) void lj_lincomb_kernel(LinComb L) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < L.n; i += (long)gridDim.x * blockDim.x) {
    double s = L.alpha[0] * L.x[0][i];
    for (int q = 1; q < L.nin; ++q) s = fma(L.alpha[q], L.x[q][i], s);
    L.out[i] = s;
  }
}

// f = f(u) and v = h f in one pass (the first stage of every scheme)
template <int KIND, int NC>
__global__ __launch_bounds__(256) void lj_rhs_scaled_kernel(OpDev op, double h, double* __restrict__ f,
                                                            double* __restrict__ v) {
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < op.npts; p += gridDim.x * blockDim.x) {
    double out[2];
    rhs_point<KIND>(op, op.state, p, out);
#pragma unroll
    for (int cc = 0; cc < NC; ++cc) {
      f[NC * p + cc] = out[cc];
      v[NC * p + cc] = h * out[cc];
    }
  }
}

// The stage arguments of the exponential Rosenbrock / EPIRK schemes in one
// pass: up to two remainders R_r = f(x_r) - f(u) - J(u)(x_r - u) (Sec. 1) at
// x_r = u + sum_t a[r][t] X[r][t], formed point by point (x_r and x_r - u are
// recomputed at the stencil neighbours from u and the X's), then up to two
// combinations of R_0, R_1 and an extra vector P.  Each combination is formed
// as the linear-combination kernel forms one (a product, then FMAs in order).
template <int KIND, int NC>
__global__ __launch_bounds__(256) void lj_stage_kernel(StageArgs A) {
  const OpDev& op = A.op;
  const double* __restrict__ u = op.state;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < op.npts; p += gridDim.x * blockDim.x) {
    int idx[5] = {p, p, p, p, p};
    if constexpr (KIND != OP_DIAG) {
      const Nbr q = neighbours<KIND>(op, p);
      idx[1] = q.w;
      idx[2] = q.e;
      idx[3] = q.s;
      idx[4] = q.n;
    }
    constexpr int NT = (KIND == OP_DIAG) ? 1 : 5;
    double uv[5][2] = {};
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c) uv[t][c] = u[NC * idx[t] + c];
    double R[2][2] = {};
    for (int r = 0; r < A.nrem; ++r) {
      double xv[5][2] = {}, dv[5][2] = {};
#pragma unroll
      for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int i = NC * idx[t] + c;
          double x = 1.0 * uv[t][c];
          x = fma(A.a[r][0], A.X[r][0][i], x);
          if (A.nterm[r] > 1) x = fma(A.a[r][1], A.X[r][1][i], x);
          xv[t][c] = x;
          dv[t][c] = fma(-1.0, uv[t][c], 1.0 * x);
        }
      double fx[2], jd[2];
      rhs_values<KIND>(op, xv, uv[0][0], fx);
      stencil_jv<KIND>(op, dv, uv, jd);
#pragma unroll
      for (int c = 0; c < NC; ++c) R[r][c] = (fx[c] - A.fu[NC * p + c]) - jd[c];
    }
    for (int o = 0; o < A.nout; ++o) {
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const int i = NC * p + c;
        auto src = [&](int t) { return A.src[o][t] == 2 ? A.P[i] : R[A.src[o][t]][c]; };
        double y = A.c[o][0] * src(0);
        if (A.nsrc[o] > 1) y = fma(A.c[o][1], src(1), y);
        A.out[o][i] = y;
      }
    }
  }
}

// The step's result from its stages: u3 = u + X1 (+ X2); with X3,
// u_out = u3 + X3 and err = u_out - u3; without, u_out = u3 and err = 0 u + 0 u
// (the same operations as the linear-combination kernel's).
__global__ __launch_bounds__(256) void lj_finish_kernel(FinishArgs F) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < F.n; i += (long)gridDim.x * blockDim.x) {
    const double uu = F.u[i];
    double u3 = 1.0 * uu;
    u3 = fma(1.0, F.X1[i], u3);
    if (F.X2) u3 = fma(1.0, F.X2[i], u3);
    if (F.X3) {
      const double uo = fma(1.0, F.X3[i], 1.0 * u3);
      F.u_out[i] = uo;
      if (F.err) F.err[i] = fma(-1.0, u3, 1.0 * uo);
    } else {
      F.u_out[i] = u3;
      if (F.err) F.err[i] = fma(0.0, uu, 0.0 * uu);
    }
  }
}

// Sums of squares of two vectors (the step controller's error and solution
// norms), in a fixed order: block g sums a contiguous chunk (thread t every
// 256th value from t, then the waves' DPP sums in wave order) into
// part[2 g], part[2 g + 1]; one block then adds the partials in block order.
__global__ __launch_bounds__(256) void lj_sumsq2_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                         long n, double* __restrict__ part) {
  __shared__ double red[2 * 4];
  const long chunk = (n + gridDim.x - 1) / gridDim.x;
  const long i0 = blockIdx.x * chunk, i1 = min(n, i0 + chunk);
  double sa = 0.0, sb = 0.0;
  for (long i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    sa += a[i] * a[i];
    sb += b[i] * b[i];
  }
  sa = wave_sum(sa);
  sb = wave_sum(sb);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    red[2 * w] = sa;
    red[2 * w + 1] = sb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double ta = 0.0, tb = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      ta += red[2 * q];
      tb += red[2 * q + 1];
    }
    part[2 * blockIdx.x] = ta;
    part[2 * blockIdx.x + 1] = tb;
  }
}

__global__ void lj_sumsq2_final(const double* __restrict__ part, int G, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double ta = 0.0, tb = 0.0;
  for (int g = 0; g < G; ++g) {
    ta += part[2 * g];
    tb += part[2 * g + 1];
  }
  out[0] = ta;
  out[1] = tb;
}

// ---------------------------------------------------------------------------
// Launch wrappers (host side).
// ---------------------------------------------------------------------------
int persistent_block() { return kBlock; }
int tile_halo() { return kMaxSuper; }

void* action_stream_ptr(int kind, int K) {
#define LJ_STREAM_CASE(K_, NC_)                                                                     \
  case K_:                                                                                          \
    return K <= 1 ? reinterpret_cast<void*>(&lj_action_stream<K_, NC_, 1>)                          \
                  : reinterpret_cast<void*>(&lj_action_stream<K_, NC_, kMaxK>);
  switch (kind) {
    LJ_STREAM_CASE(OP_DIAG, 1)
    LJ_STREAM_CASE(OP_ADVDIFF, 1)
    LJ_STREAM_CASE(OP_ALLENCAHN, 1)
    LJ_STREAM_CASE(OP_BRUSSELATOR, 2)
    LJ_STREAM_CASE(OP_BURGERS, 1)
    LJ_STREAM_CASE(OP_GRAYSCOTT, 2)
    LJ_STREAM_CASE(OP_ADR, 1)
  }
#undef LJ_STREAM_CASE
  return nullptr;
}

void* action_tile_ptr(int kind, int ept, int K) {
#define LJ_TILE_CASES(K_)                                                                            \
  if (kind == K_) {                                                                                  \
    switch (ept) {                                                                                   \
      case 1: return km1 ? reinterpret_cast<void*>(&lj_action_tile<K_, kMaxSuper, 1, 1>)             \
                         : reinterpret_cast<void*>(&lj_action_tile<K_, kMaxSuper, 1, kMaxK>);        \
      case 2: return km1 ? reinterpret_cast<void*>(&lj_action_tile<K_, kMaxSuper, 2, 1>)             \
                         : reinterpret_cast<void*>(&lj_action_tile<K_, kMaxSuper, 2, kMaxK>);        \
      case 3: return km1 ? reinterpret_cast<void*>(&lj_action_tile<K_, kMaxSuper, 3, 1>)             \
                         : reinterpret_cast<void*>(&lj_action_tile<K_, kMaxSuper, 3, kMaxK>);        \
    }                                                                                                \
    return nullptr;                                                                                  \
  }
  const bool km1 = K <= 1;
  LJ_TILE_CASES(OP_ALLENCAHN)
  LJ_TILE_CASES(OP_ADVDIFF)
  LJ_TILE_CASES(OP_ADR)
#undef LJ_TILE_CASES
  return nullptr;
}

void* action_reg_ptr(int kind, int K, bool full) {
#define LJ_REG_CASE(K_)                                                                                  \
  if (kind == K_) {                                                                                      \
    if (K <= 1)                                                                                          \
      return full ? reinterpret_cast<void*>(&lj_action_reg<K_, 1, true>)                                 \
                  : reinterpret_cast<void*>(&lj_action_reg<K_, 1, false>);                               \
    if (K == 2)                                                                                          \
      return full ? reinterpret_cast<void*>(&lj_action_reg<K_, 2, true>)                                 \
                  : reinterpret_cast<void*>(&lj_action_reg<K_, 2, false>);                               \
    if (K == 3)                                                                                          \
      return full ? reinterpret_cast<void*>(&lj_action_reg<K_, 3, true>)                                 \
                  : reinterpret_cast<void*>(&lj_action_reg<K_, 3, false>);                               \
    return full ? reinterpret_cast<void*>(&lj_action_reg<K_, kMaxK, true>)                               \
                : reinterpret_cast<void*>(&lj_action_reg<K_, kMaxK, false>);                             \
  }
  LJ_REG_CASE(OP_ALLENCAHN)
  LJ_REG_CASE(OP_ADVDIFF)
#undef LJ_REG_CASE
  return nullptr;
}
void* action_regm_ptr(int kind, int K, bool full) {
#define LJ_REGM_CASE(K_)                                                                                 \
  if (kind == K_) {                                                                                      \
    if (K <= 1)                                                                                          \
      return full ? reinterpret_cast<void*>(&lj_action_regm<K_, 1, true>)                                \
                  : reinterpret_cast<void*>(&lj_action_regm<K_, 1, false>);                              \
    return full ? reinterpret_cast<void*>(&lj_action_regm<K_, kMaxK, true>)                              \
                : reinterpret_cast<void*>(&lj_action_regm<K_, kMaxK, false>);                            \
  }
  LJ_REGM_CASE(OP_ALLENCAHN)
  LJ_REGM_CASE(OP_ADVDIFF)
#undef LJ_REGM_CASE
  return nullptr;
}
int reg_block() { return kRegBlock; }
int reg_steps() { return kRegS; }
size_t reg_lds_bytes() { return (size_t)kRegS * kRegTile * kRegTile * sizeof(double); }
size_t reg_static_lds() { return sizeof(RegShared); }

void* batch_kernel_ptr(int kind, int bs) {
#define LJ_BATCH_CASE(K_, NC_)                                                          \
  case K_:                                                                              \
    if (bs == 256) return reinterpret_cast<void*>(&lj_batch_kernel<K_, NC_, 256>);     \
    if (bs == 512) return reinterpret_cast<void*>(&lj_batch_kernel<K_, NC_, 512>);     \
    if (bs == 1024) return reinterpret_cast<void*>(&lj_batch_kernel<K_, NC_, 1024>);   \
    return nullptr;
  switch (kind) {
    LJ_BATCH_CASE(OP_DIAG, 1)
    LJ_BATCH_CASE(OP_ADVDIFF, 1)
    LJ_BATCH_CASE(OP_ALLENCAHN, 1)
    LJ_BATCH_CASE(OP_BRUSSELATOR, 2)
    LJ_BATCH_CASE(OP_BURGERS, 1)
    LJ_BATCH_CASE(OP_GRAYSCOTT, 2)
    LJ_BATCH_CASE(OP_ADR, 1)
  }
#undef LJ_BATCH_CASE
  return nullptr;
}

hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t s) {
  int g = (n + 255) / 256;
  if (g > 64) g = 64;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(lj_fill_u32, dim3(g), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

hipError_t launch_divdiff(const DDParams& P, hipStream_t s) {
  hipLaunchKernelGGL(lj_divdiff_kernel, dim3(1), dim3(256), 0, s, P);
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
hipError_t launch_rhs(const OpDev& op, const double* u, double* f, hipStream_t s) {
  switch (op.kind) {
    case OP_DIAG: rhs_t<OP_DIAG, 1>(op, u, f, s); break;
    case OP_ADVDIFF: rhs_t<OP_ADVDIFF, 1>(op, u, f, s); break;
    case OP_ALLENCAHN: rhs_t<OP_ALLENCAHN, 1>(op, u, f, s); break;
    case OP_BRUSSELATOR: rhs_t<OP_BRUSSELATOR, 2>(op, u, f, s); break;
    case OP_BURGERS: rhs_t<OP_BURGERS, 1>(op, u, f, s); break;
    case OP_GRAYSCOTT: rhs_t<OP_GRAYSCOTT, 2>(op, u, f, s); break;
    case OP_ADR: rhs_t<OP_ADR, 1>(op, u, f, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int KIND, int NC>
static void rhs_scaled_t(const OpDev& op, double h, double* f, double* v, hipStream_t s) {
  hipLaunchKernelGGL((lj_rhs_scaled_kernel<KIND, NC>), dim3(stream_grid(op.npts)), dim3(256), 0, s, op, h, f, v);
}
template <int KIND, int NC>
static void stage_t(const StageArgs& A, hipStream_t s) {
  hipLaunchKernelGGL((lj_stage_kernel<KIND, NC>), dim3(stream_grid(A.op.npts)), dim3(256), 0, s, A);
}

hipError_t launch_rhs_scaled(const OpDev& op, double h, double* f, double* v, hipStream_t s) {
  switch (op.kind) {
    case OP_DIAG: rhs_scaled_t<OP_DIAG, 1>(op, h, f, v, s); break;
    case OP_ADVDIFF: rhs_scaled_t<OP_ADVDIFF, 1>(op, h, f, v, s); break;
    case OP_ALLENCAHN: rhs_scaled_t<OP_ALLENCAHN, 1>(op, h, f, v, s); break;
    case OP_BRUSSELATOR: rhs_scaled_t<OP_BRUSSELATOR, 2>(op, h, f, v, s); break;
    case OP_BURGERS: rhs_scaled_t<OP_BURGERS, 1>(op, h, f, v, s); break;
    case OP_GRAYSCOTT: rhs_scaled_t<OP_GRAYSCOTT, 2>(op, h, f, v, s); break;
    case OP_ADR: rhs_scaled_t<OP_ADR, 1>(op, h, f, v, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_stage(const StageArgs& A, hipStream_t s) {
  switch (A.op.kind) {
    case OP_DIAG: stage_t<OP_DIAG, 1>(A, s); break;
    case OP_ADVDIFF: stage_t<OP_ADVDIFF, 1>(A, s); break;
    case OP_ALLENCAHN: stage_t<OP_ALLENCAHN, 1>(A, s); break;
    case OP_BRUSSELATOR: stage_t<OP_BRUSSELATOR, 2>(A, s); break;
    case OP_BURGERS: stage_t<OP_BURGERS, 1>(A, s); break;
    case OP_GRAYSCOTT: stage_t<OP_GRAYSCOTT, 2>(A, s); break;
    case OP_ADR: stage_t<OP_ADR, 1>(A, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sumsq2(const double* a, const double* b, long n, double* part, double* out, hipStream_t s) {
  const int G = (int)std::min<long>(kSumsqBlocks, std::max<long>(1, (n + 255) / 256));
  hipLaunchKernelGGL(lj_sumsq2_partial, dim3(G), dim3(256), 0, s, a, b, n, part);
  hipLaunchKernelGGL(lj_sumsq2_final, dim3(1), dim3(64), 0, s, part, G, out);
  return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs& F, hipStream_t s) {
  hipLaunchKernelGGL(lj_finish_kernel, dim3(stream_grid(F.n)), dim3(256), 0, s, F);
  return hipGetLastError();
}

hipError_t launch_lincomb(const LinComb& L, hipStream_t s) {
  hipLaunchKernelGGL(lj_lincomb_kernel, dim3(stream_grid(L.n)), dim3(256), 0, s, L);
  return hipGetLastError();
}

}  // namespace lj
