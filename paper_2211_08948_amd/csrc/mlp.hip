// Kernels of the learned proposal: the 16 features of an action (one
// reduction pass over the state), and a 16-64-64-2 tanh perceptron in FP32 --
// inference, back-propagated gradients and Adam training, all hand-written.
//
// The network is small (5378 parameters, ~5k multiply-adds per sample), so
// a sample is one thread's work: it forms its activations in registers, writes
// what the weight gradients need to a per-sample scratch row, and the
// gradient of each parameter is then summed over the samples of a minibatch by
// one thread in sample order (deterministic, no atomics).  Training runs as a
// single persistent block that walks every epoch and minibatch in order.
#include <hip/hip_runtime.h>

#include "device.hpp"
#include "mlp.hpp"

namespace lj {

// ---------------------------------------------------------------------------
// Features (the definitions live with the oracle's feature module; the same
// numbers are formed here from one pass over the grid).
// ---------------------------------------------------------------------------
struct FeatPartial {
  double sum, sumsq, umax, gmax, rmax, rmin, lmax;  // lmax: max|diagonal| (diagonal operators)
  double gers;                                      // max over rows of sum_j |J_ij| (Gershgorin)
};

// Largest absolute row sum of J over the NC rows of point p (the Gershgorin
// bound of the spectral radius, rows of p).  The entries of those rows are
// read off stencil_jv -- the product the action kernels apply -- with a unit
// value in one of the five stencil places and one component at a time;
// places that are the same grid point (a Neumann boundary cell is its own
// neighbour; tiny periodic grids) are summed before the absolute value.
template <int KIND, int NC>
__device__ double gershgorin_rows(const OpDev& op, int p) {
  const Nbr q = neighbours<KIND>(op, p);
  const int idx[5] = {q.c, q.w, q.e, q.s, q.n};
  double uv[5][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
  if (StateUse<KIND>::value > 0 || KIND == OP_DIAG) {
#pragma unroll
    for (int t = 0; t < 5; ++t)
#pragma unroll
      for (int c = 0; c < NC; ++c) uv[t][c] = op.state[NC * idx[t] + c];
  }
  double co[5][2][2];  // co[place][input component][output component]
#pragma unroll
  for (int t = 0; t < 5; ++t) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double x[5][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
      x[t][c] = 1.0;
      double out[2] = {0.0, 0.0};
      stencil_jv<KIND>(op, x, uv, out);
      co[t][c][0] = out[0];
      co[t][c][1] = out[1];
    }
  }
  double best = 0.0;
#pragma unroll
  for (int cc = 0; cc < NC; ++cc) {
    double row = 0.0;
#pragma unroll
    for (int t = 0; t < 5; ++t) {
      bool seen = false;
#pragma unroll
      for (int t2 = 0; t2 < t; ++t2) seen = seen || (idx[t2] == idx[t]);
      if (seen) continue;
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        double a = 0.0;
#pragma unroll
        for (int t2 = t; t2 < 5; ++t2)
          if (idx[t2] == idx[t]) a += co[t2][c][cc];
        row += fabs(a);
      }
    }
    best = fmax(best, row);
  }
  return best;
}

// local reaction rate r(p) of J and the first state component u(p)
template <int KIND, int NC>
__device__ __forceinline__ void reaction_at(const OpDev& op, int p, double& u, double& r, double& g) {
  u = 0.0;
  r = 0.0;
  g = 0.0;
  if constexpr (KIND == OP_DIAG || KIND == OP_ADVDIFF) {
    return;
  } else {
    const Nbr q = neighbours<KIND>(op, p);
    const double* s = op.state;
    u = s[NC * q.c];
    const double uw = s[NC * q.w], ue = s[NC * q.e], us = s[NC * q.s], un = s[NC * q.n];
    const double gx = (ue - uw) * 0.5, gy = (un - us) * 0.5;
    g = sqrt(gx * gx + gy * gy);
    if constexpr (KIND == OP_ALLENCAHN) {
      r = 1.0 - 3.0 * u * u;
    } else if constexpr (KIND == OP_BURGERS) {
      r = -((ue - uw) * op.i2dx + (un - us) * op.i2dy);
    } else if constexpr (KIND == OP_ADR) {  // d/du of rate u (1 - u)(u - 1/2)
      r = op.c2 * (u * (3.0 - 3.0 * u) - 0.5);
    } else if constexpr (KIND == OP_GRAYSCOTT) {  // d/du of the first species' reaction
      const double v = s[NC * q.c + 1];
      r = -(v * v) - op.c2;
    } else {  // OP_BRUSSELATOR: d/du of the first species' reaction
      r = -(op.c3 + 1.0) + 2.0 * u * s[NC * q.c + 1];
    }
  }
}

template <int KIND, int NC>
__global__ __launch_bounds__(256) void lj_feature_partials(OpDev op, FeatPartial* part) {
  double sum = 0.0, sumsq = 0.0, umax = 0.0, gmax = 0.0, rmax = -INFINITY, rmin = INFINITY, lmax = 0.0;
  double gers = 0.0;
  for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < op.npts; p += gridDim.x * blockDim.x) {
    gers = fmax(gers, gershgorin_rows<KIND, NC>(op, p));
    double u, r, g;
    reaction_at<KIND, NC>(op, p, u, r, g);
    sum += u;
    sumsq += u * u;
    umax = fmax(umax, fabs(u));
    gmax = fmax(gmax, g);
    rmax = fmax(rmax, r);
    rmin = fmin(rmin, r);
    if constexpr (KIND == OP_DIAG) lmax = fmax(lmax, fabs(op.state[p]));
  }
  __shared__ double red[8][4];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  double v[8] = {wave_sum(sum), wave_sum(sumsq), umax, gmax, rmax, rmin, lmax, gers};
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    v[2] = fmax(v[2], __shfl_xor(v[2], off, 64));
    v[3] = fmax(v[3], __shfl_xor(v[3], off, 64));
    v[4] = fmax(v[4], __shfl_xor(v[4], off, 64));
    v[5] = fmin(v[5], __shfl_xor(v[5], off, 64));
    v[6] = fmax(v[6], __shfl_xor(v[6], off, 64));
    v[7] = fmax(v[7], __shfl_xor(v[7], off, 64));
  }
  if (lane == 0)
    for (int i = 0; i < 8; ++i) red[i][w] = v[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    FeatPartial P{0.0, 0.0, 0.0, 0.0, -INFINITY, INFINITY, 0.0, 0.0};
    for (int ww = 0; ww < (int)(blockDim.x >> 6); ++ww) {
      P.sum += red[0][ww];
      P.sumsq += red[1][ww];
      P.umax = fmax(P.umax, red[2][ww]);
      P.gmax = fmax(P.gmax, red[3][ww]);
      P.rmax = fmax(P.rmax, red[4][ww]);
      P.rmin = fmin(P.rmin, red[5][ww]);
      P.lmax = fmax(P.lmax, red[6][ww]);
      P.gers = fmax(P.gers, red[7][ww]);
    }
    part[blockIdx.x] = P;
  }
}

// Combines the block partials in block order and writes the features of the
// K actions (h_k, l_k) as rows of 16 floats (feats may be NULL); gers_out
// receives the Gershgorin bound G.
__global__ void lj_feature_finish(FeatureJob J, const FeatPartial* part, int nparts, float* feats,
                                  double* gers_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const OpDev& op = J.op;
  FeatPartial P{0.0, 0.0, 0.0, 0.0, -INFINITY, INFINITY, 0.0, 0.0};
  for (int b = 0; b < nparts; ++b) {
    P.sum += part[b].sum;
    P.sumsq += part[b].sumsq;
    P.umax = fmax(P.umax, part[b].umax);
    P.gmax = fmax(P.gmax, part[b].gmax);
    P.rmax = fmax(P.rmax, part[b].rmax);
    P.rmin = fmin(P.rmin, part[b].rmin);
    P.lmax = fmax(P.lmax, part[b].lmax);
    P.gers = fmax(P.gers, part[b].gers);
  }
  const double G = P.gers;
  *gers_out = G;
  if (feats == nullptr) return;
  const bool has_state = !(op.kind == OP_DIAG || op.kind == OP_ADVDIFF);
  double sigma, A = 0.0;
  if (op.kind == OP_DIAG) {
    sigma = P.lmax;
  } else {
    const double D = (op.kind == OP_BRUSSELATOR || op.kind == OP_GRAYSCOTT) ? fmax(op.c0, op.c1) : op.c0;
    sigma = D * (op.idx2 + op.idy2);
    if (op.kind == OP_ADVDIFF) A = fabs(op.c1) * 2.0 * op.i2dx + fabs(op.c2) * 2.0 * op.i2dy;
    if (op.kind == OP_BURGERS) A = P.umax * 2.0 * (op.i2dx + op.i2dy);
    if (op.kind == OP_ADR) A = fabs(op.c1) * 2.0 * (op.i2dx + op.i2dy);
  }
  const double rmax = has_state ? P.rmax : 0.0, rmin = has_state ? P.rmin : 0.0;
  const double n = (double)op.npts;
  const double mean = has_state ? P.sum / n : 0.0;
  double var = has_state ? P.sumsq / n - mean * mean : 0.0;
  if (var < 0.0) var = 0.0;
  const double umax = has_state ? P.umax : 0.0;
  const double gmax = has_state ? P.gmax : 0.0;
  const double rat_mean = umax > 0.0 ? mean / umax : 0.0;
  const double rat_std = umax > 0.0 ? sqrt(var) / umax : 0.0;
  // dx / dy from the stored reciprocals 1/(2 dx), 1/(2 dy)
  const double dx_over_dy = (op.kind == OP_DIAG) ? 1.0 : op.i2dy / op.i2dx;
  for (int k = 0; k < J.K; ++k) {
    const double h = J.h[k];
    float* f = feats + 16 * k;
    f[0] = (float)log10(h * G);
    f[1] = (float)(J.l[k] / 4.0);
    f[2] = (float)log10(1.0 + A / sigma);
    f[3] = (float)log10(1.0 + fmax(rmax, 0.0) / sigma);
    f[4] = (float)log10(1.0 + fmax(-rmin, 0.0) / sigma);
    f[5] = (float)log10(1.0 + h * A);
    f[6] = (float)log10(1.0 + h * fmax(rmax, 0.0));
    f[7] = (float)log10(1.0 + h * fmax(-rmin, 0.0));
    f[8] = (float)rat_mean;
    f[9] = (float)rat_std;
    f[10] = (float)log10(1.0 + umax);
    f[11] = (float)log10(1.0 + gmax);
    f[12] = (float)(log10(n) / 7.0);
    f[13] = (float)log10(dx_over_dy);
    f[14] = (float)log10(G / sigma);
    f[15] = (float)(op.ncomp - 1);
  }
}

// The proposal from the network's outputs pred (K rows of 2): bound =
// margin * G * exp(max_k pred[k][0]) and s = 2^round(max_k pred[k][1]) (s in
// 1 .. 2^20); out->sub = s, or -1 when the bound is not usable or s exceeds
// max_substeps (the caller then takes the plain path).
__global__ void lj_proposal_decide(const float* pred, int K, const double* gers, double margin, int max_substeps,
                                   ProposalOut* out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double lb = pred[0], ls = pred[1];
  for (int k = 1; k < K; ++k) {
    lb = fmax(lb, (double)pred[kMlpOut * k]);
    ls = fmax(ls, (double)pred[kMlpOut * k + 1]);
  }
  const double bound = margin * (*gers) * exp(fmin(lb, 50.0));
  const int e = (int)rint(fmin(fmax(ls, 0.0), 20.0));
  const int sub = 1 << e;
  const bool ok = bound > 0.0 && isfinite(bound) && sub <= max_substeps;
  out->bound = ok ? bound : 0.0;
  out->sub = ok ? sub : -1;
}

// Training targets of one record: ln(bound / G) and log2(substeps).
__global__ void lj_proposal_targets(const double* gers, double bound, int substeps, float* target) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  target[0] = (float)log(bound / *gers);
  target[1] = (float)log2((double)substeps);
}

// ---------------------------------------------------------------------------
// The network.  Model layout (floats): theta (kMlpParams, see mlp.hpp for the
// order) | mu[16] | sd[16] | tmu[2] | tsd[2].
// ---------------------------------------------------------------------------
__device__ __forceinline__ float tanh_f(float x) { return tanhf(x); }

// per-sample scratch row of the training kernels
constexpr int kRowXn = 0, kRowH1 = 16, kRowZ1 = 80, kRowH2 = 144, kRowZ2 = 208, kRowDy = 272;
constexpr int kRow = kMlpRowFloats;  // floats per sample (274 used, padded)

// Forward and backward of one sample with the weights in LDS (w).  Writes the
// sample's scratch row (normalised input, h1, dz1, h2, dz2, dy) and returns the
// squared error; dy = 2 e / scale.
__device__ float sample_fwd_bwd(const float* w, const float* x, const float* t, float scale, float* row) {
  const float* W1 = w + kOffW1;
  const float* b1 = w + kOffB1;
  const float* W2 = w + kOffW2;
  const float* b2 = w + kOffB2;
  const float* W3 = w + kOffW3;
  const float* b3 = w + kOffB3;
  const float* mu = w + kMlpParams;
  const float* sd = mu + kMlpIn;
  const float* tmu = sd + kMlpIn;
  const float* tsd = tmu + kMlpOut;
  float xn[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) {
    xn[k] = (x[k] - mu[k]) / sd[k];
    row[kRowXn + k] = xn[k];
  }
  float h1[kMlpHidden];
#pragma unroll
  for (int j = 0; j < kMlpHidden; ++j) {
    float z = b1[j];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) z += W1[j * kMlpIn + k] * xn[k];
    h1[j] = tanh_f(z);
    row[kRowH1 + j] = h1[j];
  }
  float y0 = b3[0], y1 = b3[1];
  for (int j = 0; j < kMlpHidden; ++j) {
    float z = b2[j];
#pragma unroll
    for (int i = 0; i < kMlpHidden; ++i) z += W2[j * kMlpHidden + i] * h1[i];
    const float h2 = tanh_f(z);
    row[kRowH2 + j] = h2;
    y0 += W3[j] * h2;
    y1 += W3[kMlpHidden + j] * h2;
  }
  const float e0 = y0 - (t[0] - tmu[0]) / tsd[0];
  const float e1 = y1 - (t[1] - tmu[1]) / tsd[1];
  const float dy0 = 2.0f * e0 / scale, dy1 = 2.0f * e1 / scale;
  row[kRowDy] = dy0;
  row[kRowDy + 1] = dy1;
  // dz2 and dz1 = W2^T dz2 * (1 - h1^2)
  float g1[kMlpHidden];
#pragma unroll
  for (int i = 0; i < kMlpHidden; ++i) g1[i] = 0.0f;
  for (int j = 0; j < kMlpHidden; ++j) {
    const float h2 = row[kRowH2 + j];
    const float dz2 = (W3[j] * dy0 + W3[kMlpHidden + j] * dy1) * (1.0f - h2 * h2);
    row[kRowZ2 + j] = dz2;
#pragma unroll
    for (int i = 0; i < kMlpHidden; ++i) g1[i] += W2[j * kMlpHidden + i] * dz2;
  }
#pragma unroll
  for (int i = 0; i < kMlpHidden; ++i) row[kRowZ1 + i] = g1[i] * (1.0f - h1[i] * h1[i]);
  return e0 * e0 + e1 * e1;
}

// gradient of parameter p summed over rows [0, nrows) of the scratch, in row order
__device__ float param_grad(int p, const float* rows, int nrows) {
  int a, b = -1;  // scratch offsets of the two factors (b < 0: bias, factor 1)
  if (p < kOffB1) {
    a = kRowZ1 + p / kMlpIn;
    b = kRowXn + p % kMlpIn;
  } else if (p < kOffW2) {
    a = kRowZ1 + (p - kOffB1);
  } else if (p < kOffB2) {
    const int q = p - kOffW2;
    a = kRowZ2 + q / kMlpHidden;
    b = kRowH1 + q % kMlpHidden;
  } else if (p < kOffW3) {
    a = kRowZ2 + (p - kOffB2);
  } else if (p < kOffB3) {
    const int q = p - kOffW3;
    a = kRowDy + q / kMlpHidden;
    b = kRowH2 + q % kMlpHidden;
  } else {
    a = kRowDy + (p - kOffB3);
  }
  float g = 0.0f;
  if (b < 0) {
    for (int n = 0; n < nrows; ++n) g += rows[(size_t)n * kRow + a];
  } else {
    for (int n = 0; n < nrows; ++n) g += rows[(size_t)n * kRow + a] * rows[(size_t)n * kRow + b];
  }
  return g;
}

__device__ void load_model(const float* model, float* w) {
  for (int i = threadIdx.x; i < kModelFloats; i += blockDim.x) w[i] = model[i];
  __syncthreads();
}

// block sum of one float per thread, in a fixed order; result for all threads
__device__ float block_sum_f(float v, float* red) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double s = wave_sum((double)v);
  if (lane == 0) red[w] = (float)s;
  __syncthreads();
  float t = 0.0f;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  __syncthreads();
  return t;
}

// Inference: out[n] = (y * tsd + tmu) for every sample, one thread per sample.
__global__ __launch_bounds__(256) void lj_mlp_forward_kernel(const float* model, const float* X, int n, float* out) {
  __shared__ float w[kModelFloats];
  load_model(model, w);
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  const float* W1 = w + kOffW1;
  const float* W2 = w + kOffW2;
  const float* W3 = w + kOffW3;
  const float* mu = w + kMlpParams;
  const float* sd = mu + kMlpIn;
  const float* tmu = sd + kMlpIn;
  const float* tsd = tmu + kMlpOut;
  float xn[kMlpIn];
#pragma unroll
  for (int k = 0; k < kMlpIn; ++k) xn[k] = (X[(size_t)s * kMlpIn + k] - mu[k]) / sd[k];
  float h1[kMlpHidden];
#pragma unroll
  for (int j = 0; j < kMlpHidden; ++j) {
    float z = w[kOffB1 + j];
#pragma unroll
    for (int k = 0; k < kMlpIn; ++k) z += W1[j * kMlpIn + k] * xn[k];
    h1[j] = tanh_f(z);
  }
  float y0 = w[kOffB3], y1 = w[kOffB3 + 1];
  for (int j = 0; j < kMlpHidden; ++j) {
    float z = w[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kMlpHidden; ++i) z += W2[j * kMlpHidden + i] * h1[i];
    const float h2 = tanh_f(z);
    y0 += W3[j] * h2;
    y1 += W3[kMlpHidden + j] * h2;
  }
  out[(size_t)s * 2] = y0 * tsd[0] + tmu[0];
  out[(size_t)s * 2 + 1] = y1 * tsd[1] + tmu[1];
}

// Loss and full gradient over n samples (the mean over all of them), one block:
// samples in chunks of blockDim.x, each parameter's sum taken in sample order.
__global__ __launch_bounds__(kMlpBlock) void lj_mlp_grad_kernel(const float* model, const float* X, const float* T,
                                                                int n, float* rows, float* grad, float* loss) {
  __shared__ float w[kModelFloats];
  __shared__ float red[kMlpBlock / 64];
  load_model(model, w);
  float gacc[(kMlpParams + kMlpBlock - 1) / kMlpBlock];
#pragma unroll
  for (int i = 0; i < (kMlpParams + kMlpBlock - 1) / kMlpBlock; ++i) gacc[i] = 0.0f;
  float lsum = 0.0f;
  for (int c0 = 0; c0 < n; c0 += blockDim.x) {
    const int nb = min((int)blockDim.x, n - c0);
    const int s = c0 + threadIdx.x;
    float e2 = 0.0f;
    if ((int)threadIdx.x < nb)
      e2 = sample_fwd_bwd(w, X + (size_t)s * kMlpIn, T + (size_t)s * kMlpOut, (float)n, rows + (size_t)threadIdx.x * kRow);
    lsum += block_sum_f(e2, red);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < (kMlpParams + kMlpBlock - 1) / kMlpBlock; ++i) {
      const int p = threadIdx.x + i * kMlpBlock;
      if (p < kMlpParams) gacc[i] += param_grad(p, rows, nb);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < (kMlpParams + kMlpBlock - 1) / kMlpBlock; ++i) {
    const int p = threadIdx.x + i * kMlpBlock;
    if (p < kMlpParams) grad[p] = gacc[i];
  }
  if (threadIdx.x == 0) *loss = lsum / (float)n;
}

// Training: `epochs` passes over the n samples in minibatches of `batch`
// (<= blockDim.x) in order; after every minibatch one Adam step (Kingma & Ba)
// on the minibatch mean gradient.  loss_epoch[e] = mean squared error of the
// samples of epoch e (as seen during the epoch).  One block.
__global__ __launch_bounds__(kMlpBlock) void lj_mlp_train_kernel(float* model, float* adam_m, float* adam_v,
                                                                 int* adam_t, const float* X, const float* T, int n,
                                                                 int epochs, int batch, float lr, float* rows,
                                                                 float* loss_epoch) {
  __shared__ float w[kModelFloats];
  __shared__ float red[kMlpBlock / 64];
  const float beta1 = 0.9f, beta2 = 0.999f, eps = 1e-8f;
  int t = *adam_t;
  for (int e = 0; e < epochs; ++e) {
    float lsum = 0.0f;
    for (int c0 = 0; c0 < n; c0 += batch) {
      const int nb = min(batch, n - c0);
      load_model(model, w);
      float e2 = 0.0f;
      if ((int)threadIdx.x < nb) {
        const int s = c0 + threadIdx.x;
        e2 = sample_fwd_bwd(w, X + (size_t)s * kMlpIn, T + (size_t)s * kMlpOut, (float)nb,
                            rows + (size_t)threadIdx.x * kRow);
      }
      lsum += block_sum_f(e2, red);
      __syncthreads();
      t += 1;
      const float c1 = 1.0f - powf(beta1, (float)t);
      const float c2 = 1.0f - powf(beta2, (float)t);
      for (int p = threadIdx.x; p < kMlpParams; p += blockDim.x) {
        const float g = param_grad(p, rows, nb);
        const float m = beta1 * adam_m[p] + (1.0f - beta1) * g;
        const float v = beta2 * adam_v[p] + (1.0f - beta2) * g * g;
        adam_m[p] = m;
        adam_v[p] = v;
        model[p] = w[p] - lr * (m / c1) / (sqrtf(v / c2) + eps);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) loss_epoch[e] = lsum / (float)n;
  }
  if (threadIdx.x == 0) *adam_t = t;
}

// Standardisation constants of a training set: mean and population standard
// deviation of every feature and target column (two passes, FP64, sample
// order); a deviation below 1e-6 is replaced by 1.
__global__ void lj_mlp_normalize_kernel(float* model, const float* X, const float* T, int n) {
  const int c = threadIdx.x;
  if (c >= kMlpIn + kMlpOut) return;
  const float* src = (c < kMlpIn) ? X + c : T + (c - kMlpIn);
  const int stride = (c < kMlpIn) ? kMlpIn : kMlpOut;
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += src[(size_t)i * stride];
  const double mean = s / n;
  double q = 0.0;
  for (int i = 0; i < n; ++i) {
    const double d = src[(size_t)i * stride] - mean;
    q += d * d;
  }
  double sd = sqrt(q / n);
  if (sd < 1e-6) sd = 1.0;
  float* mu = model + kMlpParams;
  float* sdv = mu + kMlpIn;
  float* tmu = sdv + kMlpIn;
  float* tsd = tmu + kMlpOut;
  if (c < kMlpIn) {
    mu[c] = (float)mean;
    sdv[c] = (float)sd;
  } else {
    tmu[c - kMlpIn] = (float)mean;
    tsd[c - kMlpIn] = (float)sd;
  }
}

// ---------------------------------------------------------------------------
// Launch wrappers
// ---------------------------------------------------------------------------
hipError_t launch_features(const FeatureJob& J, FeatPartialBuf part, float* feats, double* gers_out,
                           hipStream_t s) {
  const int nparts = kFeatureBlocks;
  switch (J.op.kind) {
    case OP_DIAG:
      hipLaunchKernelGGL((lj_feature_partials<OP_DIAG, 1>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    case OP_ADVDIFF:
      hipLaunchKernelGGL((lj_feature_partials<OP_ADVDIFF, 1>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    case OP_ALLENCAHN:
      hipLaunchKernelGGL((lj_feature_partials<OP_ALLENCAHN, 1>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    case OP_BRUSSELATOR:
      hipLaunchKernelGGL((lj_feature_partials<OP_BRUSSELATOR, 2>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    case OP_BURGERS:
      hipLaunchKernelGGL((lj_feature_partials<OP_BURGERS, 1>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    case OP_GRAYSCOTT:
      hipLaunchKernelGGL((lj_feature_partials<OP_GRAYSCOTT, 2>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    case OP_ADR:
      hipLaunchKernelGGL((lj_feature_partials<OP_ADR, 1>), dim3(nparts), dim3(256), 0, s, J.op,
                         reinterpret_cast<FeatPartial*>(part));
      break;
    default:
      return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(lj_feature_finish, dim3(1), dim3(64), 0, s, J, reinterpret_cast<const FeatPartial*>(part),
                     nparts, feats, gers_out);
  return hipGetLastError();
}

hipError_t launch_proposal_decide(const float* pred, int K, const double* gers, double margin, int max_substeps,
                                  ProposalOut* out, hipStream_t s) {
  hipLaunchKernelGGL(lj_proposal_decide, dim3(1), dim3(64), 0, s, pred, K, gers, margin, max_substeps, out);
  return hipGetLastError();
}

hipError_t launch_proposal_targets(const double* gers, double bound, int substeps, float* target, hipStream_t s) {
  hipLaunchKernelGGL(lj_proposal_targets, dim3(1), dim3(64), 0, s, gers, bound, substeps, target);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* model, const float* X, int n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(lj_mlp_forward_kernel, dim3((n + 255) / 256), dim3(256), 0, s, model, X, n, out);
  return hipGetLastError();
}

hipError_t launch_mlp_grad(const float* model, const float* X, const float* T, int n, float* rows, float* grad,
                           float* loss, hipStream_t s) {
  hipLaunchKernelGGL(lj_mlp_grad_kernel, dim3(1), dim3(kMlpBlock), 0, s, model, X, T, n, rows, grad, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_train(float* model, float* m, float* v, int* t, const float* X, const float* T, int n,
                            int epochs, int batch, float lr, float* rows, float* loss_epoch, hipStream_t s) {
  hipLaunchKernelGGL(lj_mlp_train_kernel, dim3(1), dim3(kMlpBlock), 0, s, model, m, v, t, X, T, n, epochs, batch, lr,
                     rows, loss_epoch);
  return hipGetLastError();
}

hipError_t launch_mlp_normalize(float* model, const float* X, const float* T, int n, hipStream_t s) {
  hipLaunchKernelGGL(lj_mlp_normalize_kernel, dim3(1), dim3(64), 0, s, model, X, T, n);
  return hipGetLastError();
}

size_t feature_partial_bytes() { return sizeof(FeatPartial) * kFeatureBlocks; }

}  // namespace lj
