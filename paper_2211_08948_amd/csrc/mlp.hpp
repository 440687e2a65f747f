// The learned proposal's network and feature kernels (implemented in mlp.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lj {

// 16 -> 64 -> 64 -> 2, tanh hidden units.  Flat parameter order:
// W1 (64 x 16, row-major), b1 (64), W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).
constexpr int kMlpIn = 16, kMlpHidden = 64, kMlpOut = 2;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpHidden * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpHidden;
constexpr int kOffB2 = kOffW2 + kMlpHidden * kMlpHidden;
constexpr int kOffW3 = kOffB2 + kMlpHidden;
constexpr int kOffB3 = kOffW3 + kMlpOut * kMlpHidden;
constexpr int kMlpParams = kOffB3 + kMlpOut;                        // 5378
constexpr int kModelFloats = kMlpParams + 2 * kMlpIn + 2 * kMlpOut;  // + mu, sd, tmu, tsd
constexpr int kMlpBlock = 512;      // threads of the training / gradient kernels (one block)
constexpr int kMlpRowFloats = 276;  // scratch floats per sample of a minibatch
constexpr int kFeatureBlocks = 256; // blocks of the feature reduction

// Feature request: one operator (its state read once) and K actions (h_k, l_k).
struct FeatureJob {
  OpDev op;
  int K;
  double h[kMaxK];
  int l[kMaxK];
};

// The learned proposal's decision, written on the device: the bound and the
// substep count of the attempt (sub = -1: no usable proposal).
struct ProposalOut {
  double bound;
  int sub;
  int pad;
};

using FeatPartialBuf = void*;
size_t feature_partial_bytes();

// Features of the K actions of J (rows of 16 floats; feats may be NULL) and
// the Gershgorin bound G of J (gers_out, device).
hipError_t launch_features(const FeatureJob& J, FeatPartialBuf part, float* feats, double* gers_out,
                           hipStream_t s);
hipError_t launch_proposal_decide(const float* pred, int K, const double* gers, double margin, int max_substeps,
                                  ProposalOut* out, hipStream_t s);
hipError_t launch_proposal_targets(const double* gers, double bound, int substeps, float* target, hipStream_t s);
hipError_t launch_mlp_forward(const float* model, const float* X, int n, float* out, hipStream_t s);
hipError_t launch_mlp_grad(const float* model, const float* X, const float* T, int n, float* rows, float* grad,
                           float* loss, hipStream_t s);
hipError_t launch_mlp_train(float* model, float* m, float* v, int* t, const float* X, const float* T, int n,
                            int epochs, int batch, float lr, float* rows, float* loss_epoch, hipStream_t s);
hipError_t launch_mlp_normalize(float* model, const float* X, const float* T, int n, hipStream_t s);

}  // namespace lj
