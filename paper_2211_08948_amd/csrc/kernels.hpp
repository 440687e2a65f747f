// Launch wrappers of the kernels (implemented in kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lj {

// out = sum_{q < nin} alpha[q] * x[q], elementwise over n entries
struct LinComb {
  long n;
  int nin;
  double alpha[5];
  const double* x[5];
  double* out;
};

// Stage arguments of a scheme in one pass (see lj_stage_kernel): remainders
// R_r at x_r = state + sum_{t < nterm[r]} a[r][t] X[r][t], r < nrem <= 2, then
// out[o] = sum_{t < nsrc[o]} c[o][t] S_{src[o][t]}, o < nout <= 2, with
// S_0 = R_0, S_1 = R_1, S_2 = P.
struct StageArgs {
  OpDev op;
  const double* fu;
  int nrem;
  int nterm[2];
  double a[2][2];
  const double* X[2][2];
  const double* P;
  int nout;
  int nsrc[2];
  int src[2][2];
  double c[2][2];
  double* out[2];
};

// u_out = u + X1 (+ X2) (+ X3), err = u_out - (u + X1 (+ X2)) if X3 is given,
// else 0 (see lj_finish_kernel); n values
struct FinishArgs {
  long n;
  const double* u;
  const double* X1;
  const double* X2;
  const double* X3;
  double* u_out;
  double* err;
};

int persistent_block();  // threads per block of the action kernels
int tile_halo();         // halo width = Newton steps per barrier of the tiled kernel
void* action_stream_ptr(int kind, int K);  // K accumulators
void* action_reg_ptr(int kind, int K, bool full);  // register-tiled kernel (full: every tile 32 x 32); nullptr if the family has none
void* action_regm_ptr(int kind, int K, bool full);  // several tiles per block (grids of more tiles than CUs)
int reg_block();                        // its threads per block
int reg_steps();                        // Newton steps per super-step
size_t reg_lds_bytes();                 // its dynamic LDS (step history)
size_t reg_static_lds();                // its static LDS
void* action_tile_ptr(int kind, int ept, int K);  // K accumulators; nullptr if the family has no tiled kernel

hipError_t launch_divdiff(const DDParams& P, hipStream_t s);
void* batch_kernel_ptr(int kind, int block_size);  // block_size in {256, 512, 1024}
hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t s);
hipError_t launch_rhs(const OpDev& op, const double* u, double* f, hipStream_t s);
hipError_t launch_lincomb(const LinComb& L, hipStream_t s);
hipError_t launch_rhs_scaled(const OpDev& op, double h, double* f, double* v, hipStream_t s);  // f(state), h f
hipError_t launch_stage(const StageArgs& A, hipStream_t s);
hipError_t launch_finish(const FinishArgs& F, hipStream_t s);
// out[0] = sum a^2, out[1] = sum b^2 over n values; part holds 2 * kSumsqBlocks doubles
constexpr int kSumsqBlocks = 256;
hipError_t launch_sumsq2(const double* a, const double* b, long n, double* part, double* out, hipStream_t s);

}  // namespace lj
