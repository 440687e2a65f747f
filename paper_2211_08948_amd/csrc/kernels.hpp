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

int persistent_block();  // threads per block of the action kernels
int tile_halo();         // halo width = Newton steps per barrier of the tiled kernel
void* action_stream_ptr(int kind);
void* action_tile_ptr(int kind, int ept);  // nullptr if the family has no tiled kernel

hipError_t launch_divdiff(const DDParams& P, hipStream_t s);
void* batch_kernel_ptr(int kind, int block_size);  // block_size in {256, 512, 1024}
hipError_t launch_fill_u32(unsigned int* p, int n, unsigned int v, hipStream_t s);
hipError_t launch_rhs(const OpDev& op, const double* u, double* f, hipStream_t s);
hipError_t launch_remainder(const OpDev& op, const double* x, const double* d, const double* fu,
                            double* r, hipStream_t s);
hipError_t launch_lincomb(const LinComb& L, hipStream_t s);

}  // namespace lj
