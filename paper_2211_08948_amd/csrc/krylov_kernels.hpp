// Kernels of the Krylov evaluation of phi-function combinations (implemented
// in krylov_kernels.hip): Arnoldi's process on the augmented matrix
// A~ = [[J, B], [0, K]] of Sec. 2.1, with incomplete orthogonalisation.
// Vectors are augmented: N grid values followed by p auxiliary entries.
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lj {

constexpr int kKryBlock = 256;
constexpr int kKryBlocksMax = 512;
constexpr int kKryMaxDim = 64;   // largest Krylov dimension m
constexpr int kKryMaxP = 4;      // highest phi index in a combination
constexpr int kKryChunk = 8;     // window vectors per pass of the dot kernel

int kry_grid(long n);

// Arnoldi state shared by the kernels of one basis (device).
struct KryDev {
  long N;             // grid values
  int p;              // auxiliary entries
  long na;            // N + p, the augmented length
  double* V;          // (m + 1) basis vectors, vector j at V + j * na
  double* W;          // the product being orthogonalised (na)
  const double* B[kKryMaxP];  // B = [b_p, ..., b_1] (nullptr: zero column)
  double* H;          // (m + 1) x m Hessenberg matrix, row-major, row stride m
  int m;              // Krylov dimension
  double* part;       // kKryBlocksMax * (kKryMaxDim + 1) partial sums: dots, then norms
  double* scalars;    // [0] beta, [1] breakdown column + 1 (0: none)
};

// V_0 = w / ||w||, scalars[0] = ||w|| (two kernels)
hipError_t launch_kry_start(const KryDev& K, const double* w, hipStream_t s);
// W[0:N] holds J V_j[0:N].  With tail: add B y (y = V_j[N:N+p]) and write
// the shift K y into the tail first.  Then the dots <V_i, W> for window
// entries d = d0 .. d0 + nd - 1 (i = lo + d, nd <= kKryChunk), partial sums
// per block.  All dots are taken before W changes (classical Gram-Schmidt).
hipError_t launch_kry_tail_dots(const KryDev& K, int j, int lo, int d0, int nd, bool tail, hipStream_t s);
// the dots' sums (every block, block order) -> H[lo + d][j] for d < nd_total;
// W -= h_d V_{lo+d} in order of d; partial sums of W^2
hipError_t launch_kry_update(const KryDev& K, int j, int lo, int nd_total, hipStream_t s);
// H[j+1][j] = ||W||; V_{j+1} = W / H[j+1][j] unless the basis broke down
hipError_t launch_kry_scale(const KryDev& K, int j, hipStream_t s);
// out = beta sum_{j < m} F_j V_j (augmented length)
struct KryCoef {
  double f[kKryMaxDim];
};
hipError_t launch_kry_combine(const KryDev& K, int m, double beta, const KryCoef& F, double* out, hipStream_t s);
// w = [b_0 or 0; 0, ..., 0, 1]
hipError_t launch_kry_init(double* w, const double* b0, long N, int p, hipStream_t s);

// The whole basis in one persistent launch, for a built-in family and a
// window of 1 or 2 vectors, with one grid all-reduce per column: the
// product is applied to the orthogonalised vector before its normalisation
// (A~ is linear) and the window's dots, the next norm and the product share
// one pass (see the kernel).  Writes what the per-pass kernels write
// (V_0 .. V_{m_eff - 1}, H, scalars [0] and [1]) and scalars[2] = 1 when a
// grid barrier timed out (the launch is then to be repeated cooperatively).
// Blocks of kKryPBlock threads, at most one per CU; every block must be
// resident at once.
constexpr int kKryPBlock = 1024;
struct KryArnoldi {
  KryDev K;
  OpDev op;
  const double* w;         // start vector (augmented length), not modified
  double* U[2];            // u_k in U[k & 1] (augmented length)
  double* Z[2];            // z_k = A~ u_k in Z[k & 1] (augmented length)
  int window;              // 1 or 2
  double* partials;        // 2 x kPartStride x gridDim partial sums
  unsigned int* barrier;   // grid barrier words, zero at launch (left zero)
  unsigned int spin_limit; // bound on each barrier wait
};
// the kernel for a family (nullptr: no such family)
const void* kry_arnoldi_ptr(int kind);

}  // namespace lj
