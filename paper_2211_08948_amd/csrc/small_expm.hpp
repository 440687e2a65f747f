// Exponential of a small dense matrix on the host (implemented in
// small_expm.cpp).
#pragma once

#include <vector>

namespace lj {

// C = A B for n x n row-major matrices
void matmul_small(const double* A, const double* B, double* C, int n);
// E = exp(A) for an n x n row-major matrix, to double precision
void expm_small(const std::vector<double>& A, int n, std::vector<double>& E);

}  // namespace lj
