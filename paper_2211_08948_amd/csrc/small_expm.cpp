// Exponential of a small dense matrix on the host (the projected matrix of
// the Krylov evaluation, (m + 1) x (m + 1) with m <= 64).
#include "small_expm.hpp"

#include <algorithm>
#include <cmath>

namespace lj {

// C = A B for small dense n x n matrices (row-major), row by row so that the
// inner loop runs over contiguous entries (an AVX2 clone is picked at load
// time where the host supports it)
__attribute__((target_clones("avx2", "default"))) void matmul_small(const double* A, const double* B, double* C,
                                                                     int n) {
  for (int i = 0; i < n * n; ++i) C[i] = 0.0;
  for (int r = 0; r < n; ++r)
    for (int q = 0; q < n; ++q) {
      const double a = A[(size_t)r * n + q];
      if (a == 0.0) continue;
      const double* b = B + (size_t)q * n;
      double* c = C + (size_t)r * n;
      for (int j = 0; j < n; ++j) c[j] += a * b[j];
    }
}

// exp(A) of a small dense n x n matrix (row-major) by scaling and squaring
// (Moler and Van Loan): X = A / 2^s with ||X||_1 <= 1/2, the Taylor
// polynomial of degree 16 (remainder below ||X||^17 / 17! < 2^-65) evaluated
// by the Paterson-Stockmeyer scheme in powers of X^4 (six products instead
// of fifteen), then s squarings.
void expm_small(const std::vector<double>& A, int n, std::vector<double>& E) {
  double nrm = 0.0;
  for (int c = 0; c < n; ++c) {
    double col = 0.0;
    for (int r = 0; r < n; ++r) col += std::fabs(A[(size_t)r * n + c]);
    nrm = std::max(nrm, col);
  }
  int sq = 0;
  if (nrm > 0.5) sq = (int)std::ceil(std::log2(nrm / 0.5));
  const double scale = std::ldexp(1.0, -sq);
  const size_t nn = (size_t)n * n;
  std::vector<double> X(nn), X2(nn), X3(nn), X4(nn), R(nn), T(nn);
  for (size_t i = 0; i < nn; ++i) X[i] = A[i] * scale;
  matmul_small(X.data(), X.data(), X2.data(), n);
  matmul_small(X2.data(), X.data(), X3.data(), n);
  matmul_small(X2.data(), X2.data(), X4.data(), n);
  double cf[17];  // 1 / k!
  cf[0] = 1.0;
  for (int k = 1; k <= 16; ++k) cf[k] = cf[k - 1] / (double)k;
  // B_j = c_{4j} I + c_{4j+1} X + c_{4j+2} X^2 + c_{4j+3} X^3
  auto block = [&](int j, std::vector<double>& out) {
    for (size_t i = 0; i < nn; ++i) out[i] = cf[4 * j + 1] * X[i] + cf[4 * j + 2] * X2[i] + cf[4 * j + 3] * X3[i];
    for (int i = 0; i < n; ++i) out[(size_t)i * n + i] += cf[4 * j];
  };
  // R = B_3 + c_16 X^4, then R = B_j + X^4 R for j = 2, 1, 0
  block(3, R);
  for (size_t i = 0; i < nn; ++i) R[i] += cf[16] * X4[i];
  for (int j = 2; j >= 0; --j) {
    matmul_small(X4.data(), R.data(), T.data(), n);
    block(j, R);
    for (size_t i = 0; i < nn; ++i) R[i] += T[i];
  }
  for (int k = 0; k < sq; ++k) {
    matmul_small(R.data(), R.data(), T.data(), n);
    R.swap(T);
  }
  E.swap(R);
}

}  // namespace lj
