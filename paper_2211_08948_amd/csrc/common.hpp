// Types shared by the host control code and the kernels.
#pragma once

#include <stdint.h>

namespace lj {

enum OpKind { OP_DIAG = 0, OP_ADVDIFF = 1, OP_ALLENCAHN = 2, OP_BRUSSELATOR = 3, OP_BURGERS = 4 };

constexpr int kMaxK = 4;          // accumulators sharing one Newton basis
constexpr int kMaxL = 4;          // highest phi index
constexpr int kMaxPoints = 100;   // most Newton terms
constexpr int kTable = kMaxPoints + 1;  // Leja nodes kept on the device
constexpr int kBarrierWords = 32 * 17;  // words of one grid-barrier state (zero at launch)

// Operator as the kernels see it: coefficients plus precomputed reciprocals.
struct OpDev {
  int kind, nx, ny, ncomp;
  double c0, c1, c2, c3;  // family coefficients (leja.h, lj_operator.coef)
  double idx2, idy2;      // 1/dx^2, 1/dy^2
  double i2dx, i2dy;      // 1/(2 dx), 1/(2 dy)
  const double* state;    // linearisation state / diagonal (device)
  int npts;               // nx * ny grid points
};

// Per-accumulator outcome of one Newton recurrence, written by the kernel.
enum AccState { ACC_RUNNING = 0, ACC_CONVERGED = 1, ACC_MAXPTS = 2, ACC_HUMP = 3, ACC_NONFINITE = 4 };

struct LejaStatus {
  int state[kMaxK];
  int m_star[kMaxK];
  double err[kMaxK];
  int iters;            // Newton iterations run (Jacobian products)
  int accum_iters;      // sum over iterations of active accumulators
  double vnorm;         // ||v||_2
};

// Device scalars shared between kernels of one call.
struct Scalars {
  double lam;    // lambda_hat
  double c;      // interval centre
  double gamma;  // interval quarter-length
  double pad;
};

struct DDParams {
  int K;
  int l[kMaxK];
  double s[kMaxK];        // a_k * tau
  int npts;               // coefficients per accumulator (<= kTable)
  double lam_host;        // > 0: use this lambda_hat instead of Scalars::lam
  double safety;
  int use_cg;             // 1: take c_in, gamma_in as given (scal unused)
  double c_in, gamma_in;
  const double* xi;       // Leja table (device, kTable entries)
  Scalars* scal;          // in: lam (unless lam_host > 0); out: lam, c, gamma
  double* coef;           // out: K x kTable divided differences
  double* fmax;           // out: K values max_j |f_j|
};

struct LejaParams {
  OpDev op;
  const double* v;        // y_0 (device)
  double* ybuf0;          // Newton basis double buffer (device, n each)
  double* ybuf1;
  double* p[kMaxK];       // accumulators = outputs (device, n each)
  int K;
  int max_points;
  int relative;
  double tol;
  double hump;
  const double* coef;     // K x kTable (device)
  const double* fmax;     // K (device)
  const double* xi;       // Leja table (device)
  const Scalars* scal;    // c, gamma (device)
  double* partials;       // 2 x gridDim x (K+1) (device)
  unsigned int* barrier;  // zero at launch
  LejaStatus* status;     // out
};

struct PowerParams {
  OpDev op;
  int iters;
  uint64_t seed;
  const double* start;    // explicit x_0 or nullptr (SplitMix64 start vector)
  double* buf0;           // two work vectors (device, n each)
  double* buf1;
  double* partials;       // 2 x gridDim x 2
  unsigned int* barrier;  // zero at launch
  Scalars* scal;          // out: lam
};

}  // namespace lj
