// Kernels of the user-operator path (implemented in user_kernels.hip): the
// Newton recurrence of Sec. 2.2 for an operator given as host callbacks, run
// as short kernels between the callbacks with the stop decisions taken on the
// device, plus the Jacobian product of the built-in families (lj_jv).
#pragma once

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lj {

constexpr int kUserBlock = 256;   // threads per block of the user-path kernels
constexpr int kUserBlocksMax = 1024;

// Decision state of one user-operator recurrence or power iteration, kept in
// device memory between the kernels of a call.
struct UserState {
  int K, M, relative, fd;
  int m;      // last decided Newton step
  int done;   // no accumulator running (or the power iteration hit J x = 0)
  int state[kMaxK];
  int m_star[kMaxK];
  double err[kMaxK];
  double tol, hump;
  double nv;   // ||v||
  double nu;   // ||u|| (finite-difference step)
  double eps;  // finite-difference step of the next product
  double lam;  // power iteration: ||J x|| / ||x|| of the last product
  double ny;   // power iteration: ||J x|| of the last product
};

// What the host reads after a synchronisation (pinned, written by the kernels).
struct UserStatus {
  int done, iters;
  int state[kMaxK];
  int m_star[kMaxK];
  double err[kMaxK];
  double nv, lam;
};

int user_grid(long n);

// J(state) x of a built-in family (lj_jv)
hipError_t launch_family_jv(const OpDev& op, const double* x, double* y, hipStream_t s);

// x[i] = 0.5 + U_i (the power-iteration start vector of every path)
hipError_t launch_user_start_vector(double* x, long n, uint64_t seed, hipStream_t s);

// st->eps = sqrt(2^-52) (1 + st->nu) / ||x|| (0 for x = 0); part: user_grid(n) doubles
hipError_t launch_user_fd_step(UserState* st, const double* x, long n, double* part, hipStream_t s);
// st->nu = ||u||
hipError_t launch_user_norm_u(UserState* st, const double* u, long n, double* part, hipStream_t s);
// out = u + st->eps x
hipError_t launch_user_fd_point(const UserState* st, const double* u, const double* x, long n, double* out,
                                hipStream_t s);
// out = (fx - fu) / st->eps (0 where st->eps == 0)
hipError_t launch_user_fd_quotient(const UserState* st, const double* fx, const double* fu, long n, double* out,
                                   hipStream_t s);

// Newton recurrence: start (p_k = d_{k,0} v, ||v||), one step, one decision
struct UserRec {
  long n;
  int K;
  const double* coef;  // K x kTable divided differences (device)
  const double* fmax;  // K values max_j |f_j| (device)
  double* p[kMaxK];    // accumulators (device, n values each)
  double* part;        // user_grid(n) * (1 + K) partial sums
  UserState* st;
  UserStatus* host;    // pinned status the decisions are copied to
};
hipError_t launch_user_rec_start(const UserRec& R, const double* v, int M, double tol, int relative, double hump,
                                 int fd, hipStream_t s);
// y = ((J y_prev) - c y_prev) / gamma - xi y_prev with J y_prev = jy, or
// (fx - fu) / eps for finite differences (fu != nullptr); p_k += d_{k,m} y for
// running accumulators; partial sums of y^2 and p_k^2
hipError_t launch_user_rec_step(const UserRec& R, int m, const double* jy, const double* fu, const double* y_prev,
                                double* y, double c, double gamma, double rgamma, double xim, hipStream_t s);
hipError_t launch_user_rec_decide(const UserRec& R, int m, hipStream_t s);

// power iteration: st->done = 0, st->lam = 0 before the first product
hipError_t launch_user_power_init(UserState* st, hipStream_t s);
// power iteration: y = J x from jy or (fx - fu)/eps, partials of x^2, y^2;
// then the ratio and x_next = y / ||y|| (skipped once J x = 0)
hipError_t launch_user_power(UserState* st, const double* x, const double* jy, const double* fu, double* y,
                             double* x_next, long n, double* part, UserStatus* host, hipStream_t s);

}  // namespace lj
