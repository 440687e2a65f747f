// Types shared by the host control code and the kernels.
#pragma once

#include <stdint.h>

namespace lj {

enum OpKind {
  OP_DIAG = 0,
  OP_ADVDIFF = 1,
  OP_ALLENCAHN = 2,
  OP_BRUSSELATOR = 3,
  OP_BURGERS = 4,
  OP_GRAYSCOTT = 5,
  OP_ADR = 6
};

// families with homogeneous Neumann boundaries (cell-centred grid: the ghost
// beyond a boundary face holds the cell inside it); the others are periodic
constexpr bool family_neumann(int kind) { return kind == OP_ADR; }

// default bound on the polls of one grid-barrier wait (see wait_at_least)
constexpr unsigned int kGridSpinLimit = 1u << 22;

// components per grid point of a family
constexpr int family_ncomp(int kind) { return (kind == OP_BRUSSELATOR || kind == OP_GRAYSCOTT) ? 2 : 1; }

constexpr int kMaxK = 4;                // accumulators sharing one Newton basis
constexpr int kMaxL = 4;                // highest phi index
constexpr int kMaxPoints = 100;         // most Newton terms
constexpr int kTable = kMaxPoints + 1;  // Leja nodes kept on the device
constexpr int kBarrierWords = 32 * 19;  // words of one grid-barrier state (zero at launch)
constexpr int kPartStride = 48;         // partial sums per block and barrier slot
constexpr int kRegPartStride = 96;      // the same for the register-tiled kernel (16 steps x (1 + K) + 1)
constexpr int kMaxSuper = 8;            // Newton steps per barrier in the tiled kernel (max)
constexpr int kRegSnap = 5;             // accumulator snapshots before a predicted stop (several-tile kernel)

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
  int power_iters;      // Jacobian products of the power iteration (0 if skipped)
  int barriers;         // grid barriers used
  int aborted;          // 1: a grid barrier timed out (blocks not co-resident); results invalid
  int skipped;          // != 0: the launch did no work because the learned proposal's decision
                        // (ActionParams.skip_src) asked for that many substeps (> 1) or had no
                        // usable bound (-1)
  double vnorm;         // ||v||_2
  double lam, c, gamma; // bound used and the interval it gives
  // reduced totals of every decided Newton step m = 1..iters:
  // trace[m-1][0] = ||y_m||^2, trace[m-1][1+k] = ||p_k||^2 after term m
  double trace[kMaxPoints][1 + kMaxK];
  // wall-clock ticks spent by block 0 per phase (see kProf*), for tuning
  unsigned long long prof[8];
};

enum ProfPhase { kProfPower = 0, kProfDivdiff, kProfSteps, kProfPublish, kProfBarrier, kProfDecide, kProfCommit, kProfHalo };

// Divided differences on their own (the lj_divided_differences entry point).
struct DDParams {
  int K;
  int l[kMaxK];
  double s[kMaxK];        // a_k * tau
  int npts;               // coefficients per accumulator (<= kTable)
  double c, gamma;        // interval centre and quarter-length
  const double* xi;       // Leja table (device, kTable entries)
  double* coef;           // out: K x kTable divided differences
  double* fmax;           // out: K values max_j |f_j|
};

// One phi-action launch: optional power iteration, divided differences and the
// whole Newton recurrence.
struct ActionParams {
  OpDev op;
  // spectral bound
  int do_power;           // 1: run the power iteration; 0: use lam_in
  int power_iters;
  uint64_t seed;
  const double* start;    // explicit power-iteration start vector or nullptr
  double lam_in;
  const double* lam_src;  // if set (and do_power == 0): the bound is read from here (device)
  const int* skip_src;    // if set: the launch returns at once unless *skip_src == 1 (device)
  double* lam_out;        // if set: the bound used is written here (device)
  double safety;
  // expansion
  const double* v;        // y_0 (device)
  int K;
  int l[kMaxK];
  double s[kMaxK];        // a_k * tau
  double* p[kMaxK];       // accumulators = outputs (device)
  int max_points;
  int relative;
  double tol;
  double hump;
  const double* xi;       // Leja table (device)
  // workspace
  double* ybuf0;          // two device vectors of n entries
  double* ybuf1;
  double* partials;       // 2 x kPartStride x gridDim partial sums, slot-major
  unsigned int* barrier;  // kBarrierWords words, zero at launch; left zero at exit
  unsigned int spin_limit;  // polls before a barrier wait gives up (and the launch aborts)
  LejaStatus* status;     // out
  LejaStatus* status_host;  // optional: the status header also here (pinned host memory)
  // tiling of the LDS-resident kernel
  int tx, ty, ntx, nty;   // tile size and tiles per axis (gridDim = ntx * nty)
  int lds_h;              // offset (doubles) of the step history in dynamic LDS
  // several tiles per block (register-tiled kernel on large grids): a third
  // exchange vector, a second buffer per accumulator (committed and
  // speculative values alternate between it and the output), and K x kRegSnap
  // vectors of accumulator values at the steps before a super-step's last
  double* ybuf2;
  double* pw[kMaxK];
  double* snap;
};

// ---- batching form ---------------------------------------------------------
// One instance of a batch: its operator, input, outputs and two workspace
// vectors of its own length (device pointers).
struct BatchItem {
  OpDev op;
  const double* v;
  double* p[kMaxK];   // outputs phi_{l_k}(s_k J) v
  double* y0;         // Newton basis / power-iteration double buffer
  double* y1;
  double s[kMaxK];    // a_k * h of this instance
  double lam_in;      // > 0: spectral bound given; else power iteration
  double* sub;        // substep vectors: phi_1..phi_l at the substep, then e^{tau J} w
  size_t nsub_stride; // values between consecutive substep vectors (the instance's length)
};

// What the batch kernel reports per instance.
struct BatchStatus {
  int state[kMaxK];
  int m_star[kMaxK];           // Newton steps of the accepted attempt (substeps: all its recurrences)
  double err[kMaxK];
  int substeps[kMaxK];         // substeps of the accepted attempt (1: the shared basis)
  int iters;                   // Newton steps of every recurrence of the instance
  int accum_iters;             // accumulator updates of every recurrence
  int vec_passes;              // vectors read or written by the substep combinations
  int rejections;              // the shared basis's rejection (0 or 1) plus every failed substep attempt
  int power_iters;
  int block;                   // block that ran the instance
  double vnorm, lam, c, gamma;
  unsigned long long t0, t1;   // device wall clock at the start and end of the instance
};

struct BatchParams {
  const BatchItem* items;
  BatchStatus* status;
  const int* order;       // processing order (a permutation of 0..n-1)
  int n;
  int K;
  int l[kMaxK];
  int power_iters;
  uint64_t seed;
  double safety;
  int max_points;
  int max_substeps;
  int relative;
  double tol;
  double hump;
  const double* xi;       // Leja table (device)
  unsigned int* queue;    // [0] work counter, [1] abort word; zero at launch
  // teams: `team` blocks of one XCD share an instance (team = 1: one block)
  int team;
  unsigned int* team_words;  // per team kTeamWords words, zero at launch (barrier counter, mailbox)
  double* team_part;         // per team 2 x kQ x team partial sums
};

constexpr int kTeamWords = 64;

}  // namespace lj
