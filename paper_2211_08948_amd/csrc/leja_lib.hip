// Host control of the Leja phi-action library: context, workspace, argument
// checks, the rejection / substep logic, the vertical form and the stage
// driver.  Every numerical step runs in the kernels of kernels.hip (and, for
// operators given as callbacks, user_kernels.hip); this file only
// orchestrates launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/leja.h"
#include "common.hpp"
#include "kernels.hpp"
#include "mlp.hpp"
#include "krylov_kernels.hpp"
#include "small_expm.hpp"
#include "user_kernels.hpp"

namespace lj {
int leja_points_host(double* out, int count);
}

using namespace lj;

// Workspace vectors, each sized to the current problem length on demand.
enum Slot {
  W_Y0, W_Y1,                      // Newton basis double buffer / power-iteration vectors
  W_P0, W_P1, W_P2, W_P3,          // phi_j(tau J) v of a substepped action
  W_SW0, W_SW1, W_SE,              // substep propagation buffers
  W_FU, W_V, W_A, W_B, W_C,        // stage driver: f(u), h f(u), vertical results
  W_RA, W_T1,                      // R(a) kept for a later stage, the phi_1 input of EXPRB43
  W_T3, W_D3, W_T4, W_D4,          // phi_3 / phi_4 inputs and results
  W_IU0, W_IU1, W_IERR,            // variable-step integration: state ping-pong, error estimate
  W_UJ, W_UPT, W_UY, W_UPA, W_UPB, // user operators: product, finite-difference point, power vectors
  W_UFU, W_UXR, W_UD, W_UFX, W_UJD, W_UR0, W_UR1,  // f(u), stage remainders
  W_KV, W_KW, W_KX, W_KC,          // Krylov: basis, product, augmented vector, LeKry third stage
  W_KU0, W_KU1, W_KZ0, W_KZ1,      // Krylov, one-launch basis: orthogonalised vectors and their products
  W_Y2, W_PW0, W_PW1, W_PW2, W_PW3, W_SNAP,  // register-tiled kernel with several tiles per block
  W_NSLOTS
};

// LDS held back from the tiled kernel's dynamic allocation for its static arrays
constexpr size_t kStaticLdsReserve = 40 * 1024;
constexpr int kQ_batch = 1 + kMaxK;  // team partial sums per reduction
constexpr int kAsyncSlots = 8;       // most action launches of one step
constexpr int kPoolSlots = 64;       // status heads of launches not yet read (one step, or a deferral)
constexpr int kTimingPairs = 1024;   // event pairs of the timing pool

// Device memory of the allocation-free entry point (lj_phi_action_noalloc):
// one file-scope array that every GPU the library runs on holds from the
// first context creation on it until the process ends.  In host code the name
// `scratch` is only a stand-in; its device address on each device comes from
// hipGetSymbolAddress at context creation (g_scratch_addr).
constexpr size_t kScratchBytes = (size_t)LJ_NOALLOC_SCRATCH_BYTES;
constexpr int kScratchDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
static double* g_scratch_addr[kScratchDevices] = {};
static std::mutex g_scratch_mu;

// An operator given as host callbacks (lj_user_operator) during one call.
struct UserOp {
  lj_user_operator J;
  bool fd = false;             // finite-difference products from rhs
  const double* fu = nullptr;  // f(u) (device), set when rhs is given
};

struct lj_context {
  int device = 0;
  int num_cus = 0;
  int lds_max = 64 * 1024;  // LDS bytes one workgroup may use
  std::string err;
  double* d_xi = nullptr;
  double* vec[W_NSLOTS] = {};
  size_t vec_cap[W_NSLOTS] = {};
  double* d_coef = nullptr;
  double* d_fmax = nullptr;
  double* d_partials = nullptr;
  int partial_cap = 0;  // blocks
  unsigned int* d_barrier = nullptr;
  LejaStatus* d_status = nullptr;
  LejaStatus* h_status = nullptr;  // pinned
  double* h_coef = nullptr;        // pinned
  int grid_override = 0;   // LJ_GRID: blocks of the streaming kernel
  int force_stream = 0;    // LJ_NO_TILE=1: never use the LDS-tiled or register-tiled kernels
  int no_reg = 0;          // LJ_NO_REG=1: never use the register-tiled kernel
  int force_coop = 0;      // LJ_COOP=1: always launch the action kernels cooperatively
  std::map<std::pair<const void*, size_t>, int> occupancy;  // blocks per CU of (kernel, dynamic LDS)
  int tile_override_x = 0; // LJ_TILE=tx,ty: tile shape of the LDS-tiled kernel
  int tile_override_y = 0;
  // timing: an event pair around each action launch; the elapsed times are
  // read when the counters are (lj_timing_read), not after every launch
  bool timing = false;
  unsigned int forced_spin_limit = 0;  // LJ_FORCE_SPIN_LIMIT (test hook), 0: the default bound
  int krylov_passes = 0;   // LJ_KRYLOV_PASSES=1: build Krylov bases with the per-pass kernels only
  std::vector<hipEvent_t> tev;  // 2 * kTimingPairs, created when timing is first enabled
  int tev_next = 0;             // next free pair
  std::vector<int> tev_pending; // pairs whose launches finished but whose times are unread
  lj_timing tm = {};
  std::unordered_map<const void*, size_t> dyn_lds;  // dynamic LDS limit set per kernel
  // launches of a step enqueued back to back: their status heads, event pairs
  // and the bound the first one leaves for the others
  LejaStatus* h_pool = nullptr;  // pinned, kPoolSlots entries
  double* d_bound = nullptr;
  double* d_sumsq = nullptr;   // 2 * kSumsqBlocks partials + 2 totals
  double* h_sumsq = nullptr;   // pinned, 2 totals
  // batching form: schedule picked by the tuner, per batch shape
  std::map<std::string, int> batch_schedule;
  // learned proposal
  float* d_model = nullptr;  // kModelFloats
  float* d_adam = nullptr;   // m | v (kMlpParams each)
  int* d_adam_t = nullptr;
  float* d_rows = nullptr;   // kMlpBlock x kMlpRowFloats training scratch
  float* d_scalars = nullptr;  // loss of lj_mlp_grad, epoch losses (kMaxEpochs)
  void* d_featpart = nullptr;
  float* d_feats = nullptr;  // kMaxK x 16
  float* d_pred = nullptr;   // kMaxK x 2
  double* d_gers = nullptr;            // Gershgorin bound of the last feature pass
  ProposalOut* d_prop = nullptr;       // the learned proposal's decision (device)
  bool mlp_ready = false;
  // user operators (callbacks): the operator of the running call, its
  // decision state and pinned status, partial sums, the Leja table on the host
  const UserOp* uop = nullptr;
  UserState* d_ustate = nullptr;
  UserStatus* h_ustatus = nullptr;  // pinned, coherent: written by the decision kernels
  double* d_upart = nullptr;        // kUserBlocksMax * (1 + kMaxK)
  std::vector<double> h_xi;
  // Krylov: partial sums, Hessenberg matrix and scalars on the device, their pinned copy
  double* d_kpart = nullptr;   // kKryBlocksMax * (kKryMaxDim + 1)
  double* d_kH = nullptr;      // (kKryMaxDim + 1) * kKryMaxDim, then 2 scalars
  double* h_kH = nullptr;      // pinned copy of d_kH
  // deferred synchronisation (lj_defer_begin / lj_defer_end): the calls
  // enqueued since lj_defer_begin and the next free slot of the status pool
  bool deferring = false;
  int defer_next = 0;
  struct DeferState* defer = nullptr;
  // allocation-free calls: this device's scratch array (device address), and
  // while such a call runs, where its workspace vectors and partial sums lie
  // in it (in doubles from its start; index W_NSLOTS: the partial sums)
  double* scratch = nullptr;
  bool in_noalloc = false;
  size_t scratch_next = 0;
  size_t scratch_off[W_NSLOTS + 1] = {};
  size_t scratch_len[W_NSLOTS + 1] = {};
};

static std::string g_create_error;

namespace {

struct Fail {
  int code;
};

#define HIPCHK(ctx, expr)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);                          \
      throw Fail{LJ_EHIP};                                                                     \
    }                                                                                          \
  } while (0)

[[noreturn]] void invalid(lj_context* ctx, const std::string& msg) {
  ctx->err = msg;
  throw Fail{LJ_EINVAL};
}

// A region of the scratch array for workspace slot s (W_NSLOTS: the partial
// sums) during an allocation-free call: handed out once per call in order of
// first use, 256-byte aligned.  The entry point has checked the total first.
double* scratch_region(lj_context* ctx, int s, size_t n) {
  if (ctx->scratch_len[s] < n) {
    const size_t rn = (n + 31) & ~(size_t)31;
    if ((ctx->scratch_next + rn) * sizeof(double) > kScratchBytes) {
      ctx->err = "allocation-free call: scratch array exhausted";
      throw Fail{LJ_EINVAL};
    }
    ctx->scratch_off[s] = ctx->scratch_next;
    ctx->scratch_len[s] = rn;
    ctx->scratch_next += rn;
  }
  return ctx->scratch + ctx->scratch_off[s];
}

double* slot(lj_context* ctx, int s, size_t n) {
  if (ctx->in_noalloc) return scratch_region(ctx, s, n);
  if (ctx->vec_cap[s] < n) {
    if (ctx->vec[s]) (void)hipFree(ctx->vec[s]);
    ctx->vec[s] = nullptr;
    ctx->vec_cap[s] = 0;
    hipError_t e = hipMalloc(&ctx->vec[s], n * sizeof(double));
    if (e != hipSuccess) {
      ctx->err = std::string("workspace allocation failed: ") + hipGetErrorString(e);
      throw Fail{LJ_ENOMEM};
    }
    ctx->vec_cap[s] = n;
  }
  return ctx->vec[s];
}

struct Opts {
  int use_proposal;
  double safety;
  int power_iters;
  int max_points;
  double hump;
  int max_substeps;
  int relative;
  double bound;
  int substeps;
  uint64_t seed;
  const double* pi_start;
  const double* bound_device;  // the bound read by the launch from device memory (when bound == 0)
  const int* skip_src = nullptr;  // the learned proposal's substep decision (device), see skip_launch
};

Opts resolve(lj_context* ctx, const lj_options* o) {
  lj_options d;
  lj_default_options(&d);
  if (!o) o = &d;
  Opts r{o->use_proposal, o->safety, o->power_iters, o->max_points, o->hump_max, o->max_substeps,
         o->relative_tol, o->bound, o->substeps, o->power_seed, o->pi_start, o->bound > 0.0 ? nullptr : o->bound_device};
  if (!(r.safety > 0.0) || !std::isfinite(r.safety)) invalid(ctx, "options: safety must be > 0");
  if (r.power_iters < 1 || r.power_iters > 100000) invalid(ctx, "options: power_iters out of range");
  if (r.max_points < 1 || r.max_points > kMaxPoints) invalid(ctx, "options: max_points must be in [1, 100]");
  if (!(r.hump > 0.0)) invalid(ctx, "options: hump_max must be > 0");
  if (r.max_substeps < 1 || r.max_substeps > (1 << 20)) invalid(ctx, "options: max_substeps out of range");
  if (!(r.bound >= 0.0) || !std::isfinite(r.bound)) invalid(ctx, "options: bound must be finite and >= 0");
  if (r.substeps < 0) invalid(ctx, "options: substeps must be >= 0");
  return r;
}

void check_range(lj_context* ctx, const void* p, size_t bytes, const std::string& what);

OpDev make_op(lj_context* ctx, const lj_operator* J) {
  if (!J) invalid(ctx, "operator is NULL");
  if (J->kind < LJ_OP_DIAG || J->kind > LJ_OP_ADR2D) invalid(ctx, "operator: unknown kind");
  if (J->nx < 1 || J->ny < 1) invalid(ctx, "operator: nx and ny must be >= 1");
  const int want_nc = family_ncomp(J->kind);
  if (J->ncomp != want_nc)
    invalid(ctx, "operator: ncomp must be 2 for the Brusselator and Gray-Scott and 1 otherwise");
  const long long n = (long long)J->nx * J->ny * J->ncomp;
  if (n > (1ll << 30)) invalid(ctx, "operator: grid too large (more than 2^30 unknowns)");
  if (J->kind == LJ_OP_DIAG && J->ny != 1) invalid(ctx, "operator: DIAG needs ny == 1");
  if (J->kind != LJ_OP_DIAG && J->kind != LJ_OP_ADVDIFF2D && J->state == nullptr)
    invalid(ctx, "operator: state is NULL");
  if (J->kind == LJ_OP_DIAG && J->state == nullptr) invalid(ctx, "operator: DIAG needs its diagonal in state");
  if (J->kind != LJ_OP_DIAG && (!(J->dx > 0.0) || !(J->dy > 0.0) || !std::isfinite(J->dx) || !std::isfinite(J->dy)))
    invalid(ctx, "operator: dx and dy must be finite and > 0");
  for (int i = 0; i < 8; ++i)
    if (!std::isfinite(J->coef[i])) invalid(ctx, "operator: non-finite coefficient");
  OpDev op;
  op.kind = J->kind;
  op.nx = J->nx;
  op.ny = J->ny;
  op.ncomp = J->ncomp;
  op.c0 = J->coef[0];
  op.c1 = J->coef[1];
  op.c2 = J->coef[2];
  op.c3 = J->coef[3];
  const double dx = (J->kind == LJ_OP_DIAG) ? 1.0 : J->dx;
  const double dy = (J->kind == LJ_OP_DIAG) ? 1.0 : J->dy;
  op.idx2 = 1.0 / (dx * dx);
  op.idy2 = 1.0 / (dy * dy);
  op.i2dx = 1.0 / (2.0 * dx);
  op.i2dy = 1.0 / (2.0 * dy);
  op.state = J->state;
  op.npts = J->nx * J->ny;
  if (op.state) {
    if (reinterpret_cast<uintptr_t>(op.state) & (op.ncomp == 2 ? 15 : 7)) invalid(ctx, "operator: state is misaligned");
    check_range(ctx, op.state, (size_t)op.npts * op.ncomp * sizeof(double), "operator state");
  }
  return op;
}

inline size_t nvals(const OpDev& op) { return (size_t)op.npts * op.ncomp; }

// A vector argument must lie inside one device allocation of this context's
// device: [p, p + n) is checked against the allocation's address range, so a
// host pointer or a short buffer is an argument error, not a memory fault.
void check_range(lj_context* ctx, const void* p, size_t bytes, const std::string& what) {
  hipDeviceptr_t base = nullptr;
  size_t size = 0;
  if (hipMemGetAddressRange(&base, &size, const_cast<void*>(p)) != hipSuccess || base == nullptr) {
    (void)hipGetLastError();
    invalid(ctx, what + " is not a device allocation");
  }
  const uintptr_t b = reinterpret_cast<uintptr_t>(base);
  const uintptr_t q = reinterpret_cast<uintptr_t>(p);
  if (q < b || q + bytes > b + size) invalid(ctx, what + " is shorter than the operator's vector length");
  hipPointerAttribute_t attr;
  if (hipPointerGetAttributes(&attr, p) == hipSuccess && attr.device != ctx->device)
    invalid(ctx, what + " lives on another device");
  (void)hipGetLastError();
}

void check_vec(lj_context* ctx, const OpDev& op, const void* p, const char* what) {
  if (!p) invalid(ctx, std::string(what) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) & (op.ncomp == 2 ? 15 : 7))
    invalid(ctx, std::string(what) + " is misaligned");
  check_range(ctx, p, (size_t)op.npts * op.ncomp * sizeof(double), what);
}

void ensure_small(lj_context* ctx, int blocks) {
  if (ctx->partial_cap < blocks) {
    if (ctx->d_partials) (void)hipFree(ctx->d_partials);
    ctx->d_partials = nullptr;
    ctx->partial_cap = 0;
    // two partial-sum areas of kRegPartStride * blocks doubles (the larger of
    // the two action kernels' strides; see grid_allreduce and reg_area)
    if (hipMalloc(&ctx->d_partials, (size_t)2 * blocks * kRegPartStride * sizeof(double)) != hipSuccess) {
      ctx->err = "partials allocation failed";
      throw Fail{LJ_ENOMEM};
    }
    ctx->partial_cap = blocks;
  }
}

// Blocks of a streaming launch: one per CU at most (barrier cost grows with
// the block count), fewer for small grids, whole rounds over the 8 XCDs.
int grid_for(lj_context* ctx, int npts) {
  const int B = persistent_block();
  int want = (npts + B - 1) / B;
  int cap = ctx->num_cus;
  if (ctx->grid_override > 0 && ctx->grid_override < cap) cap = ctx->grid_override;
  int g = want < cap ? want : cap;
  if (g >= 64) g -= g % 8;
  return g < 1 ? 1 : g;
}

// Tile plan of the LDS-resident kernel: one owned point per thread, halo S,
// at most 3 extended points per thread, LDS (two buffers) within 64 KiB with
// the kernel's static LDS, at most one tile per CU.  The largest tile that
// fits wins (fewest blocks: the barrier is the per-super-step cost).
struct TilePlan {
  bool ok = false;
  int tx = 0, ty = 0, ntx = 0, nty = 0, ept = 0;
  size_t lds = 0;   // dynamic LDS bytes
  int lds_h = 0;    // offset of the step history (doubles)
};

TilePlan tile_plan(lj_context* ctx, const OpDev& op) {
  TilePlan best;
  if (ctx->force_stream || action_tile_ptr(op.kind, 1, kMaxK) == nullptr) return best;
  const int S = tile_halo();
  const int B = persistent_block();
  static const int cand[][2] = {{32, 32}, {64, 16}, {32, 16}, {16, 16}, {16, 8}, {8, 8}};
  for (const auto& c : cand) {
    int tx = c[0], ty = c[1];
    if (ctx->tile_override_x > 0) {
      tx = ctx->tile_override_x;
      ty = ctx->tile_override_y;
    }
    const int w = tx < op.nx ? tx : op.nx, h = ty < op.ny ? ty : op.ny;
    const int ntx = (op.nx + tx - 1) / tx, nty = (op.ny + ty - 1) / ty;
    const long ne = (long)(w + 2 * S) * (h + 2 * S);
    const int ept = (int)((ne + B - 1) / B);
    // two extended-tile buffers and S owned values per thread
    const size_t lds = ((size_t)2 * ne + (size_t)S * B) * sizeof(double);
    const bool fits = tx * ty <= B && ept <= 3 && lds + kStaticLdsReserve <= (size_t)ctx->lds_max &&
                      (long)ntx * nty <= ctx->num_cus;
    if (fits) {
      best.ok = true;
      best.tx = tx;
      best.ty = ty;
      best.ntx = ntx;
      best.nty = nty;
      best.ept = ept;
      best.lds = lds;
      best.lds_h = (int)(2 * ne);
      return best;
    }
    if (ctx->tile_override_x > 0) return best;
  }
  return best;
}

// Register-tiled kernel: 32 x 32 tiles, one per block with the step history
// in dynamic LDS when they fit one per CU (at most 256, the partial-sum
// reduction's assumption), else several per block.
struct RegPlan {
  bool ok = false;
  bool full = false;   // every tile is 32 x 32
  bool multi = false;  // more tiles than blocks: several per block
  int ntx = 0, nty = 0;
  int blocks = 0;
  size_t lds = 0;
};

RegPlan reg_plan(lj_context* ctx, const OpDev& op, int K) {
  RegPlan r;
  if (ctx->force_stream || ctx->no_reg || ctx->tile_override_x > 0 || action_reg_ptr(op.kind, K, true) == nullptr)
    return r;
  const int ntx = (op.nx + 31) / 32, nty = (op.ny + 31) / 32;
  const long T = (long)ntx * nty;
  const bool full = op.nx % 32 == 0 && op.ny % 32 == 0;
  if (T > ctx->num_cus || T > 256) {
    // several tiles per block: not in the allocation-free path (it needs
    // 3 + (1 + kRegSnap) K workspace vectors)
    if (ctx->in_noalloc || action_regm_ptr(op.kind, K, full) == nullptr) return r;
    if (reg_static_lds() > (size_t)ctx->lds_max) return r;
    r.ok = true;
    r.full = full;
    r.multi = true;
    r.ntx = ntx;
    r.nty = nty;
    r.blocks = std::min(ctx->num_cus, 256);
    r.lds = 0;
    return r;
  }
  if (reg_lds_bytes() + reg_static_lds() > (size_t)ctx->lds_max) return r;
  r.ok = true;
  r.full = full;
  r.ntx = ntx;
  r.nty = nty;
  r.blocks = (int)T;
  r.lds = reg_lds_bytes();
  return r;
}

// ---- one phi-action launch ------------------------------------------------
struct ActOut {
  bool aborted;  // a grid barrier timed out: the launch must be repeated cooperatively
  int skipped;   // the launch did no work: the proposal's request (LejaStatus.skipped)
  int state[kMaxK];
  int m_star[kMaxK];
  double err[kMaxK];
  int iters;
  int power_iters;
  double lam, c, gamma, vnorm;
};

// A launch whose status head is read later: its slot in the pinned pool.
struct PendingLaunch {
  int slot;
  int K;
  bool tiled;
  hipEvent_t* ev;
};

// A call enqueued in a deferral, with what lj_defer_end needs to complete
// it: its launches' status slots, and its arguments for a synchronous redo.
struct DeferredCall {
  bool is_step = false;
  int scheme = 0;  // step
  OpDev op{};
  Opts o{};
  double h = 0.0, tol = 0.0;
  double* u_out = nullptr;  // step
  double* err = nullptr;    // step
  const double* v = nullptr;  // action
  double* w = nullptr;        // action
  int l = 0;                  // action
  lj_stats* stats = nullptr;  // the caller's, filled by lj_defer_end
  std::vector<PendingLaunch> launches;
};

}  // namespace

struct DeferState {
  std::vector<DeferredCall> calls;
};

namespace {

// Where the bound of a launch comes from and goes to (device pointers, or none).
struct BoundLink {
  const double* src = nullptr;  // read the bound here (no power iteration)
  double* dst = nullptr;        // write the bound used here
};

// Whether every block of a G-block launch of `fn` fits on the device at once,
// so that a plain launch keeps them co-resident (the cooperative launch
// guarantees it but costs ~12 us more per launch).
bool coresident(lj_context* ctx, const void* fn, int G, size_t dyn, int block) {
  if (ctx->force_coop) return false;
  const auto key = std::make_pair(fn, dyn);
  auto it = ctx->occupancy.find(key);
  int nb = 0;
  if (it == ctx->occupancy.end()) {
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, fn, block, dyn) != hipSuccess) {
      (void)hipGetLastError();
      nb = 0;
    }
    ctx->occupancy[key] = nb;
  } else {
    nb = it->second;
  }
  return nb >= 1 && G <= ctx->num_cus * nb;
}

// Enqueues one action launch and the copy of its status head (everything but
// the trace) into `status_dst` (pinned host memory), without waiting.  `ev` (may be
// NULL) receives a start / end event pair around the launch.
void launch_action(lj_context* ctx, const OpDev& op, const double* v, int K, const int* l, const double* s_k,
                   double lam_host, uint64_t seed, const double* start, double* const* outs, const Opts& o,
                   double tol, hipStream_t s, const BoundLink& link, LejaStatus* status_dst, size_t status_bytes,
                   hipEvent_t* ev, bool* tiled, bool cooperative = false, bool direct_status = false) {
  const size_t n = nvals(op);
  ActionParams P;
  std::memset(&P, 0, sizeof(P));
  P.op = op;
  P.do_power = (lam_host > 0.0 || link.src != nullptr) ? 0 : 1;
  P.power_iters = o.power_iters;
  P.seed = seed;
  P.start = start;
  P.lam_in = lam_host;
  P.lam_src = link.src;
  P.skip_src = o.skip_src;
  P.lam_out = link.dst;
  P.safety = o.safety;
  P.v = v;
  P.K = K;
  for (int k = 0; k < kMaxK; ++k) {
    P.l[k] = (k < K) ? l[k] : 0;
    P.s[k] = (k < K) ? s_k[k] : 0.0;
    P.p[k] = (k < K) ? outs[k] : nullptr;
  }
  P.max_points = o.max_points;
  P.relative = o.relative;
  P.tol = tol;
  P.hump = o.hump;
  P.xi = ctx->d_xi;
  P.ybuf0 = slot(ctx, W_Y0, n);
  P.ybuf1 = slot(ctx, W_Y1, n);
  P.barrier = ctx->d_barrier;
  P.spin_limit = (!cooperative && ctx->forced_spin_limit > 0) ? ctx->forced_spin_limit : kGridSpinLimit;
  P.status = ctx->d_status;
  // a header-only status into a slot of the pinned pool is written by the
  // kernel itself; otherwise it is copied after the launch
  P.status_host = direct_status ? status_dst : nullptr;
  const RegPlan rp = reg_plan(ctx, op, K);
  const TilePlan tp = rp.ok ? TilePlan{} : tile_plan(ctx, op);
  void* fn = nullptr;
  int G = 0;
  size_t dyn = 0;
  int block = persistent_block();
  if (rp.ok) {
    fn = rp.multi ? action_regm_ptr(op.kind, K, rp.full) : action_reg_ptr(op.kind, K, rp.full);
    P.tx = 32;
    P.ty = 32;
    P.ntx = rp.ntx;
    P.nty = rp.nty;
    G = rp.blocks;
    dyn = rp.lds;
    block = reg_block();
    if (rp.multi) {
      P.ybuf2 = slot(ctx, W_Y2, n);
      for (int k = 0; k < K; ++k) P.pw[k] = slot(ctx, W_PW0 + k, n);
      P.snap = slot(ctx, W_SNAP, (size_t)K * kRegSnap * n);
    }
    if (dyn > 64 * 1024 && ctx->dyn_lds[fn] < dyn) {
      HIPCHK(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
      ctx->dyn_lds[fn] = dyn;
    }
  } else if (tp.ok) {
    fn = action_tile_ptr(op.kind, tp.ept, K);
    P.tx = tp.tx;
    P.ty = tp.ty;
    P.ntx = tp.ntx;
    P.nty = tp.nty;
    P.lds_h = tp.lds_h;
    G = tp.ntx * tp.nty;
    dyn = tp.lds;
    if (dyn > 64 * 1024 && ctx->dyn_lds[fn] < dyn) {
      HIPCHK(ctx, hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
      ctx->dyn_lds[fn] = dyn;
    }
  } else {
    fn = action_stream_ptr(op.kind, K);
    G = grid_for(ctx, op.npts);
  }
  if (ctx->in_noalloc) {
    P.partials = scratch_region(ctx, W_NSLOTS, (size_t)2 * kRegPartStride * G);
  } else {
    ensure_small(ctx, G);
    P.partials = ctx->d_partials;
  }
  void* args[] = {&P};
  if (ev) HIPCHK(ctx, hipEventRecord(ev[0], s));
  if (cooperative || !coresident(ctx, fn, G, dyn, block)) {
    HIPCHK(ctx, hipLaunchCooperativeKernel(fn, dim3(G), dim3(block), args, (unsigned)dyn, s));
  } else {
    HIPCHK(ctx, hipLaunchKernel(fn, dim3(G), dim3(block), args, (unsigned)dyn, s));
  }
  if (ev) HIPCHK(ctx, hipEventRecord(ev[1], s));
  if (!direct_status) HIPCHK(ctx, hipMemcpyAsync(status_dst, ctx->d_status, status_bytes, hipMemcpyDeviceToHost, s));
  if (tiled) *tiled = tp.ok || rp.ok;
}

// Outcome of a launch whose status has arrived; accumulates the timing
// counters when `ev` holds its (completed) event pair.
ActOut finish_action(lj_context* ctx, const OpDev& op, const LejaStatus& S, hipEvent_t* ev, bool tiled) {
  ActOut r;
  r.aborted = S.aborted != 0;
  r.skipped = S.skipped;
  if (r.aborted) ctx->tm.aborts += 1;
  for (int k = 0; k < kMaxK; ++k) {
    r.state[k] = S.state[k];
    r.m_star[k] = S.m_star[k];
    r.err[k] = S.err[k];
  }
  r.iters = S.iters;
  r.power_iters = S.power_iters;
  r.lam = S.lam;
  r.c = S.c;
  r.gamma = S.gamma;
  r.vnorm = S.vnorm;
  if (ev) {
    ctx->tev_pending.push_back((int)((ev - ctx->tev.data()) / 2));
    ctx->tm.launches += 1;
    ctx->tm.iterations += S.iters;
    ctx->tm.point_iters += (int64_t)S.iters * op.npts;
    ctx->tm.accum_point_iters += (int64_t)S.accum_iters * op.npts;
    ctx->tm.power_point_iters += (int64_t)S.power_iters * op.npts;
    ctx->tm.tiled_launches += tiled ? 1 : 0;
  }
  return r;
}

// Adds the elapsed times of the finished, unread launches to the counters and
// frees the pool.
void timing_flush(lj_context* ctx) {
  for (int pair : ctx->tev_pending) {
    float ms = 0.f;
    HIPCHK(ctx, hipEventSynchronize(ctx->tev[2 * pair + 1]));
    HIPCHK(ctx, hipEventElapsedTime(&ms, ctx->tev[2 * pair], ctx->tev[2 * pair + 1]));
    ctx->tm.kernel_ms += ms;
  }
  ctx->tev_pending.clear();
  ctx->tev_next = 0;
}

// The event pair for the next timed launch (nullptr when timing is off).  A
// full pool is read out first; launches still in flight then hold pairs the
// caller has not finished yet, so the pool is only recycled between steps.
hipEvent_t* timing_pair(lj_context* ctx) {
  if (!ctx->timing) return nullptr;
  if (ctx->tev_next >= kTimingPairs) timing_flush(ctx);
  return &ctx->tev[2 * ctx->tev_next++];
}

// K accumulators phi_{l_k}(s_k J) v (K = 0: power iteration only), one
// launch, synchronised.  The bound is lam_host when > 0, else the power
// iteration runs inside the launch.
// ---- user operators ------------------------------------------------------------
// OpDev.kind of an operator given as callbacks: never passed to a family kernel
// (run_action and the stage driver route it to the user path).
constexpr int kUserKind = 100;

bool is_user(const OpDev& op) { return op.kind == kUserKind; }

void call_rhs(lj_context* ctx, const double* x, double* fx, hipStream_t s) {
  const UserOp* U = ctx->uop;
  if (!U->J.rhs) invalid(ctx, "user operator: rhs is NULL (needed here)");
  const int rc = U->J.rhs(U->J.user, x, fx, reinterpret_cast<void*>(s));
  if (rc != 0) invalid(ctx, "user rhs callback failed with code " + std::to_string(rc));
}

void call_jv(lj_context* ctx, const double* x, double* jx, hipStream_t s) {
  const UserOp* U = ctx->uop;
  const int rc = U->J.jv(U->J.user, U->J.state, x, jx, reinterpret_cast<void*>(s));
  if (rc != 0) invalid(ctx, "user jv callback failed with code " + std::to_string(rc));
}

// out = J(u) x: the user's product, or a finite difference with its own step
void user_jv(lj_context* ctx, const double* x, double* out, hipStream_t s) {
  const UserOp* U = ctx->uop;
  if (!U->fd) {
    call_jv(ctx, x, out, s);
    return;
  }
  const long n = (long)U->J.n;
  HIPCHK(ctx, launch_user_fd_step(ctx->d_ustate, x, n, ctx->d_upart, s));
  double* pt = slot(ctx, W_UPT, n);
  HIPCHK(ctx, launch_user_fd_point(ctx->d_ustate, U->J.state, x, n, pt, s));
  double* fx = slot(ctx, W_UJ, n);
  call_rhs(ctx, pt, fx, s);
  HIPCHK(ctx, launch_user_fd_quotient(ctx->d_ustate, fx, U->fu, n, out, s));
}

// Power iteration on a user operator (the products of the other paths, same
// start vector and estimate): K products, x_{k+1} = J x_k / ||J x_k||.
double user_power(lj_context* ctx, long n, int iters, uint64_t seed, const double* start, hipStream_t s) {
  const UserOp* U = ctx->uop;
  double* xa = slot(ctx, W_UPA, n);
  double* xb = slot(ctx, W_UPB, n);
  double* jb = slot(ctx, W_UJ, n);
  double* yb = slot(ctx, W_UY, n);
  double* pt = slot(ctx, W_UPT, n);
  if (start) {
    HIPCHK(ctx, hipMemcpyAsync(xa, start, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  } else {
    HIPCHK(ctx, launch_user_start_vector(xa, n, seed, s));
  }
  HIPCHK(ctx, launch_user_power_init(ctx->d_ustate, s));
  double* cur = xa;
  double* nxt = xb;
  for (int k = 0; k < iters; ++k) {
    if (U->fd) {
      HIPCHK(ctx, launch_user_fd_step(ctx->d_ustate, cur, n, ctx->d_upart, s));
      HIPCHK(ctx, launch_user_fd_point(ctx->d_ustate, U->J.state, cur, n, pt, s));
      call_rhs(ctx, pt, jb, s);
      HIPCHK(ctx, launch_user_power(ctx->d_ustate, cur, jb, U->fu, yb, nxt, n, ctx->d_upart, ctx->h_ustatus, s));
    } else {
      call_jv(ctx, cur, jb, s);
      HIPCHK(ctx, launch_user_power(ctx->d_ustate, cur, jb, nullptr, nullptr, nxt, n, ctx->d_upart,
                                    ctx->h_ustatus, s));
    }
    std::swap(cur, nxt);
  }
  HIPCHK(ctx, hipStreamSynchronize(s));
  return ctx->h_ustatus->lam;
}

// Steps between the host's reads of the decisions: at most this many minus
// one products past the last needed one are computed and discarded.
constexpr int kUserPoll = 4;

// One vertical Newton recurrence on a user operator (the run_action of the
// callback path): power iteration unless lam_host > 0, divided differences,
// then per step the user's product, the recurrence kernel and the decision
// kernel.
ActOut run_action_user(lj_context* ctx, const OpDev& op, const double* v, int K, const int* l, const double* s_k,
                       double lam_host, uint64_t seed, const double* start, double* const* outs, const Opts& o,
                       double tol, hipStream_t s) {
  const UserOp* U = ctx->uop;
  const long n = op.npts;
  ActOut r;
  std::memset(&r, 0, sizeof(r));
  r.aborted = false;
  for (int k = 0; k < kMaxK; ++k) {
    r.state[k] = ACC_CONVERGED;
    r.m_star[k] = -1;
  }
  double lam = lam_host;
  if (!(lam > 0.0)) {
    lam = user_power(ctx, n, o.power_iters, seed, start, s);
    r.power_iters = o.power_iters;
  }
  const double alpha = -o.safety * lam;
  const double c = 0.5 * (alpha + 0.0);
  const double gamma = 0.25 * (0.0 - alpha);
  r.lam = lam;
  r.c = c;
  r.gamma = gamma;
  if (K == 0) return r;
  if (!(gamma > 0.0)) invalid(ctx, "user operator: the spectral bound is zero (J v = 0 for the start vector)");
  const double rgamma = 1.0 / gamma;
  DDParams P;
  std::memset(&P, 0, sizeof(P));
  P.K = K;
  for (int k = 0; k < K; ++k) {
    P.l[k] = l[k];
    P.s[k] = s_k[k];
  }
  P.npts = o.max_points + 1;
  P.c = c;
  P.gamma = gamma;
  P.xi = ctx->d_xi;
  P.coef = ctx->d_coef;
  P.fmax = ctx->d_fmax;
  HIPCHK(ctx, launch_divdiff(P, s));
  UserRec R;
  std::memset(&R, 0, sizeof(R));
  R.n = n;
  R.K = K;
  R.coef = ctx->d_coef;
  R.fmax = ctx->d_fmax;
  for (int k = 0; k < K; ++k) R.p[k] = outs[k];
  R.part = ctx->d_upart;
  R.st = ctx->d_ustate;
  R.host = ctx->h_ustatus;
  HIPCHK(ctx, launch_user_rec_start(R, v, o.max_points, tol, o.relative, o.hump, U->fd ? 1 : 0, s));
  double* yb[2] = {slot(ctx, W_Y0, n), slot(ctx, W_Y1, n)};
  double* jb = slot(ctx, W_UJ, n);
  double* pt = slot(ctx, W_UPT, n);
  const double* yp = v;
  HIPCHK(ctx, hipStreamSynchronize(s));
  // written by the decision kernels; read between synchronisations as a hint
  // (a stale value only enqueues a step whose work is discarded)
  const volatile int* done = &ctx->h_ustatus->done;
  for (int m = 1; m <= o.max_points && !*done; ++m) {
    if (U->fd) {
      HIPCHK(ctx, launch_user_fd_point(ctx->d_ustate, U->J.state, yp, n, pt, s));
      call_rhs(ctx, pt, jb, s);
    } else {
      call_jv(ctx, yp, jb, s);
    }
    double* y = yb[m & 1];
    HIPCHK(ctx, launch_user_rec_step(R, m, jb, U->fd ? U->fu : nullptr, yp, y, c, gamma, rgamma,
                                     ctx->h_xi[m - 1], s));
    HIPCHK(ctx, launch_user_rec_decide(R, m, s));
    yp = y;
    if (m % kUserPoll == 0 || m == o.max_points) HIPCHK(ctx, hipStreamSynchronize(s));
  }
  HIPCHK(ctx, hipStreamSynchronize(s));
  const UserStatus& S = *ctx->h_ustatus;
  for (int k = 0; k < K; ++k) {
    r.state[k] = S.state[k];
    r.m_star[k] = S.m_star[k];
    r.err[k] = S.err[k];
  }
  r.iters = S.iters;
  r.vnorm = S.nv;
  return r;
}

ActOut run_action(lj_context* ctx, const OpDev& op, const double* v, int K, const int* l, const double* s_k,
                  double lam_host, uint64_t seed, const double* start, double* const* outs, const Opts& o,
                  double tol, hipStream_t s) {
  if (is_user(op)) return run_action_user(ctx, op, v, K, l, s_k, lam_host, seed, start, outs, o, tol, s);
  bool tiled = false;
  BoundLink link;
  if (!(lam_host > 0.0) && o.bound_device) link.src = o.bound_device;
  for (int attempt = 0; attempt < 2; ++attempt) {
    hipEvent_t* ev = timing_pair(ctx);
    launch_action(ctx, op, v, K, l, s_k, lam_host, seed, start, outs, o, tol, s, link, ctx->h_status,
                  offsetof(LejaStatus, trace), ev, &tiled, attempt == 1, true);
    HIPCHK(ctx, hipStreamSynchronize(s));
    const ActOut r = finish_action(ctx, op, *ctx->h_status, ev, tiled);
    if (!r.aborted) return r;
  }
  ctx->err = "an action launch aborted twice (grid barrier timed out)";
  throw Fail{LJ_EHIP};
}

double run_bound(lj_context* ctx, const OpDev& op, const Opts& o, int iters, uint64_t seed, const double* start,
                 hipStream_t s) {
  Opts q = o;
  q.power_iters = iters;
  ActOut r = run_action(ctx, op, nullptr, 0, nullptr, nullptr, 0.0, seed, start, nullptr, q, 1.0, s);
  return r.lam;
}

void lincomb(lj_context* ctx, size_t n, double* out, int nin, const double* alpha, const double* const* x,
             hipStream_t s) {
  LinComb L;
  L.n = (long)n;
  L.nin = nin;
  for (int q = 0; q < 5; ++q) {
    L.alpha[q] = (q < nin) ? alpha[q] : 0.0;
    L.x[q] = (q < nin) ? x[q] : nullptr;
  }
  L.out = out;
  HIPCHK(ctx, launch_lincomb(L, s));
}

double factorial(int k) {
  double f = 1.0;
  for (int i = 2; i <= k; ++i) f *= (double)i;
  return f;
}

// phi_l(T J) v with s = s_start, 2 s_start, ... substeps (the identity
// w(t + tau) = e^{tau J} w(t) + sum_j tau^j t^{l-j}/(l-j)! phi_j(tau J) v for
// w(t) = t^l phi_l(t J) v, scaled by T^l).  Returns true on success.
bool substepped(lj_context* ctx, const OpDev& op, const double* v, int l, double T, int s_start,
                double lam, const Opts& o, double tol, double* w_out, lj_stats* st, int k,
                hipStream_t strm) {
  const size_t n = nvals(op);
  int s = s_start;
  while (s <= o.max_substeps) {
    const double tau = T / (double)s;
    bool ok = true;
    int used = 0;
    if (l == 0) {
      const double* in = v;
      for (int i = 0; i < s && ok; ++i) {
        double* out = (i == s - 1) ? w_out : slot(ctx, (i & 1) ? W_SW1 : W_SW0, n);
        const int l0 = 0;
        const double sk = tau;
        ActOut r = run_action(ctx, op, in, 1, &l0, &sk, lam, 0, nullptr, &out, o, tol, strm);
        used += r.iters;
        if (r.state[0] != ACC_CONVERGED) ok = false;
        in = out;
      }
    } else {
      double* P[kMaxK];
      int ls[kMaxK];
      double ss[kMaxK];
      for (int j = 0; j < l; ++j) {
        P[j] = slot(ctx, W_P0 + j, n);
        ls[j] = j + 1;
        ss[j] = tau;
      }
      ActOut r = run_action(ctx, op, v, l, ls, ss, lam, 0, nullptr, P, o, tol, strm);
      used += r.iters;
      for (int j = 0; j < l; ++j)
        if (r.state[j] != ACC_CONVERGED) ok = false;
      if (ok) {
        double* cur = (s == 1) ? w_out : slot(ctx, W_SW0, n);
        {
          const double a = 1.0 / std::pow((double)s, (double)l);
          const double* x[1] = {P[l - 1]};
          lincomb(ctx, n, cur, 1, &a, x, strm);
        }
        for (int i = 1; i < s && ok; ++i) {
          double* e = slot(ctx, W_SE, n);
          const int l0 = 0;
          const double sk = tau;
          ActOut r2 = run_action(ctx, op, cur, 1, &l0, &sk, lam, 0, nullptr, &e, o, tol, strm);
          used += r2.iters;
          if (r2.state[0] != ACC_CONVERGED) {
            ok = false;
            break;
          }
          double* nxt = (i == s - 1) ? w_out : slot(ctx, (cur == ctx->vec[W_SW0]) ? W_SW1 : W_SW0, n);
          double alpha[5];
          const double* xs[5];
          alpha[0] = 1.0;
          xs[0] = e;
          for (int j = 1; j <= l; ++j) {
            alpha[j] = std::pow((double)i, (double)(l - j)) / (factorial(l - j) * std::pow((double)s, (double)l));
            xs[j] = P[j - 1];
          }
          lincomb(ctx, n, nxt, l + 1, alpha, xs, strm);
          cur = nxt;
        }
      }
    }
    st->iters_total += used;
    if (ok) {
      st->substeps[k] = s;
      st->m_star[k] = used;
      return true;
    }
    st->rejections += 1;
    s *= 2;
  }
  st->substeps[k] = s / 2;
  st->m_star[k] = -1;
  return false;
}

// A bound the caller keeps in device memory, read on the host (synchronises).
double bound_to_host(lj_context* ctx, const double* dev, hipStream_t s) {
  double lam = 0.0;
  HIPCHK(ctx, hipMemcpyAsync(&lam, dev, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (!(lam > 0.0) || !std::isfinite(lam)) invalid(ctx, "options: bound_device holds no positive finite bound");
  return lam;
}

// Vertical action (the core of lj_phi_action / lj_phi_vertical / lj_step).
int vertical_impl(lj_context* ctx, const OpDev& op, const double* v, int K, const int* l, const double* a,
                  double h, double tol, double* const* w, const Opts& o, lj_stats* st, hipStream_t s) {
  std::memset(st, 0, sizeof(*st));
  for (int k = 0; k < LJ_MAX_K; ++k) {
    st->m_star[k] = -1;
    st->substeps[k] = 1;
  }
  double lam = o.bound > 0.0 ? o.bound : 0.0;
  int s0 = (o.substeps > 1) ? o.substeps : 1;
  if (!(lam > 0.0) && o.bound_device && (s0 > 1 || is_user(op))) lam = bound_to_host(ctx, o.bound_device, s);
  std::vector<int> pending;
  Opts os = o;  // the later launches never take the learned proposal's skip
  os.skip_src = nullptr;
  bool interval_needed = (s0 > 1);
  if (s0 == 1) {
    double sk[kMaxK];
    for (int k = 0; k < K; ++k) sk[k] = a[k] * h;
    ActOut r = run_action(ctx, op, v, K, l, sk, lam, o.seed, o.pi_start, w, o, tol, s);
    if (o.skip_src != nullptr) {  // the learned proposal's attempt (lj_phi_vertical)
      st->proposal_bound = r.skipped >= 0 ? r.lam : 0.0;
      st->proposal_substeps = r.skipped == 0 ? 1 : (r.skipped > 0 ? r.skipped : 0);
    }
    if (r.skipped < 0) return LJ_ENOTCONV;  // no usable proposal: every accumulator pending
    if (r.skipped > 1) {
      // the proposal asked for substeps and the launch did no work: one
      // attempt at that count with the bound it read
      os.max_substeps = r.skipped;
      os.bound_device = nullptr;
      lam = r.lam;
      s0 = r.skipped;
      interval_needed = true;
    } else {
      st->power_iters = r.power_iters;
      st->iters_total += r.iters;
      lam = r.lam;
      st->bound = r.lam;
      st->c = r.c;
      st->gamma = r.gamma;
      for (int k = 0; k < K; ++k) {
        if (r.state[k] == ACC_CONVERGED) {
          st->m_star[k] = r.m_star[k];
          st->err_est[k] = r.err[k];
        } else {
          pending.push_back(k);
        }
      }
      if (!pending.empty()) st->rejections += 1;
      s0 = 2;
    }
  }
  if (interval_needed) {
    if (!(lam > 0.0)) {
      lam = run_bound(ctx, op, os, o.power_iters, o.seed, o.pi_start, s);
      st->power_iters = o.power_iters;
    }
    double c = 0.0, gamma = 0.0;
    {
      const double alpha = -o.safety * lam;
      c = 0.5 * (alpha + 0.0);
      gamma = 0.25 * (0.0 - alpha);
    }
    st->bound = lam;
    st->c = c;
    st->gamma = gamma;
    for (int k = 0; k < K; ++k) pending.push_back(k);
  }
  bool all_ok = true;
  for (int k : pending) {
    if (!substepped(ctx, op, v, l[k], a[k] * h, s0, lam, os, tol, w[k], st, k, s)) all_ok = false;
  }
  st->converged = all_ok ? 1 : 0;
  return all_ok ? LJ_OK : LJ_ENOTCONV;
}

void check_action_args(lj_context* ctx, const OpDev& op, const double* v, int K, const int* l, const double* a,
                       double h, double tol, double* const* w) {
  if (K < 1 || K > LJ_MAX_K) invalid(ctx, "K must be in [1, 4]");
  if (!l || !a || !w) invalid(ctx, "l, a and w must not be NULL");
  if (!std::isfinite(h)) invalid(ctx, "h must be finite");
  if (!(tol > 0.0) || !std::isfinite(tol)) invalid(ctx, "tol must be finite and > 0");
  check_vec(ctx, op, v, "v");
  for (int k = 0; k < K; ++k) {
    if (l[k] < 0 || l[k] > LJ_MAX_L) invalid(ctx, "l must be in [0, 4]");
    if (!std::isfinite(a[k])) invalid(ctx, "a[k] must be finite");
    check_vec(ctx, op, w[k], "w[k]");
    if (w[k] == v) invalid(ctx, "w must not alias v");
    if (w[k] == op.state) invalid(ctx, "w must not alias the operator state");
    for (int q = 0; q < k; ++q)
      if (w[q] == w[k]) invalid(ctx, "the outputs w[k] must be distinct");
  }
}

// ---- user operators: per-call setup ------------------------------------------------
void user_alloc(lj_context* ctx) {
  if (!ctx->d_ustate) HIPCHK(ctx, hipMalloc(&ctx->d_ustate, sizeof(UserState)));
  if (!ctx->h_ustatus) {
    HIPCHK(ctx, hipHostMalloc(&ctx->h_ustatus, sizeof(UserStatus), hipHostMallocCoherent));
    std::memset(ctx->h_ustatus, 0, sizeof(UserStatus));
  }
  if (!ctx->d_upart) HIPCHK(ctx, hipMalloc(&ctx->d_upart, (size_t)kUserBlocksMax * (1 + kMaxK) * sizeof(double)));
  if (ctx->h_xi.empty()) {
    ctx->h_xi.resize(kTable);
    if (leja_points_host(ctx->h_xi.data(), kTable) != 0) invalid(ctx, "internal: Leja table");
  }
}

// A call on a user operator: checks it, makes it the context's current user
// operator, evaluates f(u) once when finite-difference products or the stage
// driver need it, and ||u|| for the finite-difference step.
struct UserScope {
  lj_context* ctx;
  UserOp U;
  OpDev op;
  UserScope(lj_context* c, const lj_user_operator* J, bool need_rhs, hipStream_t s) : ctx(c) {
    if (!J) invalid(ctx, "user operator is NULL");
    if (J->n < 1 || J->n > (1ll << 30)) invalid(ctx, "user operator: n must be in [1, 2^30]");
    if (!J->jv && !J->rhs) invalid(ctx, "user operator: give jv, rhs or both");
    if (need_rhs && !J->rhs) invalid(ctx, "user operator: the stage driver needs rhs");
    if (!J->state) invalid(ctx, "user operator: state is NULL");
    if (ctx->uop) invalid(ctx, "a user-operator call is already running on this context");
    U.J = *J;
    U.fd = (J->jv == nullptr);
    std::memset(&op, 0, sizeof(op));
    op.kind = kUserKind;
    op.nx = (int)J->n;
    op.ny = 1;
    op.ncomp = 1;
    op.npts = (int)J->n;
    op.state = J->state;
    check_vec(ctx, op, J->state, "user operator state");
    user_alloc(ctx);
    ctx->uop = &U;
    try {
      if (U.fd) {
        double* fu = slot(ctx, W_UFU, (size_t)J->n);
        call_rhs(ctx, J->state, fu, s);
        U.fu = fu;
        HIPCHK(ctx, launch_user_norm_u(ctx->d_ustate, J->state, (long)J->n, ctx->d_upart, s));
      }
    } catch (...) {
      ctx->uop = nullptr;
      throw;
    }
  }
  ~UserScope() { ctx->uop = nullptr; }
  UserScope(const UserScope&) = delete;
  UserScope& operator=(const UserScope&) = delete;
};

// ---- learned proposal --------------------------------------------------------
constexpr int kMaxEpochs = 4096;

void mlp_alloc(lj_context* ctx) {
  if (ctx->d_model) return;
  HIPCHK(ctx, hipMalloc(&ctx->d_model, kModelFloats * sizeof(float)));
  HIPCHK(ctx, hipMalloc(&ctx->d_adam, 2 * kMlpParams * sizeof(float)));
  HIPCHK(ctx, hipMalloc(&ctx->d_adam_t, sizeof(int)));
  HIPCHK(ctx, hipMalloc(&ctx->d_rows, (size_t)kMlpBlock * kMlpRowFloats * sizeof(float)));
  HIPCHK(ctx, hipMalloc(&ctx->d_scalars, (1 + kMaxEpochs) * sizeof(float)));
  HIPCHK(ctx, hipMalloc(&ctx->d_featpart, feature_partial_bytes()));
  HIPCHK(ctx, hipMalloc(&ctx->d_feats, kMaxK * kMlpIn * sizeof(float)));
  HIPCHK(ctx, hipMalloc(&ctx->d_pred, kMaxK * kMlpOut * sizeof(float)));
  HIPCHK(ctx, hipMalloc(&ctx->d_gers, sizeof(double)));
  HIPCHK(ctx, hipMalloc(&ctx->d_prop, sizeof(ProposalOut)));
}

// Glorot uniform weights a (2U - 1), a = sqrt(6 / (fan_in + fan_out)), U the
// SplitMix64 uniforms of the seed in parameter order; zero biases; identity
// standardisation.
void mlp_host_init(uint64_t seed, std::vector<float>& m) {
  m.assign(kModelFloats, 0.0f);
  auto fill = [&](int off, int fo, int fi) {
    const double a = std::sqrt(6.0 / (fo + fi));
    for (int i = 0; i < fo * fi; ++i) {
      uint64_t z = seed + (uint64_t)(off + i + 1) * 0x9E3779B97F4A7C15ull;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z = z ^ (z >> 31);
      const double u = (double)(z >> 11) * 0x1.0p-53;
      m[off + i] = (float)(a * (2.0 * u - 1.0));
    }
  };
  fill(kOffW1, kMlpHidden, kMlpIn);
  fill(kOffW2, kMlpHidden, kMlpHidden);
  fill(kOffW3, kMlpOut, kMlpHidden);
  for (int k = 0; k < kMlpIn; ++k) m[kMlpParams + kMlpIn + k] = 1.0f;             // sd
  for (int k = 0; k < kMlpOut; ++k) m[kMlpParams + 2 * kMlpIn + kMlpOut + k] = 1.0f;  // tsd
}

void check_fvec(lj_context* ctx, const void* p, size_t count, const char* what) {
  if (!p) invalid(ctx, std::string(what) + " is NULL");
  if (reinterpret_cast<uintptr_t>(p) & 3) invalid(ctx, std::string(what) + " is misaligned");
  check_range(ctx, p, count * sizeof(float), what);
}

// The proposal for the K actions phi_{l_k}(a_k h J) v, decided on the
// device: features of (J, a_k h, l_k) with the Gershgorin bound G of J, the
// network, and the decision kernel, which writes the bound and the substep
// count into ctx->d_prop.  Nothing is read back: the attempt's launch reads
// both from there.
void propose(lj_context* ctx, const OpDev& op, int K, const int* l, const double* a, double h, int max_substeps,
             hipStream_t s) {
  if (!ctx->mlp_ready) invalid(ctx, "use_proposal: no trained network (lj_mlp_train, lj_mlp_set or lj_mlp_load)");
  FeatureJob J;
  std::memset(&J, 0, sizeof(J));
  J.op = op;
  J.K = K;
  for (int k = 0; k < K; ++k) {
    J.h[k] = a[k] * h;
    J.l[k] = l[k];
  }
  HIPCHK(ctx, launch_features(J, ctx->d_featpart, ctx->d_feats, ctx->d_gers, s));
  HIPCHK(ctx, launch_mlp_forward(ctx->d_model, ctx->d_feats, K, ctx->d_pred, s));
  HIPCHK(ctx, launch_proposal_decide(ctx->d_pred, K, ctx->d_gers, LJ_PROPOSAL_MARGIN, max_substeps, ctx->d_prop, s));
}

// Runs an entry point: device selection, error text, no exception across the
// ABI.  While a user operator's callback runs (ctx->uop set), only the entry
// points that use no workspace (lj_rhs, lj_jv: in_callback_ok) may be called
// on the same context; the others would overwrite the running call's vectors.
template <class F>
int guarded(lj_context* ctx, F&& f, bool in_callback_ok = false) {
  if (!ctx) return LJ_EINVAL;
  if (ctx->uop && !in_callback_ok) {
    ctx->err = "only lj_rhs and lj_jv may be called on a context from its own user-operator callbacks";
    return LJ_EINVAL;
  }
  try {
    ctx->err.clear();
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != ctx->device) HIPCHK(ctx, hipSetDevice(ctx->device));
    return f();
  } catch (const Fail& e) {
    return e.code;
  } catch (...) {
    ctx->err = "unexpected internal error";
    return LJ_EHIP;
  }
}

// ---- batching form -----------------------------------------------------------
// Schedules the tuner chooses among: threads per block, blocks per CU, blocks
// per team (one instance at a time per team) and the order in which teams
// take instances from the queue (largest first, or as given).
struct BatchSchedule {
  int block;
  int per_cu;
  int team;  // blocks (of one XCD) per instance
  int largest_first;
};
constexpr BatchSchedule kBatchSchedules[] = {
    {1024, 1, 1, 1}, {1024, 1, 2, 1}, {1024, 1, 4, 1}, {1024, 1, 8, 1},
    {512, 1, 1, 1},  {512, 1, 4, 1},  {512, 1, 8, 1},  {512, 1, 16, 1},
};
constexpr int kNumBatchSchedules = (int)(sizeof(kBatchSchedules) / sizeof(kBatchSchedules[0]));

}  // namespace

struct lj_batch {
  lj_context* ctx = nullptr;
  int n = 0, K = 0, kind = 0;
  int l[kMaxK] = {};
  double a[kMaxK] = {};
  double tol = 0.0;
  Opts o{};
  std::vector<OpDev> ops;
  std::vector<const double*> v;
  std::vector<double> h;
  std::vector<double*> w;  // n * K
  std::vector<long long> nval;
  long long total_values = 0;
  BatchItem* d_items = nullptr;
  BatchStatus* d_status = nullptr;
  BatchStatus* h_status = nullptr;  // pinned
  int* d_order = nullptr;
  unsigned int* d_queue = nullptr;  // queue counter, then the team words (zeroed per launch)
  double* d_team_part = nullptr;
  int max_blocks = 0;
  double* d_work = nullptr;
  double* d_sub = nullptr;  // substep vectors of every instance
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  BatchParams P{};
  int schedule = 0;
  float tune_ms[kNumBatchSchedules] = {};
  double alg_bytes = 0.0;
};

namespace {

void batch_release(lj_batch* b) {
  if (!b) return;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cs) (void)hipStreamDestroy(b->cs);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_status) (void)hipFree(b->d_status);
  if (b->h_status) (void)hipHostFree(b->h_status);
  if (b->d_order) (void)hipFree(b->d_order);
  if (b->d_queue) (void)hipFree(b->d_queue);
  if (b->d_team_part) (void)hipFree(b->d_team_part);
  if (b->d_work) (void)hipFree(b->d_work);
  if (b->d_sub) (void)hipFree(b->d_sub);
  delete b;
}

// order of the schedule: instance indices, largest first or as given
std::vector<int> batch_order(const lj_batch* b, int largest_first) {
  std::vector<int> ord(b->n);
  std::iota(ord.begin(), ord.end(), 0);
  if (largest_first)
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return b->nval[x] > b->nval[y]; });
  return ord;
}

void batch_launch(lj_batch* b, int sched, hipStream_t s) {
  lj_context* ctx = b->ctx;
  const BatchSchedule& S = kBatchSchedules[sched];
  void* fn = batch_kernel_ptr(b->kind, S.block);
  if (!fn) invalid(ctx, "no batch kernel for this operator family / block size");
  const int G = ctx->num_cus * S.per_cu;
  const int teams = G / S.team;
  HIPCHK(ctx, launch_fill_u32(b->d_queue, kTeamWords + teams * kTeamWords, 0u, s));
  BatchParams P = b->P;
  P.team = S.team;
  P.team_words = b->d_queue + kTeamWords;
  P.team_part = b->d_team_part;
  void* args[] = {&P};
  HIPCHK(ctx, hipLaunchKernel(fn, dim3(G), dim3(S.block), args, 0, s));
}

void batch_set_order(lj_batch* b, int sched) {
  const std::vector<int> ord = batch_order(b, kBatchSchedules[sched].largest_first);
  HIPCHK(b->ctx, hipMemcpy(b->d_order, ord.data(), ord.size() * sizeof(int), hipMemcpyHostToDevice));
}

// A team's blocks must share blockIdx % 8 (one XCD), so 8 * team | blocks,
// and all blocks of the launch must be co-resident (team members wait for
// each other): per_cu blocks of this kernel must fit on one CU.
bool batch_schedule_fits(const lj_batch* b, int i) {
  const BatchSchedule& S = kBatchSchedules[i];
  const int G = b->ctx->num_cus * S.per_cu;
  if (G % (8 * S.team) != 0 || G > b->max_blocks) return false;
  void* fn = batch_kernel_ptr(b->kind, S.block);
  int per_cu = 0;
  if (!fn || hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(fn), S.block, 0) !=
                 hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return per_cu >= S.per_cu;
}

std::string batch_key(const lj_batch* b) {
  std::string k = std::to_string(b->kind) + ":" + std::to_string(b->n) + ":" + std::to_string(b->K) + ":" +
                  std::to_string(b->total_values);
  for (int q = 0; q < b->K; ++q) k += ":" + std::to_string(b->l[q]);
  return k;
}

// Times every schedule on the batch itself (each twice, the faster counts) and
// keeps the fastest; the choice is cached in the context per batch shape.
int batch_tune(lj_batch* b) {
  lj_context* ctx = b->ctx;
  if (const char* e = std::getenv("LJ_BATCH_SCHEDULE")) {
    const int i = std::atoi(e);
    if (i >= 0 && i < kNumBatchSchedules && batch_schedule_fits(b, i)) return i;
  }
  const std::string key = batch_key(b);
  auto it = ctx->batch_schedule.find(key);
  if (it != ctx->batch_schedule.end()) return it->second;
  hipEvent_t e0, e1;
  HIPCHK(ctx, hipEventCreate(&e0));
  HIPCHK(ctx, hipEventCreate(&e1));
  int best = -1;
  for (int i = 0; i < kNumBatchSchedules; ++i) {
    if (!batch_schedule_fits(b, i)) continue;
    batch_set_order(b, i);
    float t = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      HIPCHK(ctx, hipEventRecord(e0, b->cs));
      batch_launch(b, i, b->cs);
      HIPCHK(ctx, hipEventRecord(e1, b->cs));
      HIPCHK(ctx, hipEventSynchronize(e1));
      float ms = 0.0f;
      HIPCHK(ctx, hipEventElapsedTime(&ms, e0, e1));
      unsigned int qw[2] = {0, 0};
      HIPCHK(ctx, hipMemcpy(qw, b->d_queue, sizeof(qw), hipMemcpyDeviceToHost));
      if (qw[1] != 0u) ms = 1e30f;  // aborted: a team never assembled
      t = std::min(t, ms);
    }
    if (t >= 1e30f) {
      b->tune_ms[i] = 0.0f;
      continue;
    }
    b->tune_ms[i] = t;
    if (best < 0 || t < b->tune_ms[best]) best = i;
  }
  if (best < 0) invalid(ctx, "no batch schedule fits this device");
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ctx->batch_schedule[key] = best;
  return best;
}

// ---- Krylov evaluation of phi combinations (Sec. 2.1) ------------------------------
struct KryOpts {
  int m = 30;
  int window = 2;
  int max_substeps = 1000;
};

KryOpts resolve_krylov(lj_context* ctx, const lj_krylov_options* k) {
  KryOpts r;
  if (!k) return r;
  r.m = k->krylov_dim;
  r.window = k->window;
  r.max_substeps = k->max_substeps;
  if (r.m < 1 || r.m > kKryMaxDim) invalid(ctx, "krylov options: krylov_dim must be in [1, 64]");
  if (r.window < 0) invalid(ctx, "krylov options: window must be >= 0");
  if (r.max_substeps < 1) invalid(ctx, "krylov options: max_substeps must be >= 1");
  return r;
}

// w = sum_{j=0}^{p} phi_j(h J) b_j h^j (b[j] may be nullptr) as the first block
// of exp(h A~) [b_0; e_p], A~ = [[J, B], [0, K]] (Sec. 2.1 theorem), advanced
// in substeps: each projects exp(tau A~) onto an m-dimensional Krylov space
// (Arnoldi with an orthogonalisation window), accepts when the a-posteriori
// estimate beta h_{m+1,m} tau |e_m^T phi_1(tau H_m) e_1| is at most
// tol (tau / h) beta, and sizes the next substep from it; a rejected substep
// reuses the basis with a smaller tau.
int krylov_impl(lj_context* ctx, const OpDev& op, int p, const double* const* b, double h, double tol,
                double* w_out, const KryOpts& ko, lj_stats* st, hipStream_t s) {
  const long N = (long)nvals(op);
  const long na = N + p;
  const int m = ko.m;
  if (!ctx->d_kpart)
    HIPCHK(ctx, hipMalloc(&ctx->d_kpart, (size_t)kKryBlocksMax * (kKryMaxDim + 1) * sizeof(double)));
  const size_t hsz = (size_t)(kKryMaxDim + 1) * kKryMaxDim + 3;  // H, then scalars [beta, breakdown, aborted]
  if (!ctx->d_kH) HIPCHK(ctx, hipMalloc(&ctx->d_kH, hsz * sizeof(double)));
  if (!ctx->h_kH) HIPCHK(ctx, hipHostMalloc(&ctx->h_kH, hsz * sizeof(double), hipHostMallocDefault));
  KryDev K;
  std::memset(&K, 0, sizeof(K));
  K.N = N;
  K.p = p;
  K.na = na;
  K.V = slot(ctx, W_KV, (size_t)(m + 1) * na);
  K.W = slot(ctx, W_KW, na);
  for (int k = 0; k < p; ++k) K.B[k] = b[p - k];  // [b_p, ..., b_1]
  K.H = ctx->d_kH;
  K.m = m;
  K.part = ctx->d_kpart;
  K.scalars = ctx->d_kH + (size_t)(kKryMaxDim + 1) * kKryMaxDim;
  double* X = slot(ctx, W_KX, na);
  HIPCHK(ctx, launch_kry_init(X, b[0], N, p, s));
  // built-in families with a window of 1 or 2 vectors: the whole basis in
  // one persistent launch; otherwise four launches per column
  const bool persistent = !is_user(op) && ko.window >= 1 && ko.window <= 2 && !ctx->krylov_passes;
  KryArnoldi KA;
  std::memset(&KA, 0, sizeof(KA));
  const void* kfn = nullptr;
  int KG = 0;
  if (persistent) {
    KA.K = K;
    KA.op = op;
    KA.w = X;
    KA.U[0] = slot(ctx, W_KU0, na);
    KA.U[1] = slot(ctx, W_KU1, na);
    KA.Z[0] = slot(ctx, W_KZ0, na);
    KA.Z[1] = slot(ctx, W_KZ1, na);
    KA.window = ko.window;
    KG = grid_for(ctx, op.npts);
    ensure_small(ctx, KG);
    KA.partials = ctx->d_partials;
    KA.barrier = ctx->d_barrier;
    kfn = kry_arnoldi_ptr(op.kind);
    if (!kfn) invalid(ctx, "operator kind has no Krylov kernel");
  }
  // one basis from X; returns false when beta = 0
  auto basis = [&]() -> bool {
    if (persistent) {
      for (int attempt = 0; attempt < 2; ++attempt) {
        const bool coop = attempt > 0 || !coresident(ctx, kfn, KG, 0, persistent_block());
        KA.spin_limit = (!coop && ctx->forced_spin_limit > 0) ? ctx->forced_spin_limit : kGridSpinLimit;
        void* args[] = {&KA};
        if (coop) {
          HIPCHK(ctx, hipLaunchCooperativeKernel(kfn, dim3(KG), dim3(kKryPBlock), args, 0, s));
        } else {
          HIPCHK(ctx, hipLaunchKernel(kfn, dim3(KG), dim3(kKryPBlock), args, 0, s));
        }
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_kH, ctx->d_kH, hsz * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(ctx, hipStreamSynchronize(s));
        if (ctx->h_kH[hsz - 1] == 0.0) return ctx->h_kH[hsz - 3] > 0.0;
        ctx->tm.aborts += 1;
      }
      ctx->err = "a Krylov basis launch aborted twice (grid barrier timed out)";
      throw Fail{LJ_EHIP};
    }
    HIPCHK(ctx, launch_kry_start(K, X, s));
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_kH + hsz - 3, K.scalars, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (!(ctx->h_kH[hsz - 3] > 0.0)) return false;  // w = 0 stays 0
    for (int j = 0; j < m; ++j) {
      const double* vj = K.V + (size_t)j * na;
      if (is_user(op)) {
        user_jv(ctx, vj, K.W, s);
      } else {
        HIPCHK(ctx, launch_family_jv(op, vj, K.W, s));
      }
      const int lo = ko.window > 0 ? std::max(0, j - ko.window + 1) : 0;
      const int ndt = j - lo + 1;
      for (int d0 = 0; d0 < ndt; d0 += kKryChunk)
        HIPCHK(ctx, launch_kry_tail_dots(K, j, lo, d0, std::min(kKryChunk, ndt - d0), d0 == 0, s));
      HIPCHK(ctx, launch_kry_update(K, j, lo, ndt, s));
      HIPCHK(ctx, launch_kry_scale(K, j, s));
    }
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_kH, ctx->d_kH, (hsz - 1) * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return true;
  };
  std::memset(st, 0, sizeof(*st));
  for (int k = 0; k < LJ_MAX_K; ++k) {
    st->m_star[k] = -1;
    st->substeps[k] = 1;
  }
  bool converged = true;
  int substeps = 0, rejections = 0, products = 0, attempts = 0;
  double t = 0.0, tau = h, last_est = 0.0;
  std::vector<double> Hm, Mx, E;
  while (t < h) {
    if (substeps >= ko.max_substeps || attempts >= 10 * ko.max_substeps) {
      converged = false;
      break;
    }
    if (!basis()) break;  // w = 0 stays 0
    const double beta = ctx->h_kH[hsz - 3];
    const int brk = (int)ctx->h_kH[hsz - 2];  // breakdown at column brk - 1
    const int me = brk > 0 ? brk : m;
    products += me;
    const bool exact = me < m;
    // H_m with only the entries this basis wrote (the window and the subdiagonal)
    Hm.assign((size_t)(me + 1) * me, 0.0);
    for (int c = 0; c < me; ++c) {
      const int lo = ko.window > 0 ? std::max(0, c - ko.window + 1) : 0;
      for (int r = lo; r <= c + 1 && r <= me; ++r) Hm[(size_t)r * me + c] = ctx->h_kH[(size_t)r * m + c];
    }
    while (true) {
      ++attempts;
      tau = std::min(tau, h - t);
      const int n1 = me + 1;
      Mx.assign((size_t)n1 * n1, 0.0);
      for (int r = 0; r < me; ++r)
        for (int c = 0; c < me; ++c) Mx[(size_t)r * n1 + c] = tau * Hm[(size_t)r * me + c];
      Mx[me] = 1.0;  // row 0, column me: e_1
      expm_small(Mx, n1, E);
      const double est = exact ? 0.0 : beta * Hm[(size_t)me * me + (me - 1)] * tau * std::fabs(E[(size_t)(me - 1) * n1 + me]);
      const double allow = tol * (tau / h) * beta;
      const double fac = (est == 0.0) ? 2.0
                                      : std::min(2.0, std::max(0.1, 0.9 * std::pow(allow / est, 1.0 / (me + 1))));
      if (est <= allow) {
        KryCoef F;
        std::memset(&F, 0, sizeof(F));
        for (int c = 0; c < me; ++c) F.f[c] = E[(size_t)c * n1];
        HIPCHK(ctx, launch_kry_combine(K, me, beta, F, X, s));
        t = (tau >= h - t) ? h : t + tau;
        ++substeps;
        last_est = est;
        tau *= fac;
        break;
      }
      ++rejections;
      tau *= fac;
      if (attempts >= 10 * ko.max_substeps) {
        converged = false;
        break;
      }
    }
    if (!converged) break;
  }
  HIPCHK(ctx, hipMemcpyAsync(w_out, X, (size_t)N * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  st->m_star[0] = products;
  st->substeps[0] = substeps;
  st->iters_total = products;
  st->rejections = rejections;
  st->converged = converged ? 1 : 0;
  st->err_est[0] = last_est;
  return converged ? LJ_OK : LJ_ENOTCONV;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

LJ_API const char* lj_version(void) { return "leja-mi355x 0.1 (gfx950)"; }

LJ_API void lj_default_options(lj_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->safety = 1.25;
  opt->power_iters = 20;
  opt->max_points = 100;
  opt->hump_max = 1e4;
  opt->max_substeps = 64;
  opt->relative_tol = 1;
  opt->bound = 0.0;
  opt->substeps = 0;
  opt->power_seed = 0x5EED;
  opt->pi_start = nullptr;
  opt->bound_device = nullptr;
}

LJ_API const char* lj_last_error(const lj_context* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

LJ_API int lj_leja_points(double* out, int count) {
  if (!out || count < 1 || count > kTable) return LJ_EINVAL;
  return leja_points_host(out, count);
}

LJ_API int lj_create(lj_context** out, int hip_device) {
  if (!out) return LJ_EINVAL;
  *out = nullptr;
  g_create_error.clear();
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev < 1) {
    g_create_error = std::string("no HIP device: ") + hipGetErrorString(e);
    return LJ_EHIP;
  }
  if (hip_device < 0 || hip_device >= ndev) {
    g_create_error = "device index out of range";
    return LJ_EINVAL;
  }
  lj_context* ctx = new lj_context();
  ctx->device = hip_device;
  try {
    HIPCHK(ctx, hipSetDevice(hip_device));
    hipDeviceProp_t prop;
    HIPCHK(ctx, hipGetDeviceProperties(&prop, hip_device));
    ctx->num_cus = prop.multiProcessorCount;
    ctx->lds_max = (int)prop.sharedMemPerBlock;
    int coop = 0;
    HIPCHK(ctx, hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, hip_device));
    if (!coop) {
      ctx->err = "device does not support cooperative launches";
      throw Fail{LJ_EHIP};
    }
    double xi[kTable];
    leja_points_host(xi, kTable);
    HIPCHK(ctx, hipMalloc(&ctx->d_xi, kTable * sizeof(double)));
    HIPCHK(ctx, hipMemcpy(ctx->d_xi, xi, kTable * sizeof(double), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMalloc(&ctx->d_coef, kMaxK * kTable * sizeof(double)));
    HIPCHK(ctx, hipMalloc(&ctx->d_fmax, kMaxK * sizeof(double)));
    HIPCHK(ctx, hipMalloc(&ctx->d_barrier, kBarrierWords * sizeof(unsigned int)));
    HIPCHK(ctx, hipMemset(ctx->d_barrier, 0, kBarrierWords * sizeof(unsigned int)));
    HIPCHK(ctx, hipMalloc(&ctx->d_status, sizeof(LejaStatus)));
    // fine-grained: the action kernels write their status head here directly
    HIPCHK(ctx, hipHostMalloc(&ctx->h_status, sizeof(LejaStatus), hipHostMallocCoherent));
    HIPCHK(ctx, hipHostMalloc(&ctx->h_coef, kMaxK * kTable * sizeof(double), hipHostMallocDefault));
    // fine-grained: the action kernels write their status headers here directly
    HIPCHK(ctx, hipHostMalloc(&ctx->h_pool, kPoolSlots * sizeof(LejaStatus), hipHostMallocCoherent));
    HIPCHK(ctx, hipMalloc(&ctx->d_bound, sizeof(double)));
    HIPCHK(ctx, hipMalloc(&ctx->d_sumsq, (2 * kSumsqBlocks + 2) * sizeof(double)));
    HIPCHK(ctx, hipHostMalloc(&ctx->h_sumsq, 2 * sizeof(double), hipHostMallocDefault));
    if (hip_device < kScratchDevices) {  // once per device, with the device current
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      if (!g_scratch_addr[hip_device]) {
        void* addr = nullptr;
        HIPCHK(ctx, hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
        if (!addr) {
          ctx->err = "hipGetSymbolAddress(scratch) returned no address";
          throw Fail{LJ_EHIP};
        }
        g_scratch_addr[hip_device] = static_cast<double*>(addr);
      }
      ctx->scratch = g_scratch_addr[hip_device];
    }
    if (const char* g = std::getenv("LJ_GRID")) ctx->grid_override = std::atoi(g);
    if (const char* g = std::getenv("LJ_NO_TILE")) ctx->force_stream = std::atoi(g);
    if (const char* g = std::getenv("LJ_NO_REG")) ctx->no_reg = std::atoi(g);
    if (const char* g = std::getenv("LJ_COOP")) ctx->force_coop = std::atoi(g);
    if (const char* g = std::getenv("LJ_KRYLOV_PASSES")) ctx->krylov_passes = std::atoi(g);
    if (const char* g = std::getenv("LJ_FORCE_SPIN_LIMIT")) {
      const long v = std::atol(g);
      ctx->forced_spin_limit = v > 0 ? (unsigned int)std::min<long>(v, kGridSpinLimit) : 0u;
    }
    if (const char* g = std::getenv("LJ_TILE")) {
      int tx = 0, ty = 0;
      if (std::sscanf(g, "%d,%d", &tx, &ty) == 2 && tx > 0 && ty > 0) {
        ctx->tile_override_x = tx;
        ctx->tile_override_y = ty;
      }
    }
  } catch (const Fail& f) {
    g_create_error = ctx->err;
    lj_destroy(ctx);
    return f.code;
  }
  *out = ctx;
  return LJ_OK;
}

LJ_API void lj_destroy(lj_context* ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  for (int i = 0; i < W_NSLOTS; ++i)
    if (ctx->vec[i]) (void)hipFree(ctx->vec[i]);
  if (ctx->d_xi) (void)hipFree(ctx->d_xi);
  if (ctx->d_coef) (void)hipFree(ctx->d_coef);
  if (ctx->d_fmax) (void)hipFree(ctx->d_fmax);
  if (ctx->d_partials) (void)hipFree(ctx->d_partials);
  if (ctx->d_barrier) (void)hipFree(ctx->d_barrier);
  if (ctx->d_status) (void)hipFree(ctx->d_status);
  if (ctx->d_model) (void)hipFree(ctx->d_model);
  if (ctx->d_adam) (void)hipFree(ctx->d_adam);
  if (ctx->d_adam_t) (void)hipFree(ctx->d_adam_t);
  if (ctx->d_rows) (void)hipFree(ctx->d_rows);
  if (ctx->d_scalars) (void)hipFree(ctx->d_scalars);
  if (ctx->d_featpart) (void)hipFree(ctx->d_featpart);
  if (ctx->d_feats) (void)hipFree(ctx->d_feats);
  if (ctx->d_pred) (void)hipFree(ctx->d_pred);
  if (ctx->d_gers) (void)hipFree(ctx->d_gers);
  if (ctx->d_prop) (void)hipFree(ctx->d_prop);
  if (ctx->h_status) (void)hipHostFree(ctx->h_status);
  if (ctx->h_coef) (void)hipHostFree(ctx->h_coef);
  for (hipEvent_t e : ctx->tev)
    if (e) (void)hipEventDestroy(e);
  if (ctx->h_pool) (void)hipHostFree(ctx->h_pool);
  if (ctx->d_bound) (void)hipFree(ctx->d_bound);
  if (ctx->d_sumsq) (void)hipFree(ctx->d_sumsq);
  if (ctx->h_sumsq) (void)hipHostFree(ctx->h_sumsq);
  if (ctx->d_ustate) (void)hipFree(ctx->d_ustate);
  if (ctx->h_ustatus) (void)hipHostFree(ctx->h_ustatus);
  if (ctx->d_upart) (void)hipFree(ctx->d_upart);
  if (ctx->d_kpart) (void)hipFree(ctx->d_kpart);
  if (ctx->d_kH) (void)hipFree(ctx->d_kH);
  if (ctx->h_kH) (void)hipHostFree(ctx->h_kH);
  delete ctx->defer;
  delete ctx;
}

LJ_API int lj_spectral_bound(lj_context* ctx, const lj_operator* J, int iters, uint64_t seed, const double* start,
                             double* bound, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    if (!bound) invalid(ctx, "bound is NULL");
    if (iters < 1 || iters > 100000) invalid(ctx, "iters out of range");
    if (start) check_vec(ctx, op, start, "start");
    const Opts o = resolve(ctx, nullptr);
    *bound = run_bound(ctx, op, o, iters, seed, start, reinterpret_cast<hipStream_t>(stream));
    return LJ_OK;
  });
}

LJ_API int lj_divided_differences(lj_context* ctx, int l, double s_, double c, double gamma, int npts, double* d,
                                  void* stream) {
  return guarded(ctx, [&]() {
    if (!d) invalid(ctx, "d is NULL");
    if (l < 0 || l > LJ_MAX_L) invalid(ctx, "l must be in [0, 4]");
    if (npts < 1 || npts > kTable) invalid(ctx, "npts must be in [1, 101]");
    if (!std::isfinite(s_) || !std::isfinite(c) || !std::isfinite(gamma)) invalid(ctx, "non-finite argument");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    DDParams D;
    std::memset(&D, 0, sizeof(D));
    D.K = 1;
    D.l[0] = l;
    D.s[0] = s_;
    D.npts = npts;
    D.c = c;
    D.gamma = gamma;
    D.xi = ctx->d_xi;
    D.coef = ctx->d_coef;
    D.fmax = ctx->d_fmax;
    HIPCHK(ctx, launch_divdiff(D, s));
    HIPCHK(ctx, hipMemcpyAsync(ctx->h_coef, ctx->d_coef, npts * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    std::memcpy(d, ctx->h_coef, npts * sizeof(double));
    return LJ_OK;
  });
}

LJ_API int lj_rhs(lj_context* ctx, const lj_operator* J, const double* u, double* f, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    check_vec(ctx, op, u, "u");
    check_vec(ctx, op, f, "f");
    if (f == u) invalid(ctx, "f must not alias u");
    HIPCHK(ctx, launch_rhs(op, u, f, reinterpret_cast<hipStream_t>(stream)));
    return LJ_OK;
  }, true);
}

LJ_API int lj_jv(lj_context* ctx, const lj_operator* J, const double* x, double* y, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    check_vec(ctx, op, x, "x");
    check_vec(ctx, op, y, "y");
    if (y == x) invalid(ctx, "y must not alias x");
    if (y == op.state) invalid(ctx, "y must not alias the operator state");
    HIPCHK(ctx, launch_family_jv(op, x, y, reinterpret_cast<hipStream_t>(stream)));
    return LJ_OK;
  }, true);
}

LJ_API int lj_user_phi_vertical(lj_context* ctx, const lj_user_operator* J, const double* v, int K, const int* l,
                                const double* a, double h, double tol, double* const* w, const lj_options* opt,
                                lj_stats* stats, void* stream) {
  return guarded(ctx, [&]() {
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Opts o = resolve(ctx, opt);
    if (o.use_proposal) invalid(ctx, "the learned proposal needs a built-in operator family");
    UserScope us(ctx, J, false, s);
    check_action_args(ctx, us.op, v, K, l, a, h, tol, w);
    if (o.pi_start) check_vec(ctx, us.op, o.pi_start, "pi_start");
    lj_stats local;
    return vertical_impl(ctx, us.op, v, K, l, a, h, tol, w, o, stats ? stats : &local, s);
  });
}

LJ_API int lj_user_phi_action(lj_context* ctx, const lj_user_operator* J, const double* v, double* w, int l,
                              double h, double tol, const lj_options* opt, lj_stats* stats, void* stream) {
  const double a = 1.0;
  double* ws[1] = {w};
  return lj_user_phi_vertical(ctx, J, v, 1, &l, &a, h, tol, ws, opt, stats, stream);
}

LJ_API void lj_default_krylov_options(lj_krylov_options* k) {
  if (!k) return;
  const KryOpts d;
  k->krylov_dim = d.m;
  k->window = d.window;
  k->max_substeps = d.max_substeps;
  k->reserved = 0;
}

int combination_impl(lj_context* ctx, const OpDev& op, int p, const double* const* b, double h, double tol,
                     double* w, const lj_krylov_options* kopt, lj_stats* stats, hipStream_t s) {
  const KryOpts ko = resolve_krylov(ctx, kopt);
  if (p < 0 || p > kKryMaxP) invalid(ctx, "p must be in [0, 4]");
  if (!b) invalid(ctx, "b must not be NULL");
  if (!(h >= 0.0) || !std::isfinite(h)) invalid(ctx, "h must be finite and >= 0");
  if (!(tol > 0.0) || !std::isfinite(tol)) invalid(ctx, "tol must be finite and > 0");
  check_vec(ctx, op, w, "w");
  for (int j = 0; j <= p; ++j) {
    if (!b[j]) continue;
    check_vec(ctx, op, b[j], "b[j]");
    if (b[j] == w) invalid(ctx, "w must not alias b[j]");
  }
  if (w == op.state) invalid(ctx, "w must not alias the operator state");
  lj_stats local;
  return krylov_impl(ctx, op, p, b, h, tol, w, ko, stats ? stats : &local, s);
}

LJ_API int lj_phi_combination(lj_context* ctx, const lj_operator* J, int p, const double* const* b, double h,
                              double tol, double* w, const lj_krylov_options* kopt, lj_stats* stats, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    return combination_impl(ctx, op, p, b, h, tol, w, kopt, stats, reinterpret_cast<hipStream_t>(stream));
  });
}

LJ_API int lj_user_phi_combination(lj_context* ctx, const lj_user_operator* J, int p, const double* const* b,
                                   double h, double tol, double* w, const lj_krylov_options* kopt, lj_stats* stats,
                                   void* stream) {
  return guarded(ctx, [&]() {
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    UserScope us(ctx, J, false, s);
    return combination_impl(ctx, us.op, p, b, h, tol, w, kopt, stats, s);
  });
}

LJ_API int lj_phi_vertical(lj_context* ctx, const lj_operator* J, const double* v, int K, const int* l,
                           const double* a, double h, double tol, double* const* w, const lj_options* opt,
                           lj_stats* stats, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    const Opts o = resolve(ctx, opt);
    check_action_args(ctx, op, v, K, l, a, h, tol, w);
    if (o.pi_start) check_vec(ctx, op, o.pi_start, "pi_start");
    lj_stats local;
    lj_stats* st = stats ? stats : &local;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (!o.use_proposal) return vertical_impl(ctx, op, v, K, l, a, h, tol, w, o, st, s);
    // learned proposal: one attempt with the bound and substeps that the
    // device decides (propose); the attempt's launch reads both, so the host
    // waits only for the launch's status, as on the plain path ...
    propose(ctx, op, K, l, a, h, o.max_substeps, s);
    Opts o1 = o;
    o1.bound = 0.0;
    o1.bound_device = &ctx->d_prop->bound;
    o1.skip_src = &ctx->d_prop->sub;
    o1.substeps = 0;
    o1.max_substeps = 1;
    const int rc = vertical_impl(ctx, op, v, K, l, a, h, tol, w, o1, st, s);
    if (rc == LJ_OK) return LJ_OK;
    // ... and the plain path for every accumulator it did not converge
    std::vector<int> pk, pl;
    std::vector<double> pa;
    std::vector<double*> pw;
    for (int k = 0; k < K; ++k) {
      if (st->m_star[k] >= 0) continue;
      pk.push_back(k);
      pl.push_back(l[k]);
      pa.push_back(a[k]);
      pw.push_back(w[k]);
    }
    lj_stats fb;
    const int rc2 = vertical_impl(ctx, op, v, (int)pk.size(), pl.data(), pa.data(), h, tol, pw.data(), o, &fb, s);
    st->fallbacks = 1;
    st->rejections += fb.rejections;  // the proposal's failed attempt is already counted
    st->iters_total += fb.iters_total;
    st->power_iters += fb.power_iters;
    st->bound = fb.bound;
    st->c = fb.c;
    st->gamma = fb.gamma;
    for (size_t q = 0; q < pk.size(); ++q) {
      st->m_star[pk[q]] = fb.m_star[q];
      st->substeps[pk[q]] = fb.substeps[q];
      st->err_est[pk[q]] = fb.err_est[q];
    }
    st->converged = fb.converged;
    return rc2;
  });
}

int step_impl(lj_context* ctx, int scheme, const OpDev& op, Opts o, double h, double tol, double* u_out, double* err,
              lj_stats* stats, hipStream_t s);
bool collect_async(lj_context* ctx, const OpDev& op, const std::vector<PendingLaunch>& pend,
                   std::vector<lj_stats>& log, double& lam_found, int& pit);

LJ_API int lj_phi_action(lj_context* ctx, const lj_operator* J, const double* v, double* w, int l, double h,
                         double tol, const lj_options* opt, lj_stats* stats, void* stream) {
  const double a = 1.0;
  double* ws[1] = {w};
  if (ctx && ctx->deferring) {
    return guarded(ctx, [&]() {
      const OpDev op = make_op(ctx, J);
      const Opts o = resolve(ctx, opt);
      check_action_args(ctx, op, v, 1, &l, &a, h, tol, ws);
      if (o.pi_start) check_vec(ctx, op, o.pi_start, "pi_start");
      if (o.use_proposal || o.substeps > 1)
        invalid(ctx, "an action with substeps or the learned proposal cannot be deferred: call lj_defer_end first");
      const int slot = ctx->defer_next;
      if (slot + 1 > kPoolSlots) invalid(ctx, "too many deferred launches: call lj_defer_end");
      if (ctx->timing && ctx->tev_next + 1 > kTimingPairs) timing_flush(ctx);
      const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
      BoundLink link;
      if (!(o.bound > 0.0) && o.bound_device) link.src = o.bound_device;
      const double sk = h;
      bool tiled = false;
      hipEvent_t* ev = timing_pair(ctx);
      launch_action(ctx, op, v, 1, &l, &sk, o.bound > 0.0 ? o.bound : 0.0, o.seed, o.pi_start, ws, o, tol, s, link,
                    &ctx->h_pool[slot], offsetof(LejaStatus, trace), ev, &tiled, false, true);
      DeferredCall dc;
      dc.op = op;
      dc.o = o;
      dc.h = h;
      dc.tol = tol;
      dc.v = v;
      dc.w = w;
      dc.l = l;
      dc.stats = stats;
      dc.launches.push_back({slot, 1, tiled, ev});
      ctx->defer->calls.push_back(dc);
      ctx->defer_next = slot + 1;
      return LJ_OK;
    });
  }
  return lj_phi_vertical(ctx, J, v, 1, &l, &a, h, tol, ws, opt, stats, stream);
}

LJ_API int lj_defer_begin(lj_context* ctx) {
  return guarded(ctx, [&]() {
    if (ctx->deferring) invalid(ctx, "lj_defer_begin: a deferral is already open");
    if (!ctx->defer) ctx->defer = new DeferState();
    ctx->defer->calls.clear();
    ctx->defer_next = 0;
    ctx->deferring = true;
    return LJ_OK;
  });
}

LJ_API int lj_defer_end(lj_context* ctx, void* stream) {
  return guarded(ctx, [&]() {
    if (!ctx->deferring) invalid(ctx, "lj_defer_end: no deferral is open");
    ctx->deferring = false;
    std::vector<DeferredCall> calls;
    calls.swap(ctx->defer->calls);
    ctx->defer_next = 0;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(ctx, hipStreamSynchronize(s));
    bool ok = true;
    bool redo = false;  // from the first failed call on, every call is redone in order
    for (DeferredCall& dc : calls) {
      if (!redo) {
        std::vector<lj_stats> log;
        double lam_found = dc.o.bound;
        int pit = 0;
        if (collect_async(ctx, dc.op, dc.launches, log, lam_found, pit)) {
          if (dc.stats)
            for (size_t i = 0; i < log.size(); ++i) dc.stats[i] = log[i];
          continue;
        }
        redo = true;
      }
      int rc;
      if (dc.is_step) {
        rc = step_impl(ctx, dc.scheme, dc.op, dc.o, dc.h, dc.tol, dc.u_out, dc.err, dc.stats, s);
      } else {
        lj_stats local;
        const double a = 1.0;
        double* ws[1] = {dc.w};
        rc = vertical_impl(ctx, dc.op, dc.v, 1, &dc.l, &a, dc.h, dc.tol, ws, dc.o, dc.stats ? dc.stats : &local, s);
      }
      if (rc != LJ_OK) ok = false;
    }
    return ok ? LJ_OK : LJ_ENOTCONV;
  });
}

LJ_API const double* lj_bound_device(const lj_context* ctx) { return ctx ? ctx->d_bound : nullptr; }

// Doubles of scratch an allocation-free phi_l action on n values needs at
// most: the two Newton-basis vectors, the partial sums of the largest grid,
// and, when substeps may be taken, phi_1..phi_l at the substep plus three
// propagation vectors (l = 0: two).
size_t noalloc_need(const lj_context* ctx, size_t n, int l, const Opts& o) {
  auto r = [](size_t x) { return (x + 31) & ~(size_t)31; };
  size_t d = 2 * r(n) + r((size_t)2 * kRegPartStride * ctx->num_cus);
  if (o.max_substeps > 1 || o.substeps > 1) d += (size_t)(l > 0 ? l + 3 : 2) * r(n);
  return d;
}

LJ_API int lj_phi_action_noalloc(lj_context* ctx, const lj_operator* J, const double* v, double* w, int l,
                                 double h, double tol, const lj_options* opt, lj_stats* stats, void* stream) {
  return guarded(ctx, [&]() {
    if (!ctx->scratch) invalid(ctx, "lj_phi_action_noalloc: no scratch array on this device");
    const OpDev op = make_op(ctx, J);
    const Opts o = resolve(ctx, opt);
    if (o.use_proposal) invalid(ctx, "lj_phi_action_noalloc: use_proposal is not supported");
    const double a = 1.0;
    double* ws[1] = {w};
    check_action_args(ctx, op, v, 1, &l, &a, h, tol, ws);
    if (o.pi_start) check_vec(ctx, op, o.pi_start, "pi_start");
    const size_t need = noalloc_need(ctx, nvals(op), l, o) * sizeof(double);
    if (need > kScratchBytes)
      invalid(ctx, "lj_phi_action_noalloc: this action needs " + std::to_string(need) +
                       " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                       " the allocation-free path holds (use lj_phi_action)");
    struct Scope {
      lj_context* c;
      explicit Scope(lj_context* c_) : c(c_) {
        c->in_noalloc = true;
        c->scratch_next = 0;
        for (int i = 0; i <= W_NSLOTS; ++i) c->scratch_len[i] = 0;
      }
      ~Scope() { c->in_noalloc = false; }
    } scope(ctx);
    lj_stats local;
    lj_stats* st = stats ? stats : &local;
    return vertical_impl(ctx, op, v, 1, &l, &a, h, tol, ws, o, st, reinterpret_cast<hipStream_t>(stream));
  });
}

// Statistics of the launches of an asynchronous pass (their status heads in
// the pinned pool): one lj_stats per launch into `log`; lam_found / pit take
// the first launch's bound and power products.  Returns false if an
// expansion was rejected or a launch aborted (the caller redoes the work
// synchronously).
bool collect_async(lj_context* ctx, const OpDev& op, const std::vector<PendingLaunch>& pend,
                   std::vector<lj_stats>& log, double& lam_found, int& pit) {
  bool all = true;
  for (size_t i = 0; i < pend.size(); ++i) {
    const ActOut r = finish_action(ctx, op, ctx->h_pool[pend[i].slot], pend[i].ev, pend[i].tiled);
    if (r.aborted) all = false;
    lj_stats st;
    std::memset(&st, 0, sizeof(st));
    for (int k = 0; k < LJ_MAX_K; ++k) {
      st.m_star[k] = -1;
      st.substeps[k] = 1;
    }
    st.iters_total = r.iters;
    st.power_iters = r.power_iters;
    st.bound = r.lam;
    st.c = r.c;
    st.gamma = r.gamma;
    st.converged = 1;
    for (int k = 0; k < pend[i].K; ++k) {
      if (r.state[k] == ACC_CONVERGED) {
        st.m_star[k] = r.m_star[k];
        st.err_est[k] = r.err[k];
      } else {
        st.converged = 0;
        st.rejections = 1;
        all = false;
      }
    }
    if (i == 0 && !r.aborted) {  // an aborted launch's bound is not to be trusted
      lam_found = r.lam;
      pit = r.power_iters;
    }
    log.push_back(st);
  }
  return all;
}

// One step of `scheme` from u = op.state (arguments validated by the caller):
// u_out, err (nullable) and the stats of the scheme's Leja calls.
int step_impl(lj_context* ctx, int scheme, const OpDev& op, Opts o, double h, double tol, double* u_out, double* err,
              lj_stats* stats, hipStream_t s) {
  const size_t n = nvals(op);
  const double* u = op.state;
  // The scheme's stages; `act` runs one (vertical) Leja call.  Between the
  // Leja calls: f(u) and v = h f(u) in one pass, the remainders and the
  // vectors the next calls act on in one pass, the result and error
  // estimate in one pass.
  // f(u) and h f(u); the stage remainders and combinations (one fused pass
  // for a built-in family, callbacks and linear combinations for a user
  // operator, in the same order of operations)
  auto rhs_scaled = [&](double* fu, double* v) {
    if (!is_user(op)) {
      HIPCHK(ctx, launch_rhs_scaled(op, h, fu, v, s));
      return;
    }
    call_rhs(ctx, u, fu, s);
    const double* x[1] = {fu};
    lincomb(ctx, n, v, 1, &h, x, s);
  };
  auto stage = [&](const StageArgs& S) {
    if (!is_user(op)) {
      HIPCHK(ctx, launch_stage(S, s));
      return;
    }
    double* R[2] = {slot(ctx, W_UR0, n), slot(ctx, W_UR1, n)};
    double* xr = slot(ctx, W_UXR, n);
    double* d = slot(ctx, W_UD, n);
    double* fx = slot(ctx, W_UFX, n);
    double* jd = slot(ctx, W_UJD, n);
    for (int r = 0; r < S.nrem; ++r) {  // R_r = (f(x_r) - f(u)) - J(u)(x_r - u)
      const double ax[3] = {1.0, S.a[r][0], S.a[r][1]};
      const double* xs[3] = {u, S.X[r][0], S.X[r][1]};
      lincomb(ctx, n, xr, 1 + S.nterm[r], ax, xs, s);
      const double ad[2] = {1.0, -1.0};
      const double* ds[2] = {xr, u};
      lincomb(ctx, n, d, 2, ad, ds, s);
      call_rhs(ctx, xr, fx, s);
      user_jv(ctx, d, jd, s);
      const double ar[3] = {1.0, -1.0, -1.0};
      const double* rs[3] = {fx, S.fu, jd};
      lincomb(ctx, n, R[r], 3, ar, rs, s);
    }
    for (int o2 = 0; o2 < S.nout; ++o2) {
      const double* src[2];
      for (int t = 0; t < S.nsrc[o2]; ++t) src[t] = (S.src[o2][t] == 2) ? S.P : R[S.src[o2][t]];
      lincomb(ctx, n, S.out[o2], S.nsrc[o2], S.c[o2], src, s);
    }
  };
  std::vector<lj_stats> log;
  bool ok = true;
  auto krylov_log = [&](const lj_stats& kst, int rc) {
    if (rc != LJ_OK) ok = false;
    log.push_back(kst);
  };
  // EPIRK4s3 (Sec. 5.1 equation) and EPIRK4s3A (Sec. 5.2 equation): the
  // internal-stage coefficients and the R(a), R(b) weights of the phi_3 term
  // of u_3 and of the phi_4 term of u_4 - u_3
  const bool epa = (scheme == LJ_EPIRK4S3A || scheme == LJ_EPIRK4S3A_LEKRY);
  const double g1 = epa ? 0.5 : 1.0 / 8.0, g2 = epa ? 2.0 / 3.0 : 1.0 / 9.0;
  const double d3a = epa ? 32.0 : 1892.0 - 2.0 * 1458.0, d3b = epa ? -13.5 : 1458.0;
  const double d4a = epa ? -144.0 : -42336.0 + 2.0 * 34992.0, d4b = epa ? 81.0 : -34992.0;
  auto scheme_steps = [&](auto&& act) {
    double* fu = slot(ctx, W_FU, n);
    double* v = slot(ctx, W_V, n);
    rhs_scaled(fu, v);
    auto finish = [&](const double* X1, const double* X2, const double* X3) {
      FinishArgs F;
      F.n = (long)n;
      F.u = u;
      F.X1 = X1;
      F.X2 = X2;
      F.X3 = X3;
      F.u_out = u_out;
      F.err = err;
      HIPCHK(ctx, launch_finish(F, s));
    };
    auto stage_args = [&]() {
      StageArgs A;
      std::memset(&A, 0, sizeof(A));
      A.op = op;
      A.fu = fu;
      return A;
    };
    if (scheme == LJ_EXPRB2) {
      double* A = slot(ctx, W_A, n);
      const int ls[1] = {1};
      const double as[1] = {1.0};
      act(v, 1, ls, as, &A);
      finish(A, nullptr, nullptr);
    } else if (scheme == LJ_EXPRB43 || scheme == LJ_EXPRB43_U3) {
      double* A = slot(ctx, W_A, n);
      double* B = slot(ctx, W_B, n);
      double* C = slot(ctx, W_C, n);
      double* Ra = slot(ctx, W_RA, n);
      double* T1 = slot(ctx, W_T1, n);
      double* T3 = slot(ctx, W_T3, n);
      double* T4 = slot(ctx, W_T4, n);
      double* D3 = slot(ctx, W_D3, n);
      {
        const int ls[2] = {1, 1};
        const double as[2] = {0.5, 1.0};
        double* outs[2] = {A, B};
        act(v, 2, ls, as, outs);
      }
      {  // R_a at u + A/2; T1 = h R_a (and R_a kept)
        StageArgs S = stage_args();
        S.nrem = 1;
        S.nterm[0] = 1;
        S.a[0][0] = 0.5;
        S.X[0][0] = A;
        S.nout = 2;
        S.nsrc[0] = 1;
        S.src[0][0] = 0;
        S.c[0][0] = h;
        S.out[0] = T1;
        S.nsrc[1] = 1;
        S.src[1][0] = 0;
        S.c[1][0] = 1.0;
        S.out[1] = Ra;
        stage(S);
      }
      {
        const int ls[1] = {1};
        const double as[1] = {1.0};
        act(T1, 1, ls, as, &C);
      }
      {  // R_b at u + B + C; T3 = 16 h R_a - 2 h R_b (and T4 = -48 h R_a + 12 h R_b)
        StageArgs S = stage_args();
        S.nrem = 1;
        S.nterm[0] = 2;
        S.a[0][0] = 1.0;
        S.X[0][0] = B;
        S.a[0][1] = 1.0;
        S.X[0][1] = C;
        S.P = Ra;
        S.nout = (scheme == LJ_EXPRB43) ? 2 : 1;
        S.nsrc[0] = 2;
        S.src[0][0] = 2;
        S.c[0][0] = 16.0 * h;
        S.src[0][1] = 0;
        S.c[0][1] = -2.0 * h;
        S.out[0] = T3;
        S.nsrc[1] = 2;
        S.src[1][0] = 2;
        S.c[1][0] = -48.0 * h;
        S.src[1][1] = 0;
        S.c[1][1] = 12.0 * h;
        S.out[1] = T4;
        stage(S);
      }
      {
        const int ls[1] = {3};
        const double as[1] = {1.0};
        act(T3, 1, ls, as, &D3);
      }
      if (scheme == LJ_EXPRB43) {
        double* D4 = slot(ctx, W_D4, n);
        const int ls[1] = {4};
        const double as[1] = {1.0};
        act(T4, 1, ls, as, &D4);
        finish(B, D3, D4);
      } else {
        finish(B, D3, nullptr);
      }
    } else if (scheme == LJ_EPIRK4S3_LEKRY || scheme == LJ_EPIRK4S3A_LEKRY) {
      // LeKry (Sec. 5.1 text): internal stages by Leja (vertical), the third
      // stage's phi_1(hJ) h f(u) + phi_3(hJ) D_3 as one augmented exponential
      // by Krylov (b_1 = f(u), b_3 = D_3 / h^3), the phi_4 error term by Leja
      double* A = slot(ctx, W_A, n);
      double* B = slot(ctx, W_B, n);
      double* T3 = slot(ctx, W_T3, n);
      double* T4 = slot(ctx, W_T4, n);
      double* D4 = slot(ctx, W_D4, n);
      double* KC = slot(ctx, W_KC, n);
      {
        const int ls[2] = {1, 1};
        const double as[2] = {g1, g2};
        double* outs[2] = {A, B};
        act(v, 2, ls, as, outs);
      }
      {
        StageArgs S = stage_args();
        S.nrem = 2;
        S.nterm[0] = 1;
        S.a[0][0] = g1;
        S.X[0][0] = A;
        S.nterm[1] = 1;
        S.a[1][0] = g2;
        S.X[1][0] = B;
        S.nout = 2;
        S.nsrc[0] = 2;
        S.src[0][0] = 0;
        S.c[0][0] = h * d3a;
        S.src[0][1] = 1;
        S.c[0][1] = h * d3b;
        S.out[0] = T3;
        S.nsrc[1] = 2;
        S.src[1][0] = 0;
        S.c[1][0] = h * d4a;
        S.src[1][1] = 1;
        S.c[1][1] = h * d4b;
        S.out[1] = T4;
        stage(S);
      }
      {
        double* b3 = slot(ctx, W_C, n);
        const double a3 = 1.0 / (h * h * h);
        const double* x3[1] = {T3};
        lincomb(ctx, n, b3, 1, &a3, x3, s);
        const double* bs[4] = {nullptr, fu, nullptr, b3};
        lj_stats kst;
        const int rc = krylov_impl(ctx, op, 3, bs, h, tol, KC, KryOpts{}, &kst, s);
        krylov_log(kst, rc);
      }
      {
        const int ls[1] = {4};
        const double as[1] = {1.0};
        act(T4, 1, ls, as, &D4);
      }
      finish(KC, nullptr, D4);
    } else {  // EPIRK4s3, EPIRK4s3A
      double* A = slot(ctx, W_A, n);
      double* B = slot(ctx, W_B, n);
      double* C = slot(ctx, W_C, n);
      double* T3 = slot(ctx, W_T3, n);
      double* D3 = slot(ctx, W_D3, n);
      double* T4 = slot(ctx, W_T4, n);
      double* D4 = slot(ctx, W_D4, n);
      {
        const int ls[3] = {1, 1, 1};
        const double as[3] = {g1, g2, 1.0};
        double* outs[3] = {A, B, C};
        act(v, 3, ls, as, outs);
      }
      {  // R_a at u + g1 A, R_b at u + g2 B;
         // h (d3a Ra + d3b Rb) and h (d4a Ra + d4b Rb)
        StageArgs S = stage_args();
        S.nrem = 2;
        S.nterm[0] = 1;
        S.a[0][0] = g1;
        S.X[0][0] = A;
        S.nterm[1] = 1;
        S.a[1][0] = g2;
        S.X[1][0] = B;
        S.nout = 2;
        S.nsrc[0] = 2;
        S.src[0][0] = 0;
        S.c[0][0] = h * d3a;
        S.src[0][1] = 1;
        S.c[0][1] = h * d3b;
        S.out[0] = T3;
        S.nsrc[1] = 2;
        S.src[1][0] = 0;
        S.c[1][0] = h * d4a;
        S.src[1][1] = 1;
        S.c[1][1] = h * d4b;
        S.out[1] = T4;
        stage(S);
      }
      {
        const int ls[1] = {3};
        const double as[1] = {1.0};
        act(T3, 1, ls, as, &D3);
      }
      {
        const int ls[1] = {4};
        const double as[1] = {1.0};
        act(T4, 1, ls, as, &D4);
      }
      finish(C, D3, D4);
    }
  };
  int pit = 0;
  // ---- first try: every launch of the step enqueued back to back.  The
  // first action runs the power iteration (unless a bound is given) and
  // leaves the bound on the device for the others; statuses are read once
  // at the end (or, in a deferral, by lj_defer_end).  If some expansion was
  // rejected, the step is redone below synchronously, with substeps, on the
  // bound found.
  const bool try_async = o.substeps <= 1 && !o.use_proposal && !is_user(op) && scheme != LJ_EPIRK4S3_LEKRY &&
                         scheme != LJ_EPIRK4S3A_LEKRY;
  if (ctx->deferring && !try_async)
    invalid(ctx, "this step cannot be deferred (substeps, the learned proposal, a user operator or LeKry): "
                 "call lj_defer_end first");
  double lam_found = o.bound;
  if (try_async) {
    const int base = ctx->deferring ? ctx->defer_next : 0;
    if (base + kAsyncSlots > kPoolSlots) invalid(ctx, "too many deferred launches: call lj_defer_end");
    // pairs for every launch of the step up front, so a pool flush cannot
    // fall between a launch and its finish
    if (ctx->timing && ctx->tev_next + kAsyncSlots > kTimingPairs) timing_flush(ctx);
    std::vector<PendingLaunch> pend;
    auto act_async = [&](const double* vec, int K, const int* ls, const double* as, double* const* outs) {
      const int i = (int)pend.size();
      if (i >= kAsyncSlots) invalid(ctx, "internal: too many launches in one step");
      double sk[kMaxK];
      for (int k = 0; k < K; ++k) sk[k] = as[k] * h;
      BoundLink link;
      double lam_host = 0.0;
      if (o.bound > 0.0) {
        lam_host = o.bound;
      } else if (o.bound_device) {
        link.src = o.bound_device;
      } else if (i == 0) {
        link.dst = ctx->d_bound;
      } else {
        link.src = ctx->d_bound;
      }
      bool tiled = false;
      hipEvent_t* ev = timing_pair(ctx);
      launch_action(ctx, op, vec, K, ls, sk, lam_host, o.seed, o.pi_start, outs, o, tol, s, link,
                    &ctx->h_pool[base + i], offsetof(LejaStatus, trace), ev, &tiled, false, true);
      pend.push_back({base + i, K, tiled, ev});
    };
    scheme_steps(act_async);
    if (ctx->deferring) {
      DeferredCall dc;
      dc.is_step = true;
      dc.scheme = scheme;
      dc.op = op;
      dc.o = o;
      dc.h = h;
      dc.tol = tol;
      dc.u_out = u_out;
      dc.err = err;
      dc.stats = stats;
      dc.launches = pend;
      ctx->defer->calls.push_back(dc);
      ctx->defer_next = base + (int)pend.size();
      return LJ_OK;
    }
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (collect_async(ctx, op, pend, log, lam_found, pit)) {
      if (stats)
        for (size_t i = 0; i < log.size(); ++i) stats[i] = log[i];
      return LJ_OK;
    }
    log.clear();
    o.bound = lam_found;
  }
  // ---- the step, synchronously: one spectral bound for the whole step
  if (!(o.bound > 0.0) && o.bound_device) {
    o.bound = bound_to_host(ctx, o.bound_device, s);
  } else if (!(o.bound > 0.0)) {
    o.bound = run_bound(ctx, op, o, o.power_iters, o.seed, o.pi_start, s);
    pit = o.power_iters;
  }
  auto act = [&](const double* vec, int K, const int* ls, const double* as, double* const* outs) {
    lj_stats st;
    const int rc = vertical_impl(ctx, op, vec, K, ls, as, h, tol, outs, o, &st, s);
    if (rc != LJ_OK) ok = false;
    log.push_back(st);
  };
  scheme_steps(act);
  HIPCHK(ctx, hipStreamSynchronize(s));
  if (!log.empty()) log[0].power_iters = pit;
  if (stats)
    for (size_t i = 0; i < log.size(); ++i) stats[i] = log[i];
  return ok ? LJ_OK : LJ_ENOTCONV;
}

LJ_API int lj_step(lj_context* ctx, int scheme, const lj_operator* J, double h, double tol, double* u_out,
                   double* err, const lj_options* opt, lj_stats* stats, int nstats, int* ncalls, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    Opts o = resolve(ctx, opt);
    if (scheme < LJ_EXPRB2 || scheme > LJ_EPIRK4S3A_LEKRY) invalid(ctx, "unknown scheme");
    if (op.state == nullptr) invalid(ctx, "lj_step needs the state u in J->state");
    if (!std::isfinite(h)) invalid(ctx, "h must be finite");
    if (!(tol > 0.0) || !std::isfinite(tol)) invalid(ctx, "tol must be finite and > 0");
    check_vec(ctx, op, u_out, "u_out");
    if (u_out == op.state) invalid(ctx, "u_out must not alias the state");
    if (err) {
      check_vec(ctx, op, err, "err");
      if (err == op.state || err == u_out) invalid(ctx, "err must not alias the state or u_out");
    }
    const int want = (scheme == LJ_EXPRB2) ? 1 : (scheme == LJ_EXPRB43) ? 4 : 3;  // EPIRK4s3 (LeKry): 3
    if (ncalls) *ncalls = want;
    if (stats && nstats < want) invalid(ctx, "nstats is smaller than the number of Leja calls of the scheme");
    return step_impl(ctx, scheme, op, o, h, tol, u_out, err, stats, reinterpret_cast<hipStream_t>(stream));
  });
}

LJ_API int lj_user_step(lj_context* ctx, int scheme, const lj_user_operator* J, double h, double tol,
                        double* u_out, double* err, const lj_options* opt, lj_stats* stats, int nstats,
                        int* ncalls, void* stream) {
  return guarded(ctx, [&]() {
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Opts o = resolve(ctx, opt);
    if (o.use_proposal) invalid(ctx, "the learned proposal needs a built-in operator family");
    if (scheme < LJ_EXPRB2 || scheme > LJ_EPIRK4S3A_LEKRY) invalid(ctx, "unknown scheme");
    if (!std::isfinite(h)) invalid(ctx, "h must be finite");
    if (!(tol > 0.0) || !std::isfinite(tol)) invalid(ctx, "tol must be finite and > 0");
    UserScope us(ctx, J, true, s);
    check_vec(ctx, us.op, u_out, "u_out");
    if (u_out == us.op.state) invalid(ctx, "u_out must not alias the state");
    if (err) {
      check_vec(ctx, us.op, err, "err");
      if (err == us.op.state || err == u_out) invalid(ctx, "err must not alias the state or u_out");
    }
    const int want = (scheme == LJ_EXPRB2) ? 1 : (scheme == LJ_EXPRB43) ? 4 : 3;  // EPIRK4s3 (LeKry): 3
    if (ncalls) *ncalls = want;
    if (stats && nstats < want) invalid(ctx, "nstats is smaller than the number of Leja calls of the scheme");
    return step_impl(ctx, scheme, us.op, o, h, tol, u_out, err, stats, s);
  });
}

// ---- variable step sizes (Sec. 2.3) -------------------------------------------
namespace {
// cost controller constants as printed (Sec. 2.3)
constexpr double kCostAlpha = 0.65241444, kCostBeta = 0.26862269, kCostLambda = 1.37412002,
                 kCostDelta = 0.64446017;
// a rejected attempt is retried at this fraction of the traditional size: an
// error estimate that falls more slowly than dt^{p+1} (stiff order
// reduction) would otherwise creep down over many rejections
constexpr double kRetrySafety = 0.9;

double traditional_factor(double e, double tol, int p) {
  if (e == 0.0) return INFINITY;
  return std::pow(tol / e, 1.0 / (p + 1));
}

// g from the step sizes and costs per unit time of two consecutive accepted steps
double cost_factor(double dt, double dt_prev, double c, double c_prev) {
  const double D = (dt == dt_prev) ? 0.0 : (std::log(c) - std::log(c_prev)) / (std::log(dt) - std::log(dt_prev));
  const double sf = std::exp(-kCostAlpha * std::tanh(kCostBeta * D));
  if (sf >= 1.0 && sf < kCostLambda) return kCostLambda;
  if (sf >= kCostDelta && sf < 1.0) return kCostDelta;
  return sf;
}
}  // namespace

// Variable step sizes from u(0) = op0.state (Sec. 2.3).  before_step(u) runs
// before every attempt with the state it linearises at (user operators
// refresh their callbacks' state there).
extern "C++" {
template <class BeforeStep>
int integrate_impl(lj_context* ctx, int scheme, const OpDev& op0, const Opts& o, double T, double dt0, double tol,
                   double leja_tol, double* u_out, lj_integrate_stats* stats, lj_step_record* log, int log_cap,
                   int max_attempts, hipStream_t s, BeforeStep&& before_step) {
  if (scheme != LJ_EPIRK4S3 && scheme != LJ_EXPRB43 && scheme != LJ_EPIRK4S3_LEKRY && scheme != LJ_EPIRK4S3A &&
      scheme != LJ_EPIRK4S3A_LEKRY)
    invalid(ctx, "lj_integrate needs an embedded scheme");
  if (op0.state == nullptr) invalid(ctx, "lj_integrate needs u(0) in J->state");
  if (!(T >= 0.0) || !std::isfinite(T)) invalid(ctx, "T must be finite and >= 0");
  if (!(dt0 > 0.0) || !std::isfinite(dt0)) invalid(ctx, "dt0 must be finite and > 0");
  if (!(tol > 0.0) || !std::isfinite(tol)) invalid(ctx, "tol must be finite and > 0");
  if (!(leja_tol > 0.0) || !std::isfinite(leja_tol)) invalid(ctx, "leja_tol must be finite and > 0");
  if (log_cap < 0 || (log_cap > 0 && !log)) invalid(ctx, "log is NULL but log_cap > 0");
  if (max_attempts < 1) invalid(ctx, "max_attempts must be >= 1");
  check_vec(ctx, op0, u_out, "u_out");
  if (u_out == op0.state) invalid(ctx, "u_out must not alias the state");
  const size_t n = nvals(op0);
  const int p = 3;  // order of the embedded (lower-order) solution of the schemes
  double* ub[2] = {slot(ctx, W_IU0, n), slot(ctx, W_IU1, n)};
  double* errv = slot(ctx, W_IERR, n);
  HIPCHK(ctx, hipMemcpyAsync(ub[0], op0.state, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  lj_integrate_stats st{};
  int cur = 0, attempts = 0;
  double t = 0.0, dt = dt0;
  bool have_prev = false;
  double prev_dt = 0.0, prev_rate = 0.0;
  int rc = LJ_OK;
  while (t < T) {
    if (attempts >= max_attempts) {
      rc = LJ_ENOTCONV;
      break;
    }
    const bool last = dt >= T - t;
    const double h = last ? T - t : dt;
    OpDev op = op0;
    op.state = ub[cur];
    before_step(ub[cur]);
    lj_stats calls[LJ_MAX_K];
    const int src = step_impl(ctx, scheme, op, o, h, leja_tol, ub[cur ^ 1], errv, calls, s);
    const int ncalls = (scheme == LJ_EXPRB43) ? 4 : 3;
    int cost = 0;
    bool ok = src == LJ_OK;
    for (int i = 0; i < ncalls; ++i) {
      cost += calls[i].iters_total + calls[i].power_iters;
      ok = ok && calls[i].converged;
    }
    st.products += cost;
    double e = INFINITY;
    if (ok) {
      HIPCHK(ctx, launch_sumsq2(errv, ub[cur ^ 1], (long)n, ctx->d_sumsq, ctx->d_sumsq + 2 * kSumsqBlocks, s));
      HIPCHK(ctx, hipMemcpyAsync(ctx->h_sumsq, ctx->d_sumsq + 2 * kSumsqBlocks, 2 * sizeof(double),
                                 hipMemcpyDeviceToHost, s));
      HIPCHK(ctx, hipStreamSynchronize(s));
      const double ne = std::sqrt(ctx->h_sumsq[0]), nu = std::sqrt(ctx->h_sumsq[1]);
      e = nu > 0.0 ? ne / nu : ne;
    }
    const bool accept = ok && e <= tol;
    if (log && attempts < log_cap) log[attempts] = lj_step_record{t, h, e, cost, accept ? 1 : 0};
    ++attempts;
    if (!ok) {
      st.rejected += 1;
      dt = 0.5 * h;
    } else if (accept) {
      st.accepted += 1;
      t = last ? T : t + h;
      cur ^= 1;
      const double rate = cost / h;
      const double d_trad = h * traditional_factor(e, tol, p);
      const double d_cost = have_prev ? h * cost_factor(h, prev_dt, rate, prev_rate) : h * cost_factor(h, h, 1, 1);
      have_prev = true;
      prev_dt = h;
      prev_rate = rate;
      dt = std::min(d_trad, d_cost);
    } else {
      st.rejected += 1;
      dt = kRetrySafety * h * traditional_factor(e, tol, p);
    }
  }
  HIPCHK(ctx, hipMemcpyAsync(u_out, ub[cur], n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(ctx, hipStreamSynchronize(s));
  st.t = t;
  st.dt_next = dt;
  if (stats) *stats = st;
  return rc;
}
}  // extern "C++"

LJ_API int lj_integrate(lj_context* ctx, int scheme, const lj_operator* J, double T, double dt0, double tol,
                        double leja_tol, double* u_out, const lj_options* opt, lj_integrate_stats* stats,
                        lj_step_record* log, int log_cap, int max_attempts, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op0 = make_op(ctx, J);
    const Opts o = resolve(ctx, opt);
    return integrate_impl(ctx, scheme, op0, o, T, dt0, tol, leja_tol, u_out, stats, log, log_cap, max_attempts,
                          reinterpret_cast<hipStream_t>(stream), [](const double*) {});
  });
}

LJ_API int lj_user_integrate(lj_context* ctx, int scheme, const lj_user_operator* J, double T, double dt0,
                             double tol, double leja_tol, double* u_out, const lj_options* opt,
                             lj_integrate_stats* stats, lj_step_record* log, int log_cap, int max_attempts,
                             void* stream) {
  return guarded(ctx, [&]() {
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Opts o = resolve(ctx, opt);
    if (o.use_proposal) invalid(ctx, "the learned proposal needs a built-in operator family");
    UserScope us(ctx, J, true, s);
    // the callbacks see the state of each attempt; finite differences need
    // f(u) and ||u|| at it
    auto before = [&](const double* u) {
      us.U.J.state = u;
      if (us.U.fd) {
        double* fu = slot(ctx, W_UFU, (size_t)J->n);
        call_rhs(ctx, u, fu, s);
        us.U.fu = fu;
        HIPCHK(ctx, launch_user_norm_u(ctx->d_ustate, u, (long)J->n, ctx->d_upart, s));
      }
    };
    return integrate_impl(ctx, scheme, us.op, o, T, dt0, tol, leja_tol, u_out, stats, log, log_cap, max_attempts,
                          s, before);
  });
}

LJ_API int lj_last_trace(lj_context* ctx, double* out, int rows) {
  if (!ctx || !out || rows < 0) return LJ_EINVAL;
  // the trace stays in device memory (status heads reach the host directly):
  // read the last launch's status, head and trace together
  static_assert(sizeof(LejaStatus) < 16384, "status copied through the stack");
  LejaStatus S;
  if (hipSetDevice(ctx->device) != hipSuccess || hipDeviceSynchronize() != hipSuccess ||
      hipMemcpy(&S, ctx->d_status, sizeof(S), hipMemcpyDeviceToHost) != hipSuccess) {
    (void)hipGetLastError();
    return LJ_EHIP;
  }
  const int have = S.iters;
  const int n = rows < have ? rows : have;
  for (int m = 0; m < n; ++m)
    for (int q = 0; q < 1 + kMaxK; ++q) out[m * (1 + kMaxK) + q] = S.trace[m][q];
  return n;
}

LJ_API int lj_last_profile(lj_context* ctx, double* us) {
  if (!ctx || !us) return LJ_EINVAL;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0)
    return LJ_EHIP;
  for (int q = 0; q < 8; ++q) us[q] = (double)ctx->h_status->prof[q] * 1e3 / (double)khz;
  return LJ_OK;
}

LJ_API int lj_timing_enable(lj_context* ctx, int enable) {
  return guarded(ctx, [&]() {
    if (enable && ctx->tev.empty()) {
      ctx->tev.assign(2 * kTimingPairs, nullptr);
      // timing-only events: no system-scope fence (cache write-back and
      // invalidation) when they are recorded between the launches of a step
      for (auto& e : ctx->tev) HIPCHK(ctx, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    ctx->timing = enable != 0;
    return LJ_OK;
  });
}

LJ_API int lj_timing_read(lj_context* ctx, lj_timing* out, int reset) {
  if (!out) return LJ_EINVAL;
  return guarded(ctx, [&]() {
    timing_flush(ctx);
    *out = ctx->tm;
    if (reset) std::memset(&ctx->tm, 0, sizeof(ctx->tm));
    return LJ_OK;
  });
}

// ---- learned proposal ------------------------------------------------------
LJ_API int lj_features(lj_context* ctx, const lj_operator* J, double h, int l, float* feats, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    if (!std::isfinite(h) || !(h > 0.0)) invalid(ctx, "h must be finite and > 0");
    if (l < 0 || l > LJ_MAX_L) invalid(ctx, "l must be in [0, 4]");
    check_fvec(ctx, feats, kMlpIn, "feats");
    mlp_alloc(ctx);
    FeatureJob Jb;
    std::memset(&Jb, 0, sizeof(Jb));
    Jb.op = op;
    Jb.K = 1;
    Jb.h[0] = h;
    Jb.l[0] = l;
    HIPCHK(ctx, launch_features(Jb, ctx->d_featpart, feats, ctx->d_gers, reinterpret_cast<hipStream_t>(stream)));
    return LJ_OK;
  });
}

LJ_API int lj_gershgorin_bound(lj_context* ctx, const lj_operator* J, double* bound, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    if (!bound) invalid(ctx, "bound is NULL");
    if (is_user(op)) invalid(ctx, "lj_gershgorin_bound needs a built-in operator family");
    mlp_alloc(ctx);
    FeatureJob Jb;
    std::memset(&Jb, 0, sizeof(Jb));
    Jb.op = op;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(ctx, launch_features(Jb, ctx->d_featpart, nullptr, ctx->d_gers, s));
    HIPCHK(ctx, hipMemcpyAsync(bound, ctx->d_gers, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    return LJ_OK;
  });
}

LJ_API int lj_proposal_record(lj_context* ctx, const lj_operator* J, double h, int l, double bound, int substeps,
                              float* feats, float* targets, void* stream) {
  return guarded(ctx, [&]() {
    const OpDev op = make_op(ctx, J);
    if (!std::isfinite(h) || !(h > 0.0)) invalid(ctx, "h must be finite and > 0");
    if (l < 0 || l > LJ_MAX_L) invalid(ctx, "l must be in [0, 4]");
    if (!std::isfinite(bound) || !(bound > 0.0)) invalid(ctx, "bound must be finite and > 0");
    if (substeps < 1 || (substeps & (substeps - 1)) != 0) invalid(ctx, "substeps must be a power of two >= 1");
    check_fvec(ctx, feats, kMlpIn, "feats");
    check_fvec(ctx, targets, kMlpOut, "targets");
    mlp_alloc(ctx);
    FeatureJob Jb;
    std::memset(&Jb, 0, sizeof(Jb));
    Jb.op = op;
    Jb.K = 1;
    Jb.h[0] = h;
    Jb.l[0] = l;
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(ctx, launch_features(Jb, ctx->d_featpart, feats, ctx->d_gers, s));
    HIPCHK(ctx, launch_proposal_targets(ctx->d_gers, bound, substeps, targets, s));
    return LJ_OK;
  });
}

LJ_API int lj_mlp_init(lj_context* ctx, uint64_t seed) {
  return guarded(ctx, [&]() {
    mlp_alloc(ctx);
    std::vector<float> m;
    mlp_host_init(seed, m);
    HIPCHK(ctx, hipMemcpy(ctx->d_model, m.data(), kModelFloats * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(ctx->d_adam, 0, 2 * kMlpParams * sizeof(float)));
    HIPCHK(ctx, hipMemset(ctx->d_adam_t, 0, sizeof(int)));
    ctx->mlp_ready = false;
    return LJ_OK;
  });
}

LJ_API int lj_mlp_train(lj_context* ctx, const float* feats, const float* targets, int n, int epochs, int batch,
                        float lr, int fit_normalization, float* loss_per_epoch, void* stream) {
  return guarded(ctx, [&]() {
    if (!ctx->d_model) invalid(ctx, "lj_mlp_train: call lj_mlp_init (or lj_mlp_set / lj_mlp_load) first");
    if (n < 1) invalid(ctx, "n must be >= 1");
    if (epochs < 1 || epochs > kMaxEpochs) invalid(ctx, "epochs must be in [1, 4096]");
    if (batch < 1 || batch > kMlpBlock) invalid(ctx, "batch must be in [1, 512]");
    if (!(lr > 0.0f) || !std::isfinite(lr)) invalid(ctx, "lr must be finite and > 0");
    check_fvec(ctx, feats, (size_t)n * kMlpIn, "feats");
    check_fvec(ctx, targets, (size_t)n * kMlpOut, "targets");
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (fit_normalization) HIPCHK(ctx, launch_mlp_normalize(ctx->d_model, feats, targets, n, s));
    HIPCHK(ctx, launch_mlp_train(ctx->d_model, ctx->d_adam, ctx->d_adam + kMlpParams, ctx->d_adam_t, feats, targets, n,
                                 epochs, batch, lr, ctx->d_rows, ctx->d_scalars + 1, s));
    if (loss_per_epoch)
      HIPCHK(ctx, hipMemcpyAsync(loss_per_epoch, ctx->d_scalars + 1, epochs * sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    ctx->mlp_ready = true;
    return LJ_OK;
  });
}

LJ_API int lj_mlp_predict(lj_context* ctx, const float* feats, int n, float* out, void* stream) {
  return guarded(ctx, [&]() {
    if (!ctx->d_model) invalid(ctx, "no network (lj_mlp_init, lj_mlp_set or lj_mlp_load first)");
    if (n < 1) invalid(ctx, "n must be >= 1");
    check_fvec(ctx, feats, (size_t)n * kMlpIn, "feats");
    check_fvec(ctx, out, (size_t)n * kMlpOut, "out");
    HIPCHK(ctx, launch_mlp_forward(ctx->d_model, feats, n, out, reinterpret_cast<hipStream_t>(stream)));
    return LJ_OK;
  });
}

LJ_API int lj_mlp_grad(lj_context* ctx, const float* feats, const float* targets, int n, float* grad, float* loss,
                       void* stream) {
  return guarded(ctx, [&]() {
    if (!ctx->d_model) invalid(ctx, "no network (lj_mlp_init, lj_mlp_set or lj_mlp_load first)");
    if (n < 1) invalid(ctx, "n must be >= 1");
    check_fvec(ctx, feats, (size_t)n * kMlpIn, "feats");
    check_fvec(ctx, targets, (size_t)n * kMlpOut, "targets");
    check_fvec(ctx, grad, kMlpParams, "grad");
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(ctx, launch_mlp_grad(ctx->d_model, feats, targets, n, ctx->d_rows, grad, ctx->d_scalars, s));
    float l = 0.0f;
    HIPCHK(ctx, hipMemcpyAsync(&l, ctx->d_scalars, sizeof(float), hipMemcpyDeviceToHost, s));
    HIPCHK(ctx, hipStreamSynchronize(s));
    if (loss) *loss = l;
    return LJ_OK;
  });
}

LJ_API int lj_mlp_get(lj_context* ctx, float* model) {
  return guarded(ctx, [&]() {
    if (!model) invalid(ctx, "model is NULL");
    if (!ctx->d_model) invalid(ctx, "no network");
    HIPCHK(ctx, hipMemcpy(model, ctx->d_model, kModelFloats * sizeof(float), hipMemcpyDeviceToHost));
    return LJ_OK;
  });
}

LJ_API int lj_mlp_set(lj_context* ctx, const float* model) {
  return guarded(ctx, [&]() {
    if (!model) invalid(ctx, "model is NULL");
    for (int i = 0; i < kModelFloats; ++i)
      if (!std::isfinite(model[i])) invalid(ctx, "model has a non-finite value");
    for (int i = 0; i < kMlpIn; ++i)
      if (!(model[kMlpParams + kMlpIn + i] > 0.0f)) invalid(ctx, "model: feature std must be > 0");
    for (int i = 0; i < kMlpOut; ++i)
      if (!(model[kMlpParams + 2 * kMlpIn + kMlpOut + i] > 0.0f)) invalid(ctx, "model: target std must be > 0");
    mlp_alloc(ctx);
    HIPCHK(ctx, hipMemcpy(ctx->d_model, model, kModelFloats * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMemset(ctx->d_adam, 0, 2 * kMlpParams * sizeof(float)));
    HIPCHK(ctx, hipMemset(ctx->d_adam_t, 0, sizeof(int)));
    ctx->mlp_ready = true;
    return LJ_OK;
  });
}

// File: 8-byte tag "LJMLP001", int32 float count, then the model floats
// (little-endian IEEE single).
LJ_API int lj_mlp_save(lj_context* ctx, const char* path) {
  return guarded(ctx, [&]() {
    if (!path) invalid(ctx, "path is NULL");
    if (!ctx->d_model) invalid(ctx, "no network");
    std::vector<float> m(kModelFloats);
    HIPCHK(ctx, hipMemcpy(m.data(), ctx->d_model, kModelFloats * sizeof(float), hipMemcpyDeviceToHost));
    FILE* f = std::fopen(path, "wb");
    if (!f) invalid(ctx, std::string("cannot open ") + path);
    const int32_t cnt = kModelFloats;
    const bool ok = std::fwrite("LJMLP001", 1, 8, f) == 8 && std::fwrite(&cnt, 4, 1, f) == 1 &&
                    std::fwrite(m.data(), sizeof(float), m.size(), f) == m.size();
    std::fclose(f);
    if (!ok) invalid(ctx, std::string("cannot write ") + path);
    return LJ_OK;
  });
}

LJ_API int lj_mlp_load(lj_context* ctx, const char* path) {
  return guarded(ctx, [&]() {
    if (!path) invalid(ctx, "path is NULL");
    FILE* f = std::fopen(path, "rb");
    if (!f) invalid(ctx, std::string("cannot open ") + path);
    char tag[8];
    int32_t cnt = 0;
    std::vector<float> m(kModelFloats);
    const bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, "LJMLP001", 8) == 0 &&
                    std::fread(&cnt, 4, 1, f) == 1 && cnt == kModelFloats &&
                    std::fread(m.data(), sizeof(float), m.size(), f) == m.size();
    std::fclose(f);
    if (!ok) invalid(ctx, std::string("not a network file of this library: ") + path);
    return lj_mlp_set(ctx, m.data());
  });
}

// ---- batching form ---------------------------------------------------------
LJ_API int lj_batch_create(lj_context* ctx, const lj_operator* ops, int n, const double* const* v, const double* h,
                           int K, const int* l, const double* a, double tol, double* const* w, const double* bounds,
                           const lj_options* opt, lj_batch** out) {
  if (out) *out = nullptr;
  lj_batch* b = nullptr;
  const int rc = guarded(ctx, [&]() {
    if (!out) invalid(ctx, "out is NULL");
    if (n < 1) invalid(ctx, "n must be >= 1");
    if (!ops || !v || !h || !w) invalid(ctx, "ops, v, h and w must not be NULL");
    if (K < 1 || K > LJ_MAX_K) invalid(ctx, "K must be in [1, 4]");
    if (!l || !a) invalid(ctx, "l and a must not be NULL");
    if (!(tol > 0.0) || !std::isfinite(tol)) invalid(ctx, "tol must be finite and > 0");
    for (int k = 0; k < K; ++k) {
      if (l[k] < 0 || l[k] > LJ_MAX_L) invalid(ctx, "l must be in [0, 4]");
      if (!std::isfinite(a[k])) invalid(ctx, "a[k] must be finite");
    }
    b = new lj_batch();
    b->ctx = ctx;
    b->n = n;
    b->K = K;
    b->kind = ops[0].kind;
    b->tol = tol;
    b->o = resolve(ctx, opt);
    for (int k = 0; k < K; ++k) {
      b->l[k] = l[k];
      b->a[k] = a[k];
    }
    for (int i = 0; i < n; ++i) {
      if (ops[i].kind != b->kind) invalid(ctx, "all operators of a batch must be of one family");
      const OpDev op = make_op(ctx, &ops[i]);
      if (!std::isfinite(h[i])) invalid(ctx, "h[i] must be finite");
      check_vec(ctx, op, v[i], "v[i]");
      for (int k = 0; k < K; ++k) {
        double* wk = w[(size_t)i * K + k];
        check_vec(ctx, op, wk, "w[i*K+k]");
        if (wk == v[i] || wk == op.state) invalid(ctx, "w must not alias v or the operator state");
        for (int q = 0; q < k; ++q)
          if (w[(size_t)i * K + q] == wk) invalid(ctx, "the outputs of an instance must be distinct");
      }
      if (bounds && (!(bounds[i] >= 0.0) || !std::isfinite(bounds[i])))
        invalid(ctx, "bounds[i] must be finite and >= 0");
      b->ops.push_back(op);
      b->v.push_back(v[i]);
      b->h.push_back(h[i]);
      for (int k = 0; k < K; ++k) b->w.push_back(w[(size_t)i * K + k]);
      b->nval.push_back((long long)nvals(op));
      b->total_values += (long long)nvals(op);
    }
    // device-side description: two basis vectors per instance, and, when
    // substeps may be taken, max(l, 1) + 1 substep vectors per instance
    HIPCHK(ctx, hipMalloc(&b->d_work, (size_t)2 * b->total_values * sizeof(double)));
    int lmax = 0;
    for (int k = 0; k < K; ++k) lmax = std::max(lmax, l[k]);
    const int nsub = (b->o.max_substeps >= 2) ? std::max(lmax, 1) + 1 : 0;
    if (nsub > 0) HIPCHK(ctx, hipMalloc(&b->d_sub, (size_t)nsub * b->total_values * sizeof(double)));
    std::vector<BatchItem> items(n);
    size_t off = 0;
    for (int i = 0; i < n; ++i) {
      BatchItem& it = items[i];
      std::memset(&it, 0, sizeof(it));
      it.op = b->ops[i];
      it.v = v[i];
      for (int k = 0; k < K; ++k) {
        it.p[k] = w[(size_t)i * K + k];
        it.s[k] = a[k] * h[i];
      }
      it.y0 = b->d_work + off;
      it.y1 = b->d_work + off + b->nval[i];
      it.sub = (nsub > 0) ? b->d_sub + (size_t)nsub * off / 2 : nullptr;
      it.nsub_stride = (size_t)b->nval[i];
      off += 2 * (size_t)b->nval[i];
      it.lam_in = (bounds && bounds[i] > 0.0) ? bounds[i] : (b->o.bound > 0.0 ? b->o.bound : 0.0);
    }
    HIPCHK(ctx, hipMalloc(&b->d_items, n * sizeof(BatchItem)));
    HIPCHK(ctx, hipMemcpy(b->d_items, items.data(), n * sizeof(BatchItem), hipMemcpyHostToDevice));
    HIPCHK(ctx, hipMalloc(&b->d_status, n * sizeof(BatchStatus)));
    HIPCHK(ctx, hipMemset(b->d_status, 0, n * sizeof(BatchStatus)));
    HIPCHK(ctx, hipHostMalloc(&b->h_status, n * sizeof(BatchStatus), hipHostMallocDefault));
    HIPCHK(ctx, hipMalloc(&b->d_order, n * sizeof(int)));
    b->max_blocks = 0;
    for (int i = 0; i < kNumBatchSchedules; ++i)
      b->max_blocks = std::max(b->max_blocks, ctx->num_cus * kBatchSchedules[i].per_cu);
    HIPCHK(ctx, hipMalloc(&b->d_queue, (size_t)(1 + b->max_blocks) * kTeamWords * sizeof(unsigned int)));
    HIPCHK(ctx, hipMalloc(&b->d_team_part, (size_t)2 * kQ_batch * b->max_blocks * sizeof(double)));
    HIPCHK(ctx, hipStreamCreateWithFlags(&b->cs, hipStreamNonBlocking));
    BatchParams& P = b->P;
    P.items = b->d_items;
    P.status = b->d_status;
    P.order = b->d_order;
    P.n = n;
    P.K = K;
    for (int k = 0; k < kMaxK; ++k) P.l[k] = (k < K) ? l[k] : 0;
    P.power_iters = b->o.power_iters;
    P.seed = b->o.seed;
    P.safety = b->o.safety;
    P.max_points = b->o.max_points;
    P.max_substeps = b->o.max_substeps;
    P.relative = b->o.relative;
    P.tol = tol;
    P.hump = b->o.hump;
    P.xi = ctx->d_xi;
    P.queue = b->d_queue;
    // pick the schedule, then capture its launch (queue reset + kernel) in a graph
    b->schedule = batch_tune(b);
    batch_set_order(b, b->schedule);
    HIPCHK(ctx, hipStreamBeginCapture(b->cs, hipStreamCaptureModeThreadLocal));
    batch_launch(b, b->schedule, b->cs);
    HIPCHK(ctx, hipStreamEndCapture(b->cs, &b->graph));
    HIPCHK(ctx, hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    HIPCHK(ctx, hipStreamSynchronize(b->cs));
    *out = b;
    b = nullptr;
    return LJ_OK;
  });
  if (b) batch_release(b);
  return rc;
}

LJ_API int lj_batch_run(lj_batch* b, void* stream) {
  if (!b) return LJ_EINVAL;
  return guarded(b->ctx, [&]() {
    HIPCHK(b->ctx, hipGraphLaunch(b->exec, reinterpret_cast<hipStream_t>(stream)));
    return LJ_OK;
  });
}

LJ_API int lj_batch_stats(lj_batch* b, lj_stats* per_instance, void* stream) {
  if (!b) return LJ_EINVAL;
  lj_context* ctx = b->ctx;
  return guarded(ctx, [&]() {
    const hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    HIPCHK(ctx, hipStreamSynchronize(s));
    unsigned int qw[2] = {0, 0};
    HIPCHK(ctx, hipMemcpy(qw, b->d_queue, sizeof(qw), hipMemcpyDeviceToHost));
    if (qw[1] != 0u) {
      ctx->err = "batch launch aborted: a team barrier timed out (blocks of a team were not co-resident)";
      throw Fail{LJ_EHIP};
    }
    HIPCHK(ctx, hipMemcpy(b->h_status, b->d_status, b->n * sizeof(BatchStatus), hipMemcpyDeviceToHost));
    bool all_ok = true;
    double bytes = 0.0;
    for (int i = 0; i < b->n; ++i) {
      const BatchStatus& S = b->h_status[i];
      bytes += (double)b->nval[i] * (24.0 * S.iters + 16.0 * S.accum_iters + 24.0 * S.power_iters + 8.0 +
                                      8.0 * b->K + 8.0 * S.vec_passes);
      lj_stats st;
      std::memset(&st, 0, sizeof(st));
      for (int k = 0; k < LJ_MAX_K; ++k) {
        st.m_star[k] = -1;
        st.substeps[k] = 1;
      }
      st.iters_total = S.iters;
      st.power_iters = S.power_iters;
      st.bound = S.lam;
      st.c = S.c;
      st.gamma = S.gamma;
      st.rejections = S.rejections;
      st.converged = 1;
      for (int k = 0; k < b->K; ++k) {
        st.substeps[k] = S.substeps[k];
        if (S.state[k] == ACC_CONVERGED) {
          st.m_star[k] = S.m_star[k];
          st.err_est[k] = S.err[k];
        } else {
          st.converged = 0;
        }
      }
      if (!st.converged) all_ok = false;
      if (per_instance) per_instance[i] = st;
    }
    b->alg_bytes = bytes;
    return all_ok ? LJ_OK : LJ_ENOTCONV;
  });
}

LJ_API int lj_batch_info(const lj_batch* b, lj_batch_info_t* out) {
  if (!b || !out) return LJ_EINVAL;
  std::memset(out, 0, sizeof(*out));
  const BatchSchedule& S = kBatchSchedules[b->schedule];
  out->schedule = b->schedule;
  out->block_size = S.block;
  out->blocks = b->ctx->num_cus * S.per_cu;
  out->team = S.team;
  out->largest_first = S.largest_first;
  out->nschedules = kNumBatchSchedules;
  for (int i = 0; i < kNumBatchSchedules && i < 8; ++i) out->tune_ms[i] = b->tune_ms[i];
  out->total_values = b->total_values;
  out->alg_bytes = b->alg_bytes;
  return LJ_OK;
}

LJ_API int lj_batch_timeline(const lj_batch* b, int* block, double* start_us, double* end_us) {
  if (!b || !block || !start_us || !end_us) return LJ_EINVAL;
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, b->ctx->device) != hipSuccess || khz <= 0)
    return LJ_EHIP;
  unsigned long long t_min = ~0ull;
  for (int i = 0; i < b->n; ++i) t_min = std::min(t_min, b->h_status[i].t0);
  for (int i = 0; i < b->n; ++i) {
    const BatchStatus& S = b->h_status[i];
    block[i] = S.block;
    start_us[i] = (double)(S.t0 - t_min) * 1e3 / khz;
    end_us[i] = (double)(S.t1 - t_min) * 1e3 / khz;
  }
  return LJ_OK;
}

LJ_API void lj_batch_destroy(lj_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  batch_release(b);
}

}  // extern "C"
