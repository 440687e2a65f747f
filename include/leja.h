/*
 * leja.h -- C ABI of the MI355X (gfx950) Leja phi-action library.
 *
 * The library computes w = phi_l(h J) v for a matrix-free stencil Jacobian J by
 * polynomial interpolation at Leja points (Deka, Tokman, Einkemmer, "A
 * comparison of Leja- and Krylov-based iterative schemes for Exponential
 * Integrators", Sec. 2.2), in its vertical form (Sec. 4), with substepping on
 * non-convergence, plus an exponential-integrator stage driver (the schemes of
 * Sec. 5.1 and 5.4).
 *
 * Conventions for every entry point:
 *   - Vector arguments are DEVICE pointers to contiguous IEEE float64 arrays on
 *     the context's device, of length n = nx*ny*ncomp.  Grids are row-major
 *     with x fastest; two-component states are interleaved (u, v) per point.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  All
 *     device work is enqueued on it.  Calls that return statistics or a
 *     convergence verdict synchronise that stream once before returning.
 *   - The caller owns every buffer it passes.  Output vectors must not alias
 *     input vectors or the operator state.  The library owns the workspace it
 *     keeps inside the context (grown on demand, freed by lj_destroy).
 *   - A context is used by one host thread at a time; calls on one context are
 *     serialised.  Contexts on different devices are independent.
 *   - Return codes: LJ_OK (0); LJ_ENOTCONV (1): the expansion did not converge
 *     within max_substeps (outputs hold the last attempt, statistics are
 *     filled); LJ_EINVAL (-1): an argument is invalid, nothing was enqueued;
 *     LJ_EHIP (-2): a HIP runtime call failed; LJ_ENOMEM (-3): workspace
 *     allocation failed.  lj_last_error() describes the last failure.  No C++
 *     exception crosses this interface.
 */
#ifndef LEJA_H
#define LEJA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LJ_API __attribute__((visibility("default")))

#define LJ_OK 0
#define LJ_ENOTCONV 1
#define LJ_EINVAL (-1)
#define LJ_EHIP (-2)
#define LJ_ENOMEM (-3)

/* Most accumulators that share one Newton basis (vertical form, Sec. 4), and
 * the highest phi index accepted (the schemes of Sec. 5 use phi_1..phi_4). */
#define LJ_MAX_K 4
#define LJ_MAX_L 4
/* Most Leja points (the table holds LJ_MAX_POINTS + 1 nodes). */
#define LJ_MAX_POINTS 100

typedef struct lj_context lj_context;

/* Operator families (Sec. 3 test problems, 2nd-order centred differences; the
 * grids are periodic except for LJ_OP_ADR2D).  coef[] meaning per kind:
 *   LJ_OP_DIAG          J = diag(state); nx = n, ny = 1; coef unused
 *   LJ_OP_ADVDIFF2D     J = nu Lap - ax d/dx - ay d/dy;  coef = {nu, ax, ay}; state NULL
 *   LJ_OP_ALLENCAHN2D   f = eps Lap u + u - u^3, J = eps Lap + diag(1 - 3u^2); coef = {eps}
 *   LJ_OP_BRUSSELATOR2D f = (Du Lap u + a - (b+1)u + u^2 v, Dv Lap v + b u - u^2 v),
 *                       ncomp = 2, coef = {Du, Dv, a, b}
 *   LJ_OP_BURGERS2D     f = nu Lap u - (d/dx + d/dy)(u^2/2), J v = nu Lap v - (d/dx + d/dy)(u v);
 *                       coef = {nu}
 *   LJ_OP_GRAYSCOTT2D   f = (a1 Lap u - u v^2 + a(1 - u), a2 Lap v + u v^2 - (a + b) v),
 *                       ncomp = 2, coef = {a1, a2, a, b} (Sec. 3)
 *   LJ_OP_ADR2D         f = alpha Lap u + beta (d/dx + d/dy) u + rate u (1 - u)(u - 1/2),
 *                       J = alpha Lap + beta (d/dx + d/dy) + diag(rate (-3u^2 + 3u - 1/2));
 *                       coef = {alpha, beta, rate} (Sec. 3, advection-diffusion-reaction).
 *                       Homogeneous Neumann boundaries on a cell-centred grid: the
 *                       ghost value beyond a boundary face equals the cell inside it.
 * J is the exact Jacobian of the semi-discrete right-hand side at `state`. */
typedef enum {
  LJ_OP_DIAG = 0,
  LJ_OP_ADVDIFF2D = 1,
  LJ_OP_ALLENCAHN2D = 2,
  LJ_OP_BRUSSELATOR2D = 3,
  LJ_OP_BURGERS2D = 4,
  LJ_OP_GRAYSCOTT2D = 5,
  LJ_OP_ADR2D = 6
} lj_op_kind;

typedef struct {
  int32_t kind;          /* lj_op_kind */
  int32_t nx, ny, ncomp; /* grid points per axis, components per point */
  double dx, dy;         /* grid spacing */
  double coef[8];        /* family parameters, see above */
  const double* state;   /* device: linearisation state u (n entries) or the diagonal */
} lj_operator;

/* Options.  Fill with lj_default_options(); NULL means the defaults.
 * The paper leaves every constant open; the defaults are this library's. */
typedef struct {
  double safety;          /* alpha = -safety * lambda_hat (Sec. 2.2 safety factor); 1.25 */
  int32_t power_iters;    /* Jacobian products of the power iteration; 20 */
  int32_t max_points;     /* most Newton terms per expansion, <= LJ_MAX_POINTS; 100 */
  double hump_max;        /* reject when a term exceeds hump_max*||v||*max|f|; 1e4 */
  int32_t max_substeps;   /* largest substep count tried after rejections; 64 */
  int32_t relative_tol;   /* 1: stop when |d_m| ||y_m|| <= tol ||p||; 0: <= tol (Sec. 2.2); 1 */
  double bound;           /* > 0: use as lambda_hat and skip the power iteration; 0 */
  int32_t substeps;       /* > 1: start with this many substeps; 0 */
  uint64_t power_seed;    /* SplitMix64 seed of the power-iteration start vector; 0x5EED */
  const double* pi_start; /* device: explicit start vector (n entries) or NULL */
  int32_t use_proposal;   /* 1: the learned proposal supplies the bound and the substep count
                             (lj_phi_action / lj_phi_vertical); the plain path is the fallback; 0 */
  int32_t reserved;
  const double* bound_device; /* device: when bound == 0 and this is not NULL, the launches read
                             lambda_hat from this address in stream order (no power iteration),
                             e.g. lj_bound_device(ctx) after an lj_step; NULL */
} lj_options;

/* Per-call statistics (host struct).  For a vertical call entry k describes
 * accumulator k.  m_star[k]: Newton terms used when accumulator k converged on
 * the shared basis; when it needed substeps, the Jacobian products of its
 * successful substepped attempt; -1 if it never converged. */
typedef struct {
  int32_t m_star[LJ_MAX_K];
  int32_t substeps[LJ_MAX_K]; /* substep count that produced accumulator k */
  double err_est[LJ_MAX_K];   /* last |d_m| ||y_m|| of accumulator k on the shared basis */
  int32_t iters_total;        /* Jacobian products in Newton recurrences, all attempts */
  int32_t power_iters;        /* Jacobian products in the power iteration */
  int32_t rejections;         /* failed attempts (shared basis or substepped) */
  int32_t converged;          /* 1 if every accumulator converged */
  double bound;               /* lambda_hat used */
  double c, gamma;            /* interval centre and quarter-length (Sec. 2.2) */
  int32_t fallbacks;          /* 1 if the learned proposal failed and the plain path ran */
  int32_t proposal_substeps;  /* substeps the proposal chose (0: no proposal) */
  double proposal_bound;      /* bound the proposal chose (0: no proposal) */
} lj_stats;

/* ---- context --------------------------------------------------------- */

/* Create a context on HIP device `hip_device` (makes it current).  Builds the
 * Leja table and uploads it.  *out is NULL on failure. */
LJ_API int lj_create(lj_context** out, int hip_device);
/* Free the context and its workspace (NULL is a no-op). */
LJ_API void lj_destroy(lj_context* ctx);
/* Text of the last error on ctx (or of the last lj_create failure if ctx is NULL). */
LJ_API const char* lj_last_error(const lj_context* ctx);
/* Fill *opt with the defaults listed in lj_options. */
LJ_API void lj_default_options(lj_options* opt);
/* Library version string. */
LJ_API const char* lj_version(void);

/* ---- building blocks (each is a step of the path, callable on its own) -- */

/* Leja points xi_0..xi_{count-1} on [-2, 2] (Sec. 2.2): xi_0 = 2 and each next
 * point maximises prod_j |x - xi_j|; ties go to the leftmost point.  Host-only
 * (needs no GPU); out is a host array of `count` doubles, 1 <= count <= 101. */
LJ_API int lj_leja_points(double* out, int count);

/* Power-iteration bound (Sec. 2.2): lambda_hat = ||J x_{K-1}|| / ||x_{K-1}||
 * after K = iters products, x_k proportional to J^k x_0, x_0[i] = 0.5 + U_i
 * with U_i the SplitMix64 uniform number i of `seed` (or x_0 = start, a device
 * vector, when start != NULL).  Result written to *bound (host). */
LJ_API int lj_spectral_bound(lj_context* ctx, const lj_operator* J, int iters, uint64_t seed,
                             const double* start, double* bound, void* stream);

/* Newton divided differences (Sec. 2.2) of phi_l(s (c + gamma xi)) at the
 * first npts Leja points, computed on the device in FP64; d (host, npts
 * doubles) receives d_0..d_{npts-1}.  Requires 1 <= npts <= LJ_MAX_POINTS+1. */
LJ_API int lj_divided_differences(lj_context* ctx, int l, double s, double c, double gamma,
                                  int npts, double* d, void* stream);

/* f(u) of the operator family at u (device in, device out).  For LJ_OP_DIAG
 * and LJ_OP_ADVDIFF2D this is J u. */
LJ_API int lj_rhs(lj_context* ctx, const lj_operator* J, const double* u, double* f, void* stream);

/* y = J(J->state) x, the Jacobian product of the operator family (Sec. 2.2
 * applies J matrix-free; device in, device out, n values, y must not alias
 * x). */
LJ_API int lj_jv(lj_context* ctx, const lj_operator* J, const double* x, double* y, void* stream);

/* ---- the action ---------------------------------------------------------- */

/* w = phi_l(h J) v to tolerance tol (Sec. 2.2), 0 <= l <= LJ_MAX_L.
 * stats (host) may be NULL. */
LJ_API int lj_phi_action(lj_context* ctx, const lj_operator* J, const double* v, double* w,
                         int l, double h, double tol, const lj_options* opt, lj_stats* stats,
                         void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * action as lj_phi_action, with the same arguments, results and errors, but
 * the call allocates nothing -- its Newton-basis vectors, partial sums and
 * substep vectors lie in one file-scope device array of
 * LJ_NOALLOC_SCRATCH_BYTES per GPU (held from the first lj_create on that GPU
 * until the process ends; barrier words and status stay in the context,
 * allocated by lj_create).  Needs (2 + (l + 3 if substeps may be taken, i.e.
 * max_substeps > 1 or substeps > 1; l = 0: 2)) vectors of n doubles plus
 * 2 * 48 * CUs doubles of partial sums, each rounded up to 256 bytes; a larger
 * action returns LJ_EINVAL with the sizes in lj_last_error.  use_proposal = 1
 * is rejected (LJ_EINVAL).  Every call on one GPU shares that GPU's array and
 * leaves its last contents there: calls that overlap on one GPU (several
 * streams, threads or contexts) race and must be serialised by the caller. */
#define LJ_NOALLOC_SCRATCH_BYTES (32u << 20)
LJ_API int lj_phi_action_noalloc(lj_context* ctx, const lj_operator* J, const double* v, double* w,
                                 int l, double h, double tol, const lj_options* opt,
                                 lj_stats* stats, void* stream);

/* Deferred synchronisation.  A time integrator needs the results of a step
 * only when it takes the next decision, so steps and actions issued back to
 * back on one stream need not each wait for the device.  Between
 * lj_defer_begin and lj_defer_end, lj_step (built-in operators, no substeps
 * requested, no learned proposal, not LeKry) and lj_phi_action (built-in
 * operators, no substeps requested, no learned proposal) only enqueue their
 * launches and return LJ_OK at once; other such calls return LJ_EINVAL.
 * Their stats are filled by lj_defer_end, so the caller's stats arrays must
 * stay valid until then.  lj_defer_end synchronises `stream` once and reads
 * every deferred expansion's status; if one was rejected (or a launch
 * aborted), that call and every deferred call after it are redone
 * synchronously, in call order, with substeps where needed -- so the inputs
 * of deferred calls (J->state, v) must not be overwritten by later deferred
 * calls.  At most 64 launches (about 8 steps) may be deferred at once.
 * Returns LJ_ENOTCONV if a redone expansion still failed. */
LJ_API int lj_defer_begin(lj_context* ctx);
LJ_API int lj_defer_end(lj_context* ctx, void* stream);
/* Device address where lj_step leaves the spectral bound of its step (its
 * first action's power iteration) for its other actions; valid in stream
 * order until the next lj_step on the context. */
LJ_API const double* lj_bound_device(const lj_context* ctx);

/* Vertical form (Sec. 4): w[k] = phi_{l[k]}(a[k] h J) v for k < K <= LJ_MAX_K,
 * all on one Newton basis; l, a, w are host arrays of K entries (w[k] device
 * pointers, pairwise distinct).  Accumulators that are rejected on the shared
 * basis are redone one by one with substeps. */
LJ_API int lj_phi_vertical(lj_context* ctx, const lj_operator* J, const double* v, int K,
                           const int* l, const double* a, double h, double tol, double* const* w,
                           const lj_options* opt, lj_stats* stats, void* stream);

/* ---- stage driver ---------------------------------------------------------- */

typedef enum {
  LJ_EXPRB2 = 1,     /* u + phi_1(hJ) h f(u) */
  LJ_EXPRB43_U3 = 2, /* third-order u_3 of EXPRB43 (Sec. 5.4 equation) */
  LJ_EXPRB43 = 3,    /* fourth-order u_4 of EXPRB43, err = u_4 - u_3 */
  LJ_EPIRK4S3 = 4,   /* fourth-order u_4 of EPIRK4s3 (Sec. 5.1 equation), err = u_4 - u_3 */
  LJ_EPIRK4S3_LEKRY = 5 /* EPIRK4s3 as "LeKry" (Sec. 5.1 text): the internal stages by Leja (vertical),
                           phi_1(hJ) h f(u) + phi_3(hJ) D_3 of u_3 as one Krylov exponential
                           (lj_phi_combination, default Krylov options), the phi_4 term by Leja */,
  LJ_EPIRK4S3A = 6,  /* fourth-order u_4 of EPIRK4s3A (Sec. 5.2 equation: stages at 1/2 and 2/3),
                        err = u_4 - u_3 */
  LJ_EPIRK4S3A_LEKRY = 7 /* EPIRK4s3A as "LeKry" (Sec. 5.2 text), built like LJ_EPIRK4S3_LEKRY */
} lj_scheme;

/* One step from u = J->state with step size h: u_out (device) receives the
 * scheme's solution and err (device, may be NULL) the embedded difference
 * u_4 - u_3 (zero-filled for schemes without one).  One power iteration per
 * step is shared by all actions.  stats (host) may be NULL; otherwise it is an
 * array of `nstats` entries receiving the statistics of the step's Leja calls
 * in order (EXPRB2: 1, EXPRB43_U3: 3, EXPRB43: 4, EPIRK4S3 and EPIRK4S3A: 3, the LeKry forms: 3 -- the
 * vertical Leja call, the Krylov call, the phi_4 Leja call); *ncalls (may be
 * NULL) receives that count. */
LJ_API int lj_step(lj_context* ctx, int scheme, const lj_operator* J, double h, double tol,
                   double* u_out, double* err, const lj_options* opt, lj_stats* stats,
                   int nstats, int* ncalls, void* stream);

/* ---- Krylov: a linear combination of phi functions (Sec. 2.1) ------------------ */

/* Options of the Krylov evaluation.  Fill with lj_default_krylov_options(). */
typedef struct {
  int32_t krylov_dim;   /* m, the Krylov space dimension per substep, 1..64; 30 */
  int32_t window;       /* orthogonalise against the last `window` basis vectors (incomplete
                           orthogonalisation as in KIOPS); 0: against all; 2 */
  int32_t max_substeps; /* most accepted substeps (10x as many attempts); 1000 */
  int32_t reserved;
} lj_krylov_options;

LJ_API void lj_default_krylov_options(lj_krylov_options* k);

/* w = sum_{j=0}^{p} phi_j(h J) b_j h^j, 0 <= p <= 4, h >= 0: the first block of
 * exp(h A~) [b_0; e_p] with the augmented matrix A~ = [[J, B], [0, K]],
 * B = [b_p, ..., b_1], K the p x p shift (the theorem of Sec. 2.1), advanced
 * in substeps.  Each substep builds an m-dimensional Krylov space of A~ by
 * Arnoldi's process (classical Gram-Schmidt over the orthogonalisation
 * window; a zero new vector ends the space, which is then exact), takes
 * beta V_m exp(tau H_m) e_1, and accepts it when the estimate
 * beta h_{m+1,m} tau |e_m^T phi_1(tau H_m) e_1| is at most tol (tau / h) ||w||;
 * the next substep (or the retry of a rejected one, on the same basis) has
 * size 0.9 tau (allowed / estimate)^{1/(m+1)}, clamped to [tau/10, 2 tau].
 * b is a host array of p + 1 device pointers (NULL entries are zero vectors),
 * w a device vector not aliasing any b[j] or the state.  stats (host, may be
 * NULL): m_star[0] = iters_total = Jacobian products, substeps[0], rejections,
 * converged, err_est[0] = the last accepted estimate.  LJ_ENOTCONV when the
 * substep limit is reached (w then holds the value at the time reached). */
LJ_API int lj_phi_combination(lj_context* ctx, const lj_operator* J, int p, const double* const* b, double h,
                              double tol, double* w, const lj_krylov_options* kopt, lj_stats* stats, void* stream);

/* ---- variable step sizes (Sec. 2.3) ------------------------------------------ */

/* Outcome of lj_integrate (host struct). */
typedef struct {
  int32_t accepted;  /* accepted steps */
  int32_t rejected;  /* rejected attempts (error estimate above tol, or an expansion that failed) */
  int64_t products;  /* Jacobian-vector products of every attempt (power iteration + Newton terms) */
  double t;          /* time reached: T on success */
  double dt_next;    /* the controller's step size after the last accepted step */
} lj_integrate_stats;

/* One attempted step (host struct). */
typedef struct {
  double t;          /* start time of the attempt */
  double dt;         /* its step size */
  double err;        /* e = ||u_4 - u_3||_2 / ||u_4||_2 (infinity if an expansion failed) */
  int32_t products;  /* its Jacobian-vector products */
  int32_t accepted;
} lj_step_record;

/* u(T) of u_t = f(u), u(0) = J->state, with the embedded schemes (LJ_EPIRK4S3,
 * LJ_EPIRK4S3A, their LeKry forms, or LJ_EXPRB43) and the step size control
 * of Sec. 2.3: a step is accepted when
 * e = ||u_4 - u_3||_2 / ||u_4||_2 <= tol; the next size is the smaller of the
 * traditional controller's dt (tol/e)^{1/(p+1)} (p = 3, the embedded order)
 * and the cost controller's, whose cost is the step's Jacobian-vector
 * products per unit time (constants as printed in Sec. 2.3).  A rejected
 * attempt is retried with 0.9 times the traditional size, one whose
 * expansions fail with half the size; the last step ends exactly at T.  Each step linearises
 * at the current state and runs its phi actions to leja_tol.
 * J->state (device, not modified) holds u(0); u_out (device, n values, not
 * aliasing the state) receives u(T).  dt0 > 0 is the first attempt's size.
 * stats (host) may be NULL; log (host, may be NULL) receives the first
 * log_cap attempts.  At most max_attempts attempts (LJ_ENOTCONV beyond, with
 * u_out holding the state reached and stats->t its time). */
LJ_API int lj_integrate(lj_context* ctx, int scheme, const lj_operator* J, double T, double dt0, double tol,
                        double leja_tol, double* u_out, const lj_options* opt, lj_integrate_stats* stats,
                        lj_step_record* log, int log_cap, int max_attempts, void* stream);

/* ---- user operators: matrix-free callbacks ----------------------------------- */

/* Any right-hand side u' = f(u) of n unknowns, given as host callbacks that
 * enqueue device work on `stream` (a hipStream_t) and return 0 on success
 * (nonzero: the library call fails with LJ_EINVAL and the callback's code in
 * lj_last_error).  Pointers passed to a callback are device vectors of n
 * doubles owned by the library or the caller; a callback must not keep them
 * after it returns and must not write any vector other than its output.
 *   rhs(user, x, fx, stream):     fx = f(x)
 *   jv(user, u, x, jx, stream):   jx = J(u) x, the Jacobian of f at u
 * jv may be NULL: the library then forms finite-difference products
 * J(u) x ~ (f(u + eps x) - f(u)) / eps with eps = sqrt(2^-52) (1 + ||u||) / ||x||
 * (Sec. 4 computes the Jacobian product numerically; the step length is the
 * usual choice of Jacobian-free Newton-Krylov methods, Knoll & Keyes 2004),
 * f(u) evaluated once per call; their error is O(eps ||f''||) + O(2^-52 ||f|| / eps),
 * about 1e-8 relative, far above tight tolerances.  rhs may be NULL for the
 * actions when jv is given; the stage driver needs both f and J (R(x) =
 * f(x) - f(u) - J(u)(x - u), Sec. 1).  The Newton recurrence, the stop and
 * rejection tests, the divided differences and the power iteration run as
 * library kernels between the callbacks, with the decisions taken on the
 * device; the host reads them every few steps, so up to 3 products beyond
 * the last needed one may be computed (and discarded).  A callback may call
 * lj_rhs and lj_jv on the same context; any other entry point that takes
 * the context and returns a code fails with LJ_EINVAL when called from a
 * callback (it would reuse the running call's workspace), and lj_destroy must
 * not be called there. */
typedef int (*lj_rhs_fn)(void* user, const double* x, double* fx, void* stream);
typedef int (*lj_jv_fn)(void* user, const double* u, const double* x, double* jx, void* stream);

typedef struct {
  int64_t n;            /* unknowns, >= 1 */
  lj_rhs_fn rhs;        /* f (may be NULL for actions with jv given) */
  lj_jv_fn jv;          /* J(u) x (NULL: finite differences of rhs) */
  void* user;           /* passed to the callbacks */
  const double* state;  /* device: the linearisation state u (n values) */
} lj_user_operator;

/* lj_phi_action / lj_phi_vertical / lj_step for a user operator: the same
 * method, options (except use_proposal, which needs a built-in family) and
 * statistics; power iteration, substepping and the schemes as for the
 * built-in families. */
LJ_API int lj_user_phi_action(lj_context* ctx, const lj_user_operator* J, const double* v, double* w, int l,
                              double h, double tol, const lj_options* opt, lj_stats* stats, void* stream);
LJ_API int lj_user_phi_vertical(lj_context* ctx, const lj_user_operator* J, const double* v, int K,
                                const int* l, const double* a, double h, double tol, double* const* w,
                                const lj_options* opt, lj_stats* stats, void* stream);
LJ_API int lj_user_step(lj_context* ctx, int scheme, const lj_user_operator* J, double h, double tol,
                        double* u_out, double* err, const lj_options* opt, lj_stats* stats, int nstats,
                        int* ncalls, void* stream);
LJ_API int lj_user_phi_combination(lj_context* ctx, const lj_user_operator* J, int p, const double* const* b,
                                   double h, double tol, double* w, const lj_krylov_options* kopt, lj_stats* stats,
                                   void* stream);
/* lj_integrate for a user operator: u(0) = J->state; each attempt linearises
 * at its own state, which the callbacks receive as u (and finite-difference
 * products re-evaluate f there).  Needs rhs. */
LJ_API int lj_user_integrate(lj_context* ctx, int scheme, const lj_user_operator* J, double T, double dt0,
                             double tol, double leja_tol, double* u_out, const lj_options* opt,
                             lj_integrate_stats* stats, lj_step_record* log, int log_cap, int max_attempts,
                             void* stream);

/* ---- batching form --------------------------------------------------------- */

/* Many independent instances in one launch: for each instance i < n and each
 * k < K, w[i*K + k] = phi_{l[k]}(a[k] h[i] J_i) v[i] (the vertical form of
 * Sec. 4 per instance, every step of Sec. 2.2 -- power iteration unless a
 * bound is given, divided differences, Newton recurrence and stop test -- run
 * per instance inside one persistent kernel).  A block of the launch takes one
 * instance at a time from a work queue, so instances of uneven size need no
 * grid-wide synchronisation.
 *
 * lj_batch_create validates every argument, allocates the batch's workspace
 * (two vectors per instance), times the candidate schedules (threads per
 * block, blocks per CU, blocks per instance, order of the queue) on the batch
 * itself and keeps the
 * fastest (the choice is cached in the context per batch shape; the timing
 * runs write the outputs), then captures the launch -- a queue reset and the
 * kernel -- in a HIP graph.  ops: host array of n operators of ONE family;
 * v, w: host arrays of device pointers (n and n*K entries); h: host array of n
 * step sizes; l, a: host arrays of K entries; bounds: host array of n spectral
 * bounds (> 0: used; 0: power iteration for that instance) or NULL; opt: the
 * power-iteration, stop and reject settings (NULL = defaults; opt->bound > 0
 * applies to instances without their own bound).  The buffers must stay valid
 * while the batch exists.
 *
 * An accumulator that the instance's shared Newton basis rejects (Sec. 2.2,
 * last paragraph) is redone inside the same launch with s = 2, 4, ...
 * (up to opt->max_substeps) substeps: phi_1..phi_l at h/s in one recurrence,
 * then s - 1 exponentials and combinations (lj_phi_action's substepping),
 * on the instance's bound; with max_substeps >= 2 the batch holds
 * max(max_k l[k], 1) + 1 extra vectors per instance for it.
 *
 * lj_batch_run replays the graph on `stream` without synchronising.
 * lj_batch_stats synchronises `stream` and reads the per-instance outcome
 * into per_instance (n entries, may be NULL): the shared basis's rejection
 * and every failed substep attempt count as rejections, m_star and substeps
 * describe the accepted attempt, iters_total every Newton step; returns
 * LJ_ENOTCONV if some accumulator failed at every substep count.
 * lj_batch_destroy synchronises the device first. */
typedef struct lj_batch lj_batch;

typedef struct {
  int32_t schedule;      /* index of the schedule in use */
  int32_t block_size;    /* threads per block */
  int32_t blocks;        /* blocks of the persistent launch */
  int32_t largest_first; /* 1: the queue hands out the largest instances first */
  int32_t nschedules;    /* schedules the tuner considered */
  int32_t team;          /* blocks (on one XCD) that share an instance */
  float tune_ms[8];      /* tuned time per schedule in ms (0 when the choice came from the cache) */
  int64_t total_values;  /* sum of the instances' vector lengths */
  double alg_bytes;      /* algorithmic bytes of the run last read by lj_batch_stats */
} lj_batch_info_t;

LJ_API int lj_batch_create(lj_context* ctx, const lj_operator* ops, int n, const double* const* v,
                           const double* h, int K, const int* l, const double* a, double tol,
                           double* const* w, const double* bounds, const lj_options* opt,
                           lj_batch** out);
LJ_API int lj_batch_run(lj_batch* b, void* stream);
LJ_API int lj_batch_stats(lj_batch* b, lj_stats* per_instance, void* stream);
LJ_API int lj_batch_info(const lj_batch* b, lj_batch_info_t* out);
/* Diagnostics of the run last read by lj_batch_stats: for each instance the
 * block that ran it and its start and end on the device wall clock, in
 * microseconds after the earliest start (host arrays of n entries). */
LJ_API int lj_batch_timeline(const lj_batch* b, int* block, double* start_us, double* end_us);
LJ_API void lj_batch_destroy(lj_batch* b);

/* ---- learned proposal ---------------------------------------------------- */

/* Not in the paper: a small network proposes, for an action phi_l(hJ)v, the
 * spectral bound (replacing the power iteration of Sec. 2.2) and the substep
 * count (skipping expansions that would be rejected).  With
 * opt->use_proposal = 1, lj_phi_action / lj_phi_vertical compute on the
 * device the features and the Gershgorin bound G of J (the largest absolute
 * row sum of J at the state: a bound of its spectral radius), run the
 * network and decide there: bound = LJ_PROPOSAL_MARGIN * G * exp(out[0])
 * (the network corrects the Gershgorin bound; out[0] is the largest over
 * the K actions) and s = 2^round(out[1]) substeps (largest over the
 * actions).  The attempt's launch reads both from device memory, so no host
 * round trip separates the decision from the expansion; when s > 1 that
 * launch returns at once and the host, which reads its status anyway, runs
 * the substepped attempt at the bound it read.  Every accumulator that the
 * attempt does not converge (or all of them, when the bound is not usable or
 * s exceeds opt->max_substeps) is redone by the plain path (power iteration,
 * then s = 1, 2, 4, ...), whose stop test remains the judge of the error.
 * lj_stats.proposal_bound / proposal_substeps report the decision.
 *
 * Network: 16 -> 64 -> 64 -> 2, tanh hidden units, FP32; inputs and targets
 * standardised with constants kept in the model.  Model layout (floats):
 * W1 (64x16, row-major), b1 (64), W2 (64x64), b2 (64), W3 (2x64), b3 (2),
 * feature mean (16), feature std (16), target mean (2), target std (2).
 * Targets: ln(bound / G) and log2(accepted substeps).  Features: 16
 * dimensionless numbers of the operator, its state, h and l, among them
 * log10(h G) and log10(G / sigma) with sigma the diffusive rate (the 16
 * values are documented with the CPU reference implementation). */
#define LJ_NFEATURES 16
#define LJ_MLP_NPARAM 5378
#define LJ_MLP_MODEL_FLOATS 5414
#define LJ_PROPOSAL_MARGIN 1.02

/* feats (device, 16 floats) = the features of phi_l(h J) v. */
LJ_API int lj_features(lj_context* ctx, const lj_operator* J, double h, int l, float* feats, void* stream);
/* *bound (host) = the Gershgorin bound of J at its state: the largest sum of
 * absolute entries of a row of the Jacobian the action kernels apply (a
 * boundary cell's own-neighbour entries summed first).  One reduction pass
 * over the state; synchronises the stream.  Built-in families only. */
LJ_API int lj_gershgorin_bound(lj_context* ctx, const lj_operator* J, double* bound, void* stream);
/* One training record of the network for phi_l(h J) v whose plain run used
 * spectral bound `bound` (> 0) and accepted `substeps` (a power of two):
 * feats (device, 16 floats) as lj_features, targets (device, 2 floats) =
 * ln(bound / G), log2(substeps).  Enqueued on the stream, no host wait. */
LJ_API int lj_proposal_record(lj_context* ctx, const lj_operator* J, double h, int l, double bound, int substeps,
                              float* feats, float* targets, void* stream);
/* Glorot-uniform weights from SplitMix64(seed) in parameter order, zero
 * biases, identity standardisation, Adam state cleared. */
LJ_API int lj_mlp_init(lj_context* ctx, uint64_t seed);
/* Trains on n samples (feats: device n x 16, targets: device n x 2) for
 * `epochs` passes in minibatches of `batch` (<= 512) samples, in order, one
 * Adam step (learning rate lr) per minibatch; with fit_normalization = 1 the
 * standardisation constants are first set from the data.  loss_per_epoch
 * (host, epochs floats, may be NULL) receives the mean squared error of each
 * epoch in standardised units.  Synchronises the stream. */
LJ_API int lj_mlp_train(lj_context* ctx, const float* feats, const float* targets, int n, int epochs, int batch,
                        float lr, int fit_normalization, float* loss_per_epoch, void* stream);
/* out (device, n x 2) = network outputs in target units for n feature rows. */
LJ_API int lj_mlp_predict(lj_context* ctx, const float* feats, int n, float* out, void* stream);
/* grad (device, LJ_MLP_NPARAM floats) = gradient of the mean loss over the n
 * samples at the current weights; *loss (host) = that loss.  Synchronises. */
LJ_API int lj_mlp_grad(lj_context* ctx, const float* feats, const float* targets, int n, float* grad, float* loss,
                       void* stream);
/* Model transfer (host arrays of LJ_MLP_MODEL_FLOATS floats) and files. */
LJ_API int lj_mlp_get(lj_context* ctx, float* model);
LJ_API int lj_mlp_set(lj_context* ctx, const float* model);
LJ_API int lj_mlp_save(lj_context* ctx, const char* path);
LJ_API int lj_mlp_load(lj_context* ctx, const char* path);

/* ---- measurement ------------------------------------------------------------ */

/* Attainable HBM bandwidth of the current device (the ceiling the roofline
 * fractions are read against): gbs[0] copy (1 read + 1 write), gbs[1] read
 * only, gbs[2] the access pattern of a Newton step at one accumulator (3 reads
 * + 2 writes), GB/s, best of 5 timed runs, streaming FP64 vectors of `bytes`
 * each (>= 64 MiB, a multiple of 16).  Allocates and frees four such vectors
 * on the current device; synchronises it.  No context needed. */
LJ_API int lj_measure_bandwidth(long long bytes, double* gbs);

/* The same three patterns at a chosen launch shape: `blocks` (1 .. 2^20)
 * blocks of `threads` (64 .. 1024, a multiple of 64) threads, each thread
 * keeping `unroll` (1, 2 or 4) 16-byte accesses per vector in flight, with
 * ordinary (nontemporal = 0) or non-temporal loads and stores (1).
 * lj_measure_bandwidth is this call at 1024 x 256, unroll 1, ordinary
 * accesses.  LJ_EINVAL for arguments out of range (nothing allocated). */
LJ_API int lj_measure_bandwidth_shape(long long bytes, int blocks, int threads, int unroll, int nontemporal,
                                      double* gbs);

/* Kernel timing of the phi-action kernel.  While enabled, the library
 * brackets every launch of that kernel (power iteration + divided differences
 * + Newton recurrence in one persistent launch) with HIP events on the launch
 * stream and accumulates its durations and the work it did. */
typedef struct {
  int64_t launches;          /* action-kernel launches */
  int64_t iterations;        /* Newton iterations run by those launches */
  int64_t point_iters;       /* grid points x Newton iterations */
  int64_t accum_point_iters; /* grid points x sum over iterations of active accumulators */
  int64_t power_point_iters; /* grid points x power-iteration products */
  int64_t tiled_launches;    /* launches that ran a tiled kernel (register-tiled or LDS-tiled: several
                                Newton steps per grid barrier) instead of the streaming one */
  double kernel_ms;          /* summed event-measured duration */
  int64_t aborts;            /* launches whose grid barrier gave up (counted whether or not timing is
                                enabled; each was repeated with a cooperative launch) */
} lj_timing;

/* Test hook: when the environment variable LJ_FORCE_SPIN_LIMIT holds a
 * positive number at lj_create, the first (ordinary) launch of every action
 * bounds each grid-barrier wait by that many polls instead of the default
 * 2^22.  A small value makes those launches give up, so the abort-and-retry
 * path (the cooperative relaunch) runs; results are unchanged.  The same
 * bound applies to the first launch of each one-launch Krylov basis
 * (lj_phi_combination, the LeKry third stage).
 *
 * Test hook: LJ_KRYLOV_PASSES=1 at lj_create makes the Krylov evaluation of
 * built-in families build every basis with four launches per column (the
 * form user operators and windows wider than 2 always use) instead of one
 * launch per basis; results agree up to the order of the dot products'
 * partial sums. */

/* Diagnostics: the reduced norms the last Newton recurrence on ctx decided
 * on.  Row m-1 (m = 1..iterations) holds ||y_m||_2^2 followed by ||p_k||_2^2
 * (k < LJ_MAX_K) after term m, as summed on the device.  out is a host array
 * of rows x (1 + LJ_MAX_K) doubles; returns the number of rows written.
 * Synchronises the device (the trace is read from device memory). */
LJ_API int lj_last_trace(lj_context* ctx, double* out, int rows);

/* Diagnostics: where block 0 of the last action launch spent its time, in
 * microseconds of the device wall clock: us[0] set-up and power iteration,
 * [1] divided differences, [2] Newton steps, [3] publishing partial sums,
 * [4] grid barriers with the reduction of the partial sums, [5] stop
 * decisions, [6] term commits and [7] halo reloads (LDS-tiled kernel).
 * us is a host array of 8 doubles. */
LJ_API int lj_last_profile(lj_context* ctx, double* us);

LJ_API int lj_timing_enable(lj_context* ctx, int enable);
LJ_API int lj_timing_read(lj_context* ctx, lj_timing* out, int reset);

#ifdef __cplusplus
}
#endif

#endif /* LEJA_H */
