/*
 * birk.h -- fast Birkhoff-Chebyshev products and the Birkhoff-preconditioned Krylov
 * solve on AMD Instinct MI355X (gfx950).  C ABI; no C++ or framework types cross it.
 *
 * Method: arXiv 2509.01855, "A Million-Point Fast Trajectory Optimization Solver".
 *
 *   CGL grid        tau_j = -cos(j pi / N), j = 0..N, N_n = N + 1 nodes   (eq:CGLpts)
 *   B^a             [B^a]_ij = B_j^a(tau_i), B_j^a(-1) = 0, dB_j^a/dtau(tau_i) = delta_ij
 *                   (eq:birk-conditions, eq:manyDefs)
 *   FastBV          B^a V = Fasta2v(c^(Fastv2a(V))): DCT-I, coefficient-space
 *                   integration recurrence with the T_{N+1} alias, inverse DCT-I
 *                   (Sec. "An FFT Algorithm for Computing B^a V", eq:c_k=bydef,
 *                   eq:chatk=, App. B, App. C)
 *   FastAX          A chi = chi - B^a (J chi), J = blockdiag_k(J_k)  (eq:Achibetadef)
 *   Preconditioner  P = I - B~^a J, B~^a lower triangular from the CC weights
 *                   (Sec. "Development of a Special Birkhoff-Centric Preconditioner")
 *   FastLinSol      right-preconditioned GMRES on A P^{-1} Upsilon = beta,
 *                   chi = P^{-1} Upsilon (eq:rightPx2, FastLinSol box)
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Plan.     A plan fixes a batch of independent instances i = 0..batch-1, each with its
 *           own node count N_n[i] >= 3 and state count n_x[i] >= 1, the storage
 *           precision, and a HIP stream.  It owns every scratch buffer: those of the
 *           products and the preconditioner are allocated at creation (those calls
 *           allocate nothing); the Krylov workspace (3 restart + 1 vectors in double
 *           plans, 2 restart + 1 in mixed ones, plus a small pinned host staging
 *           buffer) on the first birk_krylov_solve that needs it, kept for later solves.
 * Layout.   Component-major and contiguous: instance i, component r, node k lives at
 *           offset(i) + r * N_n[i] + k, where offset(i) is the prefix sum of
 *           n_x * N_n over earlier instances.  Per-node Jacobians are stored
 *           J[r][c][k] (entry (r, c) contiguous over nodes), i.e. at
 *           joff(i) + (r * n_x[i] + c) * N_n[i] + k with joff the prefix sum of
 *           n_x^2 * N_n; constant Jacobians are J[r][c] at the prefix sum of n_x^2.
 * Memory.   Every array argument is a caller-owned DEVICE pointer on the plan's device,
 *           except where a parameter name ends in _host.  The library never frees or
 *           retains caller memory.
 * Types.    BIRK_F64: vectors are double.  BIRK_F32 and BIRK_F32_REFINE_F64: vectors
 *           passed to birk_apply / birk_apply_T / birk_precond are float.  BIRK_DF32:
 *           every vector element is a double-float pair of floats stored interleaved,
 *           element k at floats 2k (hi) and 2k + 1 (lo), value = hi + lo (about 48
 *           significant bits when |lo| <= ulp(hi) / 2).  Jacobians, beta and chi are
 *           always double.
 * Streams.  Work is enqueued on the plan's stream in call order.  birk_apply,
 *           birk_apply_T and birk_precond are asynchronous; birk_krylov_solve
 *           synchronises the stream before it returns.
 * Errors.   Functions return a birk_status.  Argument, size and precision errors are
 *           found on the host before anything is enqueued, and leave outputs
 *           untouched.  A plan must not be used from two host threads at once.
 */
#ifndef BIRK_H
#define BIRK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BIRK_OK = 0,
  BIRK_ERR_ARG = -1,         /* null pointer, bad enum, inconsistent arguments          */
  BIRK_ERR_SIZE = -2,        /* batch < 1, N_n < 3, n_x < 1, or a size beyond limits    */
  BIRK_ERR_DEVICE = -3,      /* a HIP runtime call failed                               */
  BIRK_ERR_NOMEM = -4,       /* allocation failed (plan creation, first Krylov solve)   */
  BIRK_ERR_SINGULAR = -5,    /* I - w_k J_k / 2 is singular at some node                */
  BIRK_ERR_NOCONV = -6,      /* the solve hit max_iter before rtol                      */
  BIRK_ERR_BREAKDOWN = -7,   /* Krylov breakdown without convergence                    */
  BIRK_ERR_NONFINITE = -8,   /* NaN or Inf met in a norm during the solve               */
  BIRK_ERR_UNSUPPORTED = -9  /* valid request this build does not implement             */
} birk_status;

typedef enum {
  BIRK_F64 = 0,              /* everything in double                                    */
  BIRK_F32 = 1,              /* float storage and arithmetic                            */
  BIRK_F32_REFINE_F64 = 2,   /* float products; solve = float GMRES inside double
                                iterative refinement on the true residual               */
  BIRK_DF32 = 3              /* double-float (hi + lo float pairs) compensated products */
} birk_precision;

typedef enum {
  BIRK_J_CONSTANT = 0,       /* one n_x x n_x Jacobian per instance (LTI)               */
  BIRK_J_PER_NODE = 1        /* one n_x x n_x Jacobian per node                         */
} birk_jac_kind;

typedef struct birk_plan birk_plan;

/* Create a plan.  n_nodes_host[i] = N_n of instance i (N = N_n - 1), n_x_host[i] = its
 * state count; both host arrays of length batch, read during the call only.
 * hip_stream is a hipStream_t (NULL = the device's null stream); the plan is bound to
 * the device current at creation.  Allocates all scratch, the CGL weights and the
 * transform tables (CC weights computed on the device through B^aT e_N).
 * Consecutive instances with the same power-of-two N >= 512 share the launches of the
 * three-pass product; all other instances, whatever their sizes, are covered by one
 * fixed set of launches per product (work lists built here).
 * Errors: BIRK_ERR_ARG (out/arrays NULL, bad precision), BIRK_ERR_SIZE (batch < 1,
 * N_n < 3, n_x < 1, N_n - 1 > 2^22 (2^23 when N_n - 1 is a power of two), total length
 * > 2^31), BIRK_ERR_NOMEM, BIRK_ERR_DEVICE. */
birk_status birk_plan_create(birk_plan** out, int32_t batch, const int64_t* n_nodes_host,
                             const int32_t* n_x_host, birk_precision prec, void* hip_stream);

/* Release a plan and all memory it owns.  NULL is accepted and ignored. */
birk_status birk_plan_destroy(birk_plan* plan);

/* Total vector length sum_i n_x[i] * N_n[i] of the plan (elements, not bytes). */
int64_t birk_plan_length(const birk_plan* plan);

/* Autotuner of the product schedules.  Power-of-two path (N = 2^p >= 512): for each group of
 * same-length components it times B^a (FastBV box) in the plan's precision over a
 * fixed set of tile schedules: both splits 2N = L1 L2 of the two-step DCTs, two or four
 * rows per middle-pass tile, the plain or XCD-grouped tile order, four- or eight-column
 * tiles in the first and last passes where their transforms are 512 or 1024 points long,
 * and the components on one stream or in two or three parts on as many streams (forked
 * from and joined back into the plan's stream by events; same kernels per component).
 * In each of two interleaved rounds a candidate runs once to warm up, then four times
 * between events on the plan's stream, alternating two input/output pairs; its best
 * round counts.  The
 * default schedule stays unless a candidate is more than 2 % faster; the choice stays
 * with the plan for every later product.  The schedule changes only the
 * order of floating-point operations (results stay within the product tolerance).
 * Then the general path (N not a power of two: DCT-I by Bluestein's chirp convolution): for each
 * chirp-convolution length M = 2^m above 4096 in the plan, the two-step FFTs M = M1 M2 are
 * timed (whole products, same rounds) with every split 2^7 <= M1 <= 2^12, 2^6 <= M2 <= 2^12,
 * one length at a time, and the fastest kept (default M1 = 2^ceil(m/2), again kept unless
 * beaten by 2 %); the filter spectra of that length are moved into the new order and the
 * tile lists rebuilt (re-allocated: the only allocations of the call).
 * Inputs are the plan's own scratch vectors.  Blocks until done.
 * report: optional host buffer (NULL, or report_len > 0) that receives a NUL-terminated
 * summary of every timing and choice, truncated to report_len - 1 characters.
 * Errors: BIRK_ERR_ARG (NULL plan), BIRK_ERR_DEVICE. */
birk_status birk_plan_tune(birk_plan* plan, char* report, int64_t report_len);

/* Graph mode of birk_apply / birk_apply_T (enable = 1): the launches of one product are
 * recorded once into a HIP graph per (direction, input pointer, output pointer) and
 * replayed with a single graph launch.  The first call with a given triple runs as usual,
 * the second records and replays, later calls replay; at most eight triples are kept
 * (least recently used dropped).  A replay reads the buffers' current contents, so the
 * same pointers may carry new data; buffers must stay allocated while their triple is in
 * use.  In graph mode birk_krylov_solve also records each chunk of Arnoldi steps it runs
 * (the steps between two host reads of the convergence flags: single steps at first, then
 * 2 and 4 steps on plans shorter than 2^20 elements) the first time a (precision, first
 * step, chunk length, restart, Jacobian pointer and kind, preconditioner, P^{-1} formed on
 * the fly or from the per-node tables cached after the first application) chunk occurs,
 * and replays it afterwards; the Jacobian must stay allocated while such graphs exist
 * (at most 48, all dropped beyond that).  enable = 0
 * (the default) drops every recorded graph.  birk_plan_tune drops them too (they hold the
 * old schedule).  Requires a plan created on a non-null stream.  Other entry points are
 * unaffected.  Errors: BIRK_ERR_ARG, BIRK_ERR_UNSUPPORTED (plan on the legacy null
 * stream). */
birk_status birk_plan_set_graphs(birk_plan* plan, int32_t enable);

/* Copy the Clenshaw-Curtis weights w_B (the last row of B^a, eq:manyDefs and the
 * B~^a section) of instance inst into w_host[0 .. N_n-1] (host memory, double).
 * Synchronises the plan's stream.  Errors: BIRK_ERR_ARG (NULL), BIRK_ERR_SIZE (inst
 * out of range), BIRK_ERR_DEVICE. */
birk_status birk_weights(birk_plan* plan, int32_t inst, double* w_host);

/* out = (I_{n_x} (x) B^a) v for every instance: FastBV on each component
 * (FastBV box; Fastv2a / Fasta2v boxes; eq:c_k=bydef; eq:chatk=).
 * v and out: device arrays of birk_plan_length elements in the plan's storage type;
 * out must not overlap v.  BIRK_DF32 plans run every step (twiddles, butterflies,
 * stencil) in compensated double-float arithmetic; the c^_0 reduction accumulates in
 * double in all precisions.  Errors: BIRK_ERR_ARG (NULL or v == out). */
birk_status birk_apply(birk_plan* plan, const void* v, void* out);

/* out = (I_{n_x} (x) B^aT) g: the exact transpose of FastBV.  The paper does not give
 * it; it is derived from the same factorisation, B^aT = (2/N) E C (S M^T S) C E^{-1}
 * with C the DCT-I of eq:vm=DCT-1, E = diag(1/2, 1, ..., 1, 1/2), S = diag((-1)^k)
 * and M the integration recurrence.  Same arguments and errors as birk_apply. */
birk_status birk_apply_T(birk_plan* plan, const void* g, void* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): transpose = 0 computes birk_apply,
 * transpose = 1 birk_apply_T, with the same kernels, but their work buffers and partial
 * sums live in one fixed array of 128 MiB per device inside the library instead of the
 * plan's buffers.  The call allocates nothing and never uses graph mode.  The array is
 * created with the library's device code on each device it runs on and held until the
 * process ends; its address is resolved once per device (at the first plan creation,
 * else the first call).  Every call on one device shares that device's array, so calls
 * that overlap in time on one device (two streams, two threads, two plans) race: the
 * caller orders them.  Nothing carries over between calls (each kernel writes every
 * workspace element before reading it).  The plan's products need at most 128 MiB of
 * workspace: two complex double work buffers of the plan's transform size (three when
 * an instance has a non-power-of-two N or N < 512) plus the partial sums, about
 * 2 x 16 x N_n n_x / 2 bytes for power-of-two N, e.g. 101 MB for N_n = 2^20 + 1 with
 * n_x = 6.  v, out: as for birk_apply.  Asynchronous on the plan's stream.
 * Errors: BIRK_ERR_ARG (NULL, v == out, transpose not 0 or 1), BIRK_ERR_SIZE (the plan
 * needs more workspace than the array holds; nothing is enqueued), BIRK_ERR_DEVICE. */
birk_status birk_apply_noalloc(birk_plan* plan, const void* v, void* out, int32_t transpose);

/* out = (I_{n_x} (x) B^b) v: the b-form product (eq:xN=Birka+b).  B_j^b is anchored at
 * tau = +1 (B_j^b(1) = 0) with the derivative conditions of eq:birk-conditions, so
 * B^b = B^a - 1 w_B^T.  Computed as the B^a product (FastBV) followed by subtracting,
 * per component, its last node (B^a v)_N = w_B^T v from every node; node N of out is
 * exactly zero.  Same arguments, storage types and errors as birk_apply; graph mode
 * covers the B^a part.  Uses the plan's per-component scratch (allocates nothing). */
birk_status birk_apply_b(birk_plan* plan, const void* v, void* out);

/* out = (I_{n_x} (x) B^bT) g = B^aT g - w_B (1^T g) per component.  The component sums
 * 1^T g accumulate in double over a fixed tile split.  Same arguments and errors as
 * birk_apply_T. */
birk_status birk_apply_bT(birk_plan* plan, const void* g, void* out);

/* The endpoint row of (P_a^N) (eq:Prob-PNa): xb = xa + (I_{n_x} (x) w_B^T) v, one value
 * per component.  xa, xb: device double arrays with one entry per component, instance
 * by instance (instance i, component r at the prefix sum of n_x over earlier instances
 * plus r); xa == xb is allowed; neither may overlap v.  v: plan storage type, plan
 * layout.  The weighted sums accumulate in double over a fixed tile split.
 * Asynchronous; allocates nothing.  Errors: BIRK_ERR_ARG (NULL). */
birk_status birk_endpoint(birk_plan* plan, const double* xa, const void* v, double* xb);

/* Birkhoff preconditioner P = I - (I (x) B~^a) J (B~^a section).
 * inverse = 0: out = P y  (FastBccV applied to J y; an exclusive prefix sum).
 * inverse = 1: out = P^{-1} y by exact block forward substitution,
 *              xi_k = (I - w_k J_k/2)^{-1} (y_k + S_k), S_{k+1} = S_k + w_k J_k xi_k
 *              (FastPinvY box; its printed running-sum update is read as exact
 *              forward substitution), evaluated as a parallel scan of affine maps.
 * inverse = 2: out = P^{-T} y by block backward substitution with P^T (row j:
 *              (I - w_j J_j^T / 2) x_j - w_j J_j^T sum_{k>j} x_k = y_j), evaluated as a
 *              scan of affine maps from the last node down; BIRK_F64 plans only (the
 *              preconditioner of birk_kkt_solve).
 * J: device, double, laid out per jac_kind (see Layout).  y, out: plan storage type
 * (BIRK_DF32 plans: not supported, BIRK_ERR_UNSUPPORTED).  out must not overlap y.
 * Errors: BIRK_ERR_ARG, BIRK_ERR_UNSUPPORTED (n_x > 12, BIRK_DF32, inverse = 2 on plans
 * other than BIRK_F64).  A singular pivot is not reported by this call (it yields
 * non-finite values); birk_krylov_solve checks pivots and returns BIRK_ERR_SINGULAR. */
birk_status birk_precond(birk_plan* plan, birk_jac_kind jac_kind, const double* J,
                         const void* y, void* out, int32_t inverse);

/* out = A x = x - (I (x) B^a)(J x)  (FastAX box, eq:Achibetadef), double in and out
 * regardless of the plan precision (the product runs in double).  Errors as above. */
birk_status birk_fast_ax(birk_plan* plan, birk_jac_kind jac_kind, const double* J,
                         const double* x, double* out);

typedef struct {
  int32_t method;       /* 0 = GMRES; 1 = MINRES on the symmetric KKT form (see
                           birk_kkt_solve; in birk_krylov_solve: H = I, f = 0, g = beta,
                           BIRK_F64 plans, no use_x0)                                  */
  int32_t restart;      /* GMRES restart length m, 1..31 (default 30)                 */
  int32_t max_iter;     /* total inner iterations allowed (default 300)               */
  double rtol;          /* target ||beta - A chi||_2 / ||beta||_2, true residual in
                           double (default 1e-10)                                     */
  int32_t use_precond;  /* 1 = right-precondition with P (default), 0 = none          */
  int32_t use_x0;       /* 1 = start from chi as passed in, 0 = start from zero       */
  int32_t max_refine;   /* BIRK_F32_REFINE_F64: outer refinement steps (default 8)    */
  double inner_rtol;    /* BIRK_F32_REFINE_F64: inner float GMRES tolerance (1e-5)    */
} birk_solve_opts;

/* Fill opts with the defaults listed above. */
void birk_solve_opts_default(birk_solve_opts* opts);

typedef struct {
  int32_t* status;          /* per instance birk_status (host array [batch]) or NULL   */
  int32_t* inner_iters;     /* per instance Krylov iterations, or NULL                 */
  int32_t* outer_iters;     /* per instance refinement steps (1 for plain), or NULL    */
  double* rel_resid_fp64;   /* per instance final ||beta - A chi|| / ||beta||, or NULL */
} birk_solve_info;

/* Solve [I - (I (x) B^a) J] chi = beta for every instance (eq:Newton-ivp) by
 * right-preconditioned, matrix-free GMRES (FastLinSol box), stopping on the true
 * relative residual in double.  BIRK_F64 plans run the Krylov process in double;
 * BIRK_F32_REFINE_F64 plans run float GMRES on A d = r inside double refinement
 * chi += d, r = beta - A chi.  beta, chi: device, double, birk_plan_length elements;
 * chi holds x0 on entry when opts->use_x0, and the best iterate on return, also when
 * the status is an error.  opts may be NULL (defaults); info may be NULL.
 * Returns BIRK_OK when every instance converged, else the first failing instance's
 * status.  The first call (or one with a larger restart) allocates the Krylov workspace
 * (see Plan).  opts->method = 1 solves the same system by MINRES on the symmetric form
 * [[I, A^T], [A, 0]] [chi; lambda] = [0; beta] (birk_kkt_solve with H = I, f = 0; A is
 * square and invertible, so chi solves A chi = beta; the stopping test is then on the
 * residual of the symmetric system).  Errors: BIRK_ERR_ARG, BIRK_ERR_UNSUPPORTED
 * (BIRK_F32 or BIRK_DF32 plans, n_x > 12 with the preconditioner; MINRES also: mixed
 * plans or use_x0), BIRK_ERR_NOMEM, BIRK_ERR_SINGULAR, BIRK_ERR_NOCONV,
 * BIRK_ERR_BREAKDOWN, BIRK_ERR_NONFINITE, BIRK_ERR_DEVICE. */
birk_status birk_krylov_solve(birk_plan* plan, birk_jac_kind jac_kind, const double* J,
                              const double* beta, double* chi, const birk_solve_opts* opts,
                              birk_solve_info* info);

/* Symmetric saddle-point (KKT) form, solved by MINRES.  The paper counts matrix-free KKT
 * solves per SQP iteration (Table 1 and the orbit-transfer results) without stating the
 * system; this library's reading is the equality-constrained quadratic model of one step,
 *     min 1/2 (chi - chi_r)^T H (chi - chi_r)   s.t.   A chi = g,
 * A = I - (I (x) B^a) J (eq:Newton-ivp), H = diag(h) > 0, f = H chi_r, whose optimality
 * conditions are
 *     [ H  A^T ] [ chi    ]   [ f ]
 *     [ A  0   ] [ lambda ] = [ g ].
 * MINRES (Paige-Saunders) on this symmetric indefinite system, preconditioned (use_precond)
 * by M = blockdiag(H, P H^{-1} P^T) with the Birkhoff preconditioner P = I - B~^a J
 * (B~^a section; P^{-T} by backward substitution), restarted on the true residual in
 * double until ||[f; g] - K [chi; lambda]||_2 <= rtol ||[f; g]||_2 per instance.  The
 * Lanczos, rotation and step scalars stay on the device; the host reads them after 2, 2
 * and 4 iterations of a cycle, then once per 8.
 * J: as for birk_krylov_solve.  h: device double, birk_plan_length entries, positive, or
 * NULL for H = I.  f: device double (length as h) or NULL for f = 0.  g: device double.
 * chi (and lam, if not NULL): device double outputs (and the starting point when
 * opts->use_x0 = 1, which needs lam).  BIRK_F64 plans only.  opts: rtol, max_iter (total
 * MINRES iterations), use_precond and use_x0 are used; NULL = defaults.  info: inner =
 * MINRES iterations, outer = restarts, rel_resid = the final relative KKT residual.
 * The first call allocates the KKT workspace (nine pairs of vectors and the scan
 * scratch), kept with the plan.  Synchronous.  Errors: BIRK_ERR_ARG (NULL, overlaps,
 * bad options), BIRK_ERR_UNSUPPORTED (plans other than BIRK_F64, n_x > 12 with the
 * preconditioner), BIRK_ERR_NOMEM, BIRK_ERR_NOCONV, BIRK_ERR_NONFINITE, BIRK_ERR_DEVICE. */
birk_status birk_kkt_solve(birk_plan* plan, birk_jac_kind jac_kind, const double* J, const double* h,
                           const double* f, const double* g, double* chi, double* lam,
                           const birk_solve_opts* opts, birk_solve_info* info);

/* ---- Nonlinear IVP: Newton's method on X - x^a b - B^a f(X) = 0 (eq:X-V=nonlin) ---- */

/* Caller-supplied right-hand side: enqueue on hip_stream (a hipStream_t) the evaluation
 * F = f(X) node by node and, when J is not NULL, the per-node Jacobian df/dx in the
 * BIRK_J_PER_NODE layout.  X, F, J: device, double, plan layout.  Return BIRK_OK, or an
 * error status, which ends the Newton solve with that status. */
typedef birk_status (*birk_rhs_fn)(void* ctx, const double* X, double* F, double* J, void* hip_stream);

typedef enum {
  BIRK_MODEL_TWO_BODY = 0,   /* built in: x = (r, v), dx/dtau = scale (v, -mu r / |r|^3)   */
  BIRK_MODEL_CALLBACK = 1    /* fn(ctx, ...) as above                                      */
} birk_model_kind;

typedef struct {
  int32_t kind;        /* birk_model_kind                                                  */
  double mu;           /* two-body: gravitational parameter                                */
  double scale;        /* two-body: (t_b - t_a) / 2, the time scale of tau in [-1, 1]      */
  birk_rhs_fn fn;      /* callback model                                                   */
  void* ctx;           /* passed to fn                                                     */
} birk_ivp_model;

/* The two-body right-hand side F = scale (v, -mu r / |r|^3) and its Jacobian
 * J = scale [[0, I], [mu (3 r r^T / |r|^2 - I) / |r|^3, 0]] at every node of every
 * instance (all instances need n_x = 6: components r_x, r_y, r_z, v_x, v_y, v_z).
 * X, F, J: device, double; F or J may be NULL (not both); no two may be the same array.
 * Asynchronous.  Errors: BIRK_ERR_ARG, BIRK_ERR_UNSUPPORTED (an instance with n_x != 6). */
birk_status birk_two_body(birk_plan* plan, double mu, double scale, const double* X, double* F, double* J);

typedef struct {
  int32_t max_newton;        /* Newton steps allowed (default 30)                           */
  double tol;                /* stop when ||G||_2 <= tol ||X||_2 per instance (1e-13)       */
  int32_t line_search;       /* 1 = Armijo backtracking on ||G||_2 (default), 0 = full steps */
  birk_solve_opts linear;    /* the Newton systems (birk_krylov_solve; use_x0 is ignored)    */
} birk_newton_opts;

/* Fill opts with the defaults listed above (linear: birk_solve_opts_default). */
void birk_newton_opts_default(birk_newton_opts* opts);

typedef struct {
  int32_t* status;        /* per instance birk_status, or NULL                             */
  int32_t* newton_iters;  /* per instance Newton steps taken, or NULL                      */
  int32_t* linear_iters;  /* per instance Krylov iterations over all steps, or NULL        */
  double* rel_resid;      /* per instance final ||G||_2 / ||X||_2, or NULL                 */
} birk_newton_info;

/* Solve the a-form IVP X - x^a b - (I (x) B^a) f(X) = 0 (eq:X-V=nonlin, b = ones) for
 * every instance by Newton's method: each step solves [I - (I (x) B^a) df(X)] D = -G(X)
 * (eq:Newton-ivp) with birk_krylov_solve (right-preconditioned GMRES, per-node Jacobian)
 * and, with line_search, halves the step until ||G(X + l D)|| <= (1 - 1e-4 l) ||G(X)||
 * (the paper gives the Newton system only; this globalisation is the library's).  A step
 * below 2^-12 fails the instance with BIRK_ERR_NOCONV and keeps its X.
 * xa: device, double, one entry per component (the layout of birk_endpoint); X: device,
 * double, plan layout, the starting guess on entry and the last iterate on return.
 * Plans of precision BIRK_F64 (or BIRK_F32_REFINE_F64, whose linear solves then use
 * refinement); the product in G(X) is always double.  Synchronous.  The first call
 * allocates the Newton workspace (6 vectors plus the per-node Jacobians), kept with the
 * plan.  Returns BIRK_OK when every instance converged, else the first failing status.
 * Errors: BIRK_ERR_ARG, BIRK_ERR_UNSUPPORTED (two-body model with n_x != 6, BIRK_F32 or
 * BIRK_DF32 plans, n_x > 12 with the preconditioner), BIRK_ERR_NOMEM,
 * BIRK_ERR_SINGULAR, BIRK_ERR_NOCONV, BIRK_ERR_NONFINITE, BIRK_ERR_DEVICE, or the
 * callback's own status. */
birk_status birk_newton_ivp(birk_plan* plan, const birk_ivp_model* model, const double* xa, double* X,
                            const birk_newton_opts* opts, birk_newton_info* info);

/* Static, NUL-terminated description of a status code (never NULL). */
const char* birk_status_string(birk_status status);

#ifdef __cplusplus
}
#endif

#endif /* BIRK_H */
