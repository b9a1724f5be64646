/*
 * ppals.h -- C ABI of the MI355X pairwise-perturbation CP-ALS library.
 *
 * The library computes CP decompositions of dense tensors with alternating
 * least squares (ALS, Algorithm 1 of Ma & Solomonik, "Accelerating Alternating
 * Least Squares for Tensor Decomposition by Pairwise Perturbation") and with
 * pairwise perturbation (PP-CP-ALS, Algorithm 3).  Notation follows the paper:
 * X is an order-N tensor of size s_1 x .. x s_N, A^(n) are s_n x R factor
 * matrices, S^(n) = A^(n)T A^(n), Gamma^(n) is the Hadamard product of the
 * other modes' S, M^(n) is the MTTKRP right-hand side.
 *
 * Layout conventions (all row-major):
 *   X        s_1 x .. x s_N, last mode fastest, FP64 or FP32 elements.
 *   X_bf16   same shape, bfloat16 bit patterns (uint16), only for the BF16
 *            first-level tier; produced by ppals_cast_bf16.
 *   A[n]     s_n x R doubles (k fastest).  The factors are always FP64; the
 *            FP32 / BF16 tiers convert them when they enter a contraction.
 *   S        N consecutive R x R doubles, S[n] = A[n]^T A[n].
 *
 * Ownership: every device buffer (X, X_bf16, A[n], S, ws, records) is
 * allocated and freed by the caller.  The entry points that take a stream
 * never allocate device memory.  Pointer arrays (A) are host arrays of device
 * pointers.  A plan is a host object owned by the caller
 * (ppals_plan_create / ppals_plan_destroy).
 *
 * Errors: argument errors are detected on the host before anything is
 * enqueued and return PPALS_E_ARG / PPALS_E_UNSUPPORTED; a failed launch
 * returns PPALS_E_HIP.  ppals_last_error() returns a thread-local message for
 * the last failure.  Numerical conditions found on the device (a Cholesky
 * factorisation that needed the diagonal shift) are reported in the sweep
 * record, because the calls are asynchronous.
 *
 * Streams: every call that takes a hipStream_t only enqueues work on it and
 * returns without synchronising, except ppals_run, which drives a whole
 * decomposition and synchronises once per sweep to read the sweep record.
 */
#ifndef PPALS_H
#define PPALS_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PPALS_OK = 0,
  PPALS_E_ARG = -1,          /* invalid argument (null pointer, bad size)        */
  PPALS_E_UNSUPPORTED = -2,  /* valid but not supported (order, rank, dtype mix)  */
  PPALS_E_HIP = -3,          /* a HIP runtime call or launch failed               */
  PPALS_E_WORKSPACE = -4,    /* workspace pointer null or not 256-byte aligned     */
  PPALS_E_STATE = -5         /* pp_sweep before pp_build_operators                 */
} ppals_status;

typedef enum { PPALS_FP64 = 0, PPALS_FP32 = 1, PPALS_BF16 = 2 } ppals_dtype;

typedef enum { PPALS_SWEEP_ALS = 0, PPALS_SWEEP_PP_INIT = 1, PPALS_SWEEP_PP_APPROX = 2 } ppals_sweep_kind;

#define PPALS_MAX_ORDER 8
#define PPALS_MAX_RANK 128

/* Problem description.  Supported: 3 <= order <= 8, 1 <= rank <= 128,
 * dims >= 1, 0 < step_size <= 1 (0 is read as 1).  Precision tiers (tensor_dtype,
 * level1_dtype):
 *   (FP64, FP64)  every contraction in FP64;
 *   (FP32, FP32)  contractions in FP32 with FP32 MFMA accumulation;
 *   (FP32, BF16)  first-level contractions take bfloat16 inputs (X_bf16 and
 *                 bf16-rounded factors) with FP32 accumulation, the rest FP32.
 * Gram matrices, Hadamard products, Cholesky solves, norms and the fit are
 * FP64 in every tier.  use_second_order selects the V^(n,i,j) correction of
 * the general PP update (Section 3.2.1). */
typedef struct {
  int32_t order;
  int32_t rank;
  int64_t dims[PPALS_MAX_ORDER];
  int32_t tensor_dtype;
  int32_t level1_dtype;
  int32_t use_second_order;
  /* Operator build (Section 3.2.3, cost and memory footprint): the number l of leading
   * levels of the PP dimension tree to combine.  0 or 1 runs the tree, whose first level
   * keeps intermediates of O(s^(N-1) R) elements; l >= 2 computes the nodes of tree level
   * l + 1 straight from X, contracting l modes at once with their Khatri-Rao product (one
   * pass over X per node), and only the later levels from parents; l >= N - 2 computes
   * every operator M_p^(i,j) from X (no intermediates).  -1 lets the plan choose l from a
   * roofline model of the build (ppals_plan_describe reports it).  l >= 2 needs the FP64
   * or FP32 first level and contracted extents below 2^31 - 64.  Order 3 always runs
   * the tree (its first level holds the operators). */
  int32_t pp_build_levels;
  /* Update step size lambda of the step-size variant of ALS (Section 5.1): every factor
   * update of the ALS and PP sweeps is A_new = (1 - lambda) A + lambda M Gamma^-1; the
   * record's gradient stays the one at A before the update, (A - M Gamma^-1) Gamma.
   * 1 (or 0) is Algorithm 1.  gram_solve always takes the full step. */
  double step_size;
} ppals_desc;

/* Per-sweep record, written on the device at the end of every sweep call.
 *   fit_est        1 - sqrt(max(0, ||X||^2 - 2<M^(N), A^(N)> + 1^T(Gamma^(N)*S^(N))1)) / ||X||
 *                  with M^(N) the right-hand side used for the last mode
 *                  (approximate in PP sweeps);
 *   grad_norm[n]   ||G^(n)||_F, G^(n) = (A_old - A_new) Gamma^(n) (Algorithm 1);
 *   rel_change[n]  ||dA^(n)||_F / ||A^(n)||_F with dA the change over the sweep
 *                  (ALS) or since the operator build (PP), Algorithm 3;
 *   chol_status[n] 0: clean Cholesky; 1: factorised Gamma + delta I with
 *                  delta = R 2^-52 max(diag Gamma); 2: failed after the shift
 *                  (A^(n) left unchanged).
 *   chol_pivot[n]  0-based index of the first pivot of the unshifted factorisation of
 *                  Gamma^(n) that was not positive and finite (Gamma^(n) is not SPD at
 *                  that leading block), -1 if the factorisation went through.
 *   nonfinite[n]   1 if the new A^(n), its gradient or the fit term of mode n holds a
 *                  value that is not finite (NaN or infinity), else 0.
 * The ctrl_* fields are written by ppals_run when a learned controller is
 * attached (ppals_set_controller); otherwise ppals_run sets them to
 * ctrl_pred = NaN, ctrl_true_err = -1, ctrl_leave = -1, ctrl_fallback = 0:
 *   ctrl_pred      the network's prediction of log10 of the PP right-hand-side
 *                  error after this PP sweep;
 *   ctrl_true_err  the measured error max_n ||M~^(n) - M^(n)||_F / ||M^(n)||_F
 *                  when this sweep was a periodic check, else -1;
 *   ctrl_leave     1 if the prediction asked to leave the PP phase;
 *   ctrl_fallback  1 once a check disabled the controller for the run. */
typedef struct {
  double fit_est;
  double grad_norm[PPALS_MAX_ORDER];
  double rel_change[PPALS_MAX_ORDER];
  int32_t chol_status[PPALS_MAX_ORDER];
  int32_t sweep_kind;
  int32_t pad;
  double ctrl_pred;
  double ctrl_true_err;
  int32_t ctrl_leave;
  int32_t ctrl_fallback;
  int32_t chol_pivot[PPALS_MAX_ORDER];
  int32_t nonfinite[PPALS_MAX_ORDER];
} ppals_sweep_record;

typedef struct ppals_plan ppals_plan;

/* Thread-local text of the last error (never NULL). */
const char* ppals_last_error(void);

/* Host only; allocates the host plan (schedules of the dimension trees and
 * the workspace layout).  No device memory is touched. */
ppals_status ppals_plan_create(const ppals_desc* desc, ppals_plan** out);
void ppals_plan_destroy(ppals_plan* plan);

/* Bytes of device workspace the plan needs (intermediates of the dimension
 * trees, the C(N,2) pairwise perturbation operators, staging and scratch).
 * Every workspace argument of this library must be 256-byte aligned (device
 * allocations are); a NULL or misaligned one fails with PPALS_E_WORKSPACE. */
size_t ppals_workspace_bytes(const ppals_plan* plan);

/* Host only: writes a JSON description of the schedules (contractions of the
 * ALS dimension tree of Section 2.5 and of the PP operator tree of Section
 * 3.2.3) with their flop counts.  Returns PPALS_E_ARG if len is too small. */
ppals_status ppals_plan_describe(const ppals_plan* plan, char* buf, size_t len);

/* One CP-ALS sweep (Algorithm 1, loop body) over n = 1..N with the binary
 * dimension-tree MTTKRP (Section 2.5).  A and S are updated in place; rec
 * (device pointer) receives the sweep record with sweep_kind = ALS and
 * rel_change = per-sweep change.  normX2 = ||X||_F^2 (see ppals_tensor_norm2).
 * X_bf16 is required in the BF16 tier and ignored otherwise. */
ppals_status cp_als_sweep(ppals_plan* plan, const void* X, const void* X_bf16,
                          double* const* A, double* S, double normX2, void* ws,
                          ppals_sweep_record* rec, hipStream_t stream);

/* Pairwise perturbation initialisation (Algorithm 3): A_p := A, dA := 0, and
 * the operators M_p^(i,j) (i < j) and M_p^(n) are built with the PP dimension
 * tree of Section 3.2.3.  The operators live in ws. */
ppals_status pp_build_operators(ppals_plan* plan, const void* X, const void* X_bf16,
                                double* const* A, void* ws, hipStream_t stream);

/* One approximated sweep (Algorithm 3, inner loop): for n = 1..N the
 * right-hand side is the general PP update
 *   M~^(n) = M_p^(n) + sum_{i!=n} M_p^(i,n) x_i dA^(i) + A^(n) W^(n),
 *   W^(n)  = sum over unordered pairs {i,j} of modes != n of
 *            (A^(i)T dA^(i)) * (A^(j)T dA^(j)) * Hadamard_{k!=i,j,n} S^(k)
 * (the last term only if use_second_order), followed by the same normal
 * equation solve as ALS and dA^(n) = A^(n) - A_p^(n).  rec->sweep_kind is
 * PP_INIT for the first sweep after a build, PP_APPROX afterwards.
 * Returns PPALS_E_STATE if no operators were built with this plan. */
ppals_status pp_sweep(ppals_plan* plan, double* const* A, double* S, double normX2,
                      void* ws, ppals_sweep_record* rec, hipStream_t stream);

/* Standalone normal-equation solve (Algorithm 1, the factor update and its
 * gradient):
 * A_new Gamma = M for `rows` right-hand-side rows, Gamma = L L^T (Cholesky,
 * with the diagonal-shift retry), then grad_norm = ||(A_old - A_new) Gamma||_F
 * and A_inout := A_new.  Gamma: R x R doubles; M: rows x R in m_dtype (FP64
 * or FP32); A_inout: rows x R doubles.  grad_norm_out and chol_status_out are
 * device pointers (one double, one int32).  ws must hold
 * ppals_gram_solve_workspace_bytes(R, rows) bytes.
 * *chol_status_out (written on the device):
 *   bits 0-1   0 clean, 1 factorised Gamma + delta I (delta = R 2^-52 max diag Gamma),
 *              2 failed after the shift (A_inout left unchanged);
 *   bit 4      set when the new factor or the gradient holds a value that is not finite;
 *   bits 8-30  one plus the 0-based index of the first pivot of the unshifted
 *              factorisation that was not positive and finite (0 if none), i.e. the
 *              order of the first leading block of Gamma that is not positive definite. */
size_t ppals_gram_solve_workspace_bytes(int32_t R, int64_t rows);
ppals_status gram_solve(int32_t R, int64_t rows, const double* Gamma, const void* M,
                        int32_t m_dtype, double* A_inout, double* grad_norm_out,
                        int32_t* chol_status_out, void* ws, hipStream_t stream);

/* gram_solve without a workspace argument, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as gram_solve; the scratch (L, the
 * per-row partial sums and the status word) is a fixed array inside the library, one
 * copy per GPU, held until the process ends: PPALS_MAX_RANK^2 doubles plus 4 doubles
 * per row for up to PPALS_GRAM_SOLVE_NOALLOC_MAX_ROWS rows (about 2.1 MiB).
 *   rows > PPALS_GRAM_SOLVE_NOALLOC_MAX_ROWS  -> PPALS_E_UNSUPPORTED (nothing enqueued).
 * The call allocates nothing (no hipMalloc, hipFree or allocating library routine); the
 * first call on a device looks the array's address up once (hipGetSymbolAddress).
 * Every call on one GPU shares that GPU's array and leaves its last contents there
 * (no entry of it needs to start at zero): calls that overlap on one GPU, on different
 * streams or from different threads, race and must be serialised by the caller. */
#define PPALS_GRAM_SOLVE_NOALLOC_MAX_ROWS 65536
ppals_status gram_solve_noalloc(int32_t R, int64_t rows, const double* Gamma, const void* M,
                                int32_t m_dtype, double* A_inout, double* grad_norm_out,
                                int32_t* chol_status_out, hipStream_t stream);

/* ||X||_F^2 accumulated in FP64 into *out (device double).  dtype FP64/FP32.
 * ws must hold ppals_norm2_workspace_bytes() bytes. */
size_t ppals_norm2_workspace_bytes(void);
ppals_status ppals_tensor_norm2(const void* X, int32_t dtype, int64_t count, double* out,
                                void* ws, hipStream_t stream);

/* Round FP32 values to bfloat16 (nearest, ties to even); out holds uint16
 * bit patterns.  Used to make X_bf16 for the BF16 first-level tier. */
ppals_status ppals_cast_bf16(const float* in, uint16_t* out, int64_t count, hipStream_t stream);

/* MTTKRP of one mode through the library's contraction kernels (the ALS
 * dimension tree up to that mode, without any solve): out = X_(n) times the
 * Khatri-Rao product of the other factors (Section 2.3), s_n x R doubles.
 * 0 <= mode < N. */
ppals_status ppals_mttkrp(ppals_plan* plan, const void* X, const void* X_bf16,
                          double* const* A, int32_t mode, void* out, void* ws,
                          hipStream_t stream);

/* First-level contraction alone (Section 2.5): contracts X with the factors
 * of the modes in the contiguous bit range `contract_mask` (a single mode, or
 * a leading or trailing block of modes, whose Khatri-Rao product is formed on
 * the device), producing M^(kept modes) with the kept modes in increasing
 * order and k last, in the bulk dtype. */
ppals_status ppals_level1(ppals_plan* plan, const void* X, const void* X_bf16,
                          double* const* A, uint32_t contract_mask, void* out, void* ws,
                          hipStream_t stream);

/* Approximated right-hand side M~^(n) for the current factors A (after
 * pp_build_operators): recomputes dA^(i) = A^(i) - A_p^(i) and
 * A^(i)T dA^(i) for all modes, then evaluates the general PP update for mode
 * n into out (s_n x R doubles).  S holds the current Grams. */
ppals_status ppals_pp_rhs(ppals_plan* plan, double* const* A, const double* S, int32_t mode,
                          double* out, void* ws, hipStream_t stream);

/* Read back a pairwise perturbation operator M_p^(i,j), i < j (0-based), as
 * s_i x s_j x R values of the bulk dtype (device-to-device copy). */
ppals_status ppals_get_operator(ppals_plan* plan, const void* ws, int32_t i, int32_t j,
                                void* out, hipStream_t stream);

/* Exact residual ||X - [[A]]||_F^2 (Section 5 fit metric), FP64 accumulation,
 * written to *out (device double).  Costs about one first-level contraction. */
ppals_status ppals_exact_residual2(ppals_plan* plan, const void* X, double* const* A,
                                   double* out, void* ws, hipStream_t stream);

/* Whole decomposition driven natively (Algorithm 3 control, or Algorithm 1
 * when eps <= 0): starts from the factors in A (S is recomputed), runs at most
 * max_sweeps sweeps and stops early when sum_n ||G^(n)||_F <= delta ||X||_F
 * (delta <= 0 disables this).  After every sweep the record is copied to
 * host_records[i] (host memory, max_sweeps entries) and, if sweep_ms is not
 * NULL, the sweep's device time to sweep_ms[i].  *n_done = sweeps run.  The
 * switching test is strict: PP is entered (operators rebuilt) after a sweep
 * whose rel_change is below eps for every mode, and PP sweeps continue while
 * that holds.  replay (host, may be NULL) forces the sweep kinds instead. */
ppals_status ppals_run(ppals_plan* plan, const void* X, const void* X_bf16, double* const* A,
                       double* S, double normX2, void* ws, ppals_sweep_record* rec_dev,
                       double eps, double delta, int32_t max_sweeps, const int32_t* replay,
                       ppals_sweep_record* host_records, float* sweep_ms, int32_t* n_done,
                       hipStream_t stream);

/* ---- Learned PP controller ------------------------------------------------
 * Algorithm 3 leaves the PP phase when some ||dA^(i)|| / ||A^(i)|| reaches eps;
 * other switching schemes are named as future work (Section 6).  The library
 * provides a small network that predicts log10 of the PP right-hand-side error
 * e = max_n ||M~^(n) - M^(n)||_F / ||M^(n)||_F from the state of the iteration,
 * its training kernels, and a driver mode that leaves PP when the prediction
 * reaches log10(tau).
 *
 * Network: d = order + 2 inputs, `hidden` tanh units, one linear output, FP32:
 *   h = tanh(W1 x + b1), y = W2 . h + b2.
 * Parameters: a device array of P = hidden*d + 2*hidden + 1 floats laid out as
 * [W1 (hidden x d, row-major), b1 (hidden), W2 (hidden), b2].
 * Inputs x for a PP iterate: log10(rel_change_i + 1e-12) for each mode,
 * log1p(sweep index), -log10(1 - fit_est + 1e-16) (sweep index = 0-based index
 * of the sweep just finished).  Limits: 1 <= d <= 16, 1 <= hidden <= 1024. */

/* Forward pass for B samples: X is B x d (row-major, device), y (B floats,
 * device) receives the outputs; hcache (B x hidden floats, device, may be
 * NULL) receives the hidden activations for ppals_mlp_backward. */
ppals_status ppals_mlp_forward(const float* params, int32_t d, int32_t hidden, const float* X,
                               int64_t B, float* y, float* hcache, hipStream_t stream);

/* Gradient of L = (1/B) sum_b (y_b - t_b)^2 with respect to the parameters
 * (same layout as params) from the forward pass's y and hcache; t: B targets.
 * loss (one float, device, may be NULL) receives L.  Reductions run in a fixed
 * order (deterministic). */
ppals_status ppals_mlp_backward(const float* params, int32_t d, int32_t hidden, const float* X,
                                const float* hcache, const float* y, const float* t, int64_t B,
                                float* grad, float* loss, hipStream_t stream);

/* One Adam step (Kingma & Ba, 2015) on P parameters, in place: with the step
 * count `step` >= 1, m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * p -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps).
 * m and v (P floats each) start at zero. */
ppals_status ppals_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t P,
                            int32_t step, float lr, float beta1, float beta2, float eps,
                            hipStream_t stream);

/* Measured PP right-hand-side error at the current iterate (the controller's
 * label): e = max_n ||M~^(n) - M^(n)||_F / ||M^(n)||_F, where M~^(n) is the
 * general PP update (Section 3.2.1) from the operators of the last
 * pp_build_operators and the current factors, and M^(n) the exact MTTKRP of
 * the current factors (dimension tree, no solves).  err: one device double.
 * Returns PPALS_E_STATE if no operators were built with this plan. */
ppals_status ppals_pp_rhs_error(ppals_plan* plan, const void* X, const void* X_bf16,
                                double* const* A, const double* S, void* ws, double* err,
                                hipStream_t stream);

typedef struct {
  const float* params;      /* device parameters, d = order + 2 inputs        */
  int32_t hidden;           /* hidden units (1..1024)                          */
  int32_t check_period;     /* every check_period-th PP sweep of a run the true
                               error is measured (0: never)                   */
  double log10_tau;         /* leave PP when the prediction >= log10_tau       */
  double rho_cap;           /* also leave PP when some rel_change >= rho_cap    */
  double fallback_factor;   /* a measured error > fallback_factor * tau turns the
                               controller off for the rest of the run (the fixed
                               threshold rule of Algorithm 3 then decides)     */
} ppals_controller;

/* Attach (ctl != NULL, copied) or detach (NULL) a learned controller for
 * ppals_run.  Entering the PP phase always follows the threshold rule; with a
 * controller attached, staying in it follows the network (and rho_cap) until a
 * periodic check falls back.  The parameters must stay valid while attached. */
ppals_status ppals_set_controller(ppals_plan* plan, const ppals_controller* ctl);

/* ---- Batched execution ------------------------------------------------------
 * Many independent order-3 decompositions of uneven size and rank advanced
 * together: every problem runs PP-CP-ALS (Algorithm 3 with the threshold rule,
 * dimension-tree ALS sweeps of Section 2.5, PP sweeps of Section 3.2.1) with its
 * own state machine on the device, so one batched sweep is a fixed sequence of
 * grouped kernels that a HIP graph can capture once and replay.  Tensors are
 * FP32, factors FP64; Grams, Cholesky solves, norms and fits FP64.  A problem
 * stops when |fit - previous fit| < tol or after max_sweeps sweeps.
 * Limits: 1 <= dims <= 256, 1 <= rank <= 64. */
typedef struct ppals_batch ppals_batch;
typedef struct {
  int32_t dims[3];
  int32_t rank;
} ppals_batch_problem;

typedef struct {
  int32_t sweeps;            /* sweeps run                                        */
  int32_t converged_sweep;   /* sweep count at convergence, -1 if not converged    */
  int32_t n_als, n_pp_init, n_pp_approx;
  int32_t done;
  int32_t chol_status[3];    /* of the last sweep, as in ppals_sweep_record         */
  int32_t pad;
  double fit;                /* fit estimate after the last sweep (identity form)   */
  double normX2;
  double rel_change[3];
  double time_to_converge_ms;/* device clock, first batched sweep to convergence
                                (-1 if not converged)                              */
} ppals_batch_result;

/* Host only: copies the problem list and lays out the workspace.  Every problem
 * gets its own regions for the three pairwise operators, M_p, A_p, dA, Grams,
 * right-hand side and sweep-kind log. */
ppals_status ppals_batch_create(const ppals_batch_problem* problems, int32_t count,
                                int32_t max_sweeps, ppals_batch** out);
void ppals_batch_destroy(ppals_batch* batch);
size_t ppals_batch_workspace_bytes(const ppals_batch* batch);

/* Binds the caller's tensors X[p] (device, FP32, row-major) and factors
 * A[3p + n] (device, FP64, dims[n] x rank, updated in place) and the workspace,
 * sets eps (PP threshold), tol and the second-order switch, and initialises every
 * problem (||X||^2, Grams, state).  Synchronises the stream. */
ppals_status ppals_batch_bind(ppals_batch* batch, const float* const* X, double* const* A,
                              void* ws, double eps, double tol, int32_t second_order,
                              hipStream_t stream);

/* Measures the first-level contraction kernel's tile variants (64 or 128 output
 * rows) on the bound problems of every (rank, size) bucket and keeps the faster
 * one per bucket (ppals_batch_describe reports the table).  Call after bind,
 * before the run; it overwrites operator scratch only. */
ppals_status ppals_batch_autotune(ppals_batch* batch, void* ws, int32_t reps, hipStream_t stream);

/* Enqueues one batched sweep (no host synchronisation; graph-capturable). */
ppals_status ppals_batch_sweep(ppals_batch* batch, void* ws, hipStream_t stream);

/* Enqueues `sweeps` batched sweeps; with use_graph the sweep is captured once in
 * a HIP graph (kept until the binding or tuning changes) and replayed. */
ppals_status ppals_batch_run(ppals_batch* batch, void* ws, int32_t sweeps, int32_t use_graph,
                             hipStream_t stream);

/* Per-problem results (host array of count entries); synchronises the stream. */
ppals_status ppals_batch_results(ppals_batch* batch, const void* ws, ppals_batch_result* out,
                                 hipStream_t stream);

/* Sweep kinds (PPALS_SWEEP_* + 1; 0 = none) of every problem, count x max_sweeps
 * bytes into a host buffer; synchronises the stream. */
ppals_status ppals_batch_kind_log(ppals_batch* batch, const void* ws, uint8_t* out,
                                  hipStream_t stream);

/* JSON text: sizes, workspace bytes and the autotuner's per-bucket table. */
ppals_status ppals_batch_describe(const ppals_batch* batch, char* buf, size_t len);

/* Optional timing of kernel classes with HIP events recorded on the launch
 * stream around each launch (level-1 GEMM, PP correction TTV, dimension-tree
 * TTV, PP combine, per-mode FP64 tail, operand preparation, PP-tree TTV,
 * split reduction).  Statistics accumulate while enabled and are resolved at
 * the per-sweep synchronisation of ppals_run or by ppals_get_profile (which
 * waits for the recorded events).  flops and bytes are the algorithmic work
 * of the timed launches (compulsory HBM traffic: inputs read once, outputs
 * written once). */
#define PPALS_PROF_CLASSES 8
typedef struct {
  char name[32];
  int64_t launches;
  double total_ms;
  double flops;
  double bytes;
} ppals_kernel_stat;
ppals_status ppals_set_profiling(ppals_plan* plan, int32_t enable);
ppals_status ppals_get_profile(ppals_plan* plan, ppals_kernel_stat* out, int32_t max_entries,
                               int32_t* n_out, int32_t reset);

/* ---------------------------------------------------------------------------
 * Tucker decomposition of an order-N tensor (3 <= N <= 8) by ALS (HOOI, Algorithm 2) and
 * by pairwise perturbation (PP-Tucker-ALS, Algorithm 4 with the first-order approximation
 * of Section 3.2.2), FP64 throughout.
 *
 *   X       s_1 x .. x s_N doubles, row-major (device).
 *   A[n]    s_n x R doubles, orthonormal columns (device), updated in place.
 *   G       the core, R^N doubles, index order (r_1, .., r_N) (device).
 *   ws      caller-allocated workspace of tucker_workspace_bytes() bytes, 256-byte
 *           aligned; it holds the PP operators between tucker_pp_build and later
 *           tucker_pp_sweep calls.
 * The TTMc Y^(n) = X x_{i != n} A^(i)T (Section 2.4) is stored as s_n x R^(N-1) doubles:
 * x_n first, then the rank indices of the other modes in increasing mode order.
 *
 * HOOI sweep: Y^(1) from X; then the prefix P_n = X x_1 A^(1)T .. x_(n-1) A^(n-1)T, with
 * the factors already updated in the sweep, grows by one contraction per mode and gives
 * Y^(n) with the later modes contracted: two passes over X per sweep.  Operator build:
 * Y_p^(i,n) for every pair, from the three first-level contractions X x_c A_p^(c)T,
 * c = 1, 2, 3.
 *
 * Factor update.  A^(n) <- the R leading left singular vectors of Y^(n)_(n), i.e.
 * the eigenvectors of W = Y_(n) Y_(n)^T for its R largest eigenvalues (the
 * Gram-matrix route of Section 2.4), found by subspace iteration started from the
 * current A^(n): C = W V applied as Y_(n) (Y_(n)^T V) without forming W, a
 * Rayleigh-Ritz step on span(V) (V^T V normalised by its inverse square root or
 * Cholesky factor, Jacobi rotations of the projected R x R matrix), the next basis
 * C T Lambda^-1, until the largest Ritz residual ||W u_j - lambda_j u_j|| / lambda_1 is
 * at most `tol` or after `max_iters` iterations.  Columns are in decreasing eigenvalue
 * order; each new column is oriented to a non-negative inner product with the column it
 * replaces.  The entry points that update factors synchronise the stream (once per
 * iteration, or once per PP sweep when every mode converges in one iteration) and
 * return with it idle.
 *
 * Limits: 1 <= R <= 64, R <= s_n for every n; for every inner mode n the product of the
 * other dimensions is below 2^31 - 64; R^N <= 10^12.
 * ------------------------------------------------------------------------- */
#define TUCKER_MAX_RANK 64
typedef struct tucker_plan tucker_plan;

typedef struct {
  int32_t kind;                          /* PPALS_SWEEP_ALS / _PP_INIT / _PP_APPROX   */
  int32_t iters[PPALS_MAX_ORDER];        /* subspace iterations of the update of A^(n) */
  int32_t converged[PPALS_MAX_ORDER];    /* 1 if the Ritz residual reached tol       */
  int32_t rr_status[PPALS_MAX_ORDER];    /* 1 if a Rayleigh-Ritz step met a V^T V that
                                            was not positive definite                */
  int32_t pad;
  double fit;               /* 1 - sqrt(max(0, ||X||^2 - ||G||^2)) / ||X||           */
  double core_norm;         /* ||G||_F of the core this sweep formed                 */
  double f_norm;            /* ||F||_F, F = G_new - G_old (Algorithm 4)              */
  double rel_change[PPALS_MAX_ORDER];    /* ||dA^(n)||_F / ||A^(n)||_F: the change over
                                            the sweep (ALS) or since the operator build
                                            (PP)                                       */
  double ritz_residual[PPALS_MAX_ORDER]; /* final Ritz residual of each update        */
  double ms;                /* host wall time of the sweep (enqueue to completion)   */
} tucker_sweep_record;

/* Host only: checks the sizes and lays out the workspace.  dims holds `order` sizes. */
ppals_status tucker_plan_create(int32_t order, const int64_t* dims, int32_t rank,
                                tucker_plan** out);
void tucker_plan_destroy(tucker_plan* plan);
size_t tucker_workspace_bytes(const tucker_plan* plan);
/* Subspace-iteration limits (defaults: tol 1e-12, 500 iterations for sweeps, 5000 for
 * the HOSVD). */
ppals_status tucker_set_solver(tucker_plan* plan, double tol, int32_t max_iters,
                               int32_t hosvd_max_iters);

/* Y^(mode) = X x_{i != mode} A^(i)T into Y (s_mode x R^(N-1), layout above); mode is
 * 0-based.  Enqueues only. */
ppals_status tucker_ttmc(tucker_plan* plan, void* ws, const double* X, double* const* A,
                         int32_t mode, double* Y, hipStream_t stream);

/* Factor update of mode `mode` from a TTMc Y (s_mode x R^(N-1), rows indexed by the mode):
 * A_out <- leading eigenvectors of Y Y^T, started from and oriented against A_prev.
 * A_out may equal A_prev.  info (host, may be NULL) receives {iterations, converged,
 * rr_status} and *residual the final Ritz residual.  Synchronises the stream. */
ppals_status tucker_factor_update(tucker_plan* plan, void* ws, const double* Y, int32_t mode,
                                  const double* A_prev, double* A_out, int32_t* info,
                                  double* residual, hipStream_t stream);

/* Classical HOSVD start (Section 2.4): A^(n) <- leading eigenvectors of
 * X_(n) X_(n)^T by the same subspace iteration, started from the caller's V0[n]
 * (s_n x R, full column rank), with W applied through X (X_(n)^T V, then X_(n) times
 * it; W is never formed); the entry of largest magnitude of every column made positive;
 * G <- X x_1 A^(1)T .. x_N A^(N)T.  info (host, N x 3 ints, may be NULL) as in
 * tucker_factor_update per mode.  Synchronises the stream. */
ppals_status tucker_hosvd(tucker_plan* plan, void* ws, const double* X, double* const* V0,
                          double* const* A, double* G, int32_t* info, hipStream_t stream);

/* Interlaced HOSVD start (Section 2.4; the start the paper's TTMc error bound assumes):
 * with Z^(1) = X, A^(n) <- leading eigenvectors of Z^(n)_(n) Z^(n)_(n)^T by the subspace
 * iteration above (W applied through Z^(n), started from V0[n]) and
 * Z^(n+1) = Z^(n) x_n A^(n)T, which has the ranks of the modes before n + 1 in place of
 * their sizes; G <- the last Z.  Each Z^(n) after the first is s_n / R times smaller than
 * the one before, so the factor updates after the first cost little.  Signs, info,
 * arguments and errors as in tucker_hosvd.  Synchronises the stream. */
ppals_status tucker_hosvd_interlaced(tucker_plan* plan, void* ws, const double* X,
                                    double* const* V0, double* const* A, double* G,
                                    int32_t* info, hipStream_t stream);

/* One Tucker-ALS sweep (Algorithm 2 loop body) with the prefix chain above; then G from
 * the last TTMc.  G holds the previous core on entry (for ||F||).  normX2 = ||X||^2. */
ppals_status tucker_als_sweep(tucker_plan* plan, void* ws, const double* X, double* const* A,
                              double* G, double normX2, tucker_sweep_record* rec,
                              hipStream_t stream);

/* PP-Tucker operator build (Algorithm 4): with A_p = A, the pairwise operators
 * Y_p^(i,n) = X x_{j not in {i,n}} A_p^(j)T (i < n; layout x_i, x_n, then the ranks of the
 * other modes in increasing order) and Y_p^(n) for every n; dA <- 0.  Enqueues only. */
ppals_status tucker_pp_build(tucker_plan* plan, void* ws, const double* X, double* const* A,
                             hipStream_t stream);

/* First-order PP TTMc of Section 3.2.2 with the workspace's current dA:
 * Y~^(mode) = Y_p^(mode) + sum_{i != mode} Y_p^(i,mode) x_i dA^(i)T, into Y (layout of
 * tucker_ttmc).  PPALS_E_STATE before a build.  Enqueues only. */
ppals_status tucker_pp_rhs(tucker_plan* plan, void* ws, int32_t mode, double* Y,
                           hipStream_t stream);

/* One PP-Tucker sweep (Algorithm 4 inner loop body): for every mode the approximated
 * TTMc, the factor update and dA^(n) = A^(n) - A_p^(n); then G from Y~^(3).  kind is
 * recorded as given (PP_INIT or PP_APPROX).  PPALS_E_STATE before a build. */
ppals_status tucker_pp_sweep(tucker_plan* plan, void* ws, double* const* A, double* G,
                             double normX2, int32_t kind, tucker_sweep_record* rec,
                             hipStream_t stream);

/* PP-Tucker-ALS control (Algorithm 4) for at most `sweeps` sweeps from A and G (the
 * HOSVD start, normally).  PP is entered after a sweep in which every
 * ||dA^(n)|| < eps ||A^(n)|| and ||F|| < eps ||X||, and PP sweeps continue while
 * ||F|| < eps ||X||; eps = 0 gives plain Tucker-ALS.  delta > 0 stops once
 * ||F|| <= delta ||X||.  replay (host, may be NULL): replay_len sweep kinds to follow
 * instead of deciding.  recs (host) receives one record per sweep, *n_out their number. */
ppals_status tucker_run(tucker_plan* plan, void* ws, const double* X, double* const* A,
                        double* G, double eps, int32_t sweeps, double delta,
                        const int32_t* replay, int32_t replay_len, tucker_sweep_record* recs,
                        int32_t* n_out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* PPALS_H */
