// Batched PP-CP-ALS for many independent order-3 problems: device descriptors and
// per-problem state shared by the batched kernels (k_batch.hip) and the host engine
// (batch.cpp).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ppk {

// kind of the current sweep of one problem
enum { BK_NONE = 0, BK_ALS = 1, BK_PP_INIT = 2, BK_PP_APPROX = 3 };
constexpr int BMASK_ALS = 1 << BK_ALS;
constexpr int BMASK_INIT = 1 << BK_PP_INIT;
constexpr int BMASK_APPROX = 1 << BK_PP_APPROX;
constexpr int BMASK_PP = BMASK_INIT | BMASK_APPROX;

constexpr int BATCH_MAX_R = 64;
constexpr int BATCH_MAX_S = 256;
constexpr int BATCH_GEMM_VARIANTS = 2;  // rows per GEMM tile: 64 or 128
constexpr int BATCH_RUN_ROWS = 1024;   // rows of one problem per GEMM work item (a run of tiles)

// Static description of one problem (device pointers into the caller's buffers and
// the batch workspace).
struct BProb {
  int s[3];
  int R;
  const float* X;   // s0 x s1 x s2, row-major
  double* A[3];     // factors, s_n x R
  float* Af[3];     // the factors transposed in FP32 for the contraction kernel:
                    // BATCH_MAX_R columns of ceil(s_n / 32) * 32 entries, zero beyond R x s_n
  double* S;        // 3 x R x R Grams
  double* U;        // 3 x R x R, A^(n)T dA^(n)
  float* op[3];     // op[0] = M^(0,1) (s0 x s1 x R), op[1] = M^(0,2) (s0 x s2 x R),
                    // op[2] = M^(1,2) (s1 x s2 x R); in ALS sweeps op[0] and op[2] hold
                    // the dimension-tree intermediates X x_2 A^(2) and X x_0 A^(0)
  double* Mp[3];    // M_p^(n), s_n x R
  double* Ap[3];    // factors at the last operator build
  double* dA[3];    // A^(n) - A_p^(n)
  double* M;        // right-hand side of the mode being solved, max_s x R
  uint8_t* klog;    // kind of every sweep (max_sweeps bytes)
};

// Per-problem iteration state (device).
struct BState {
  int kind, prev_kind, sweep, done;
  int conv_sweep, n_als, n_init, n_approx;
  int chol[3];
  int pad;
  double normX2, fit, fit_prev;
  double rel[3];
  double sums[3][3];  // per mode: ||dA||^2, ||A||^2, <M, A>
  double gs;          // sum of Gamma^(2) * S^(2) after the last mode
  long long t_start, t_conv;
};

// Run-wide settings (device).
struct BConf {
  double eps;       // PP threshold on ||dA|| / ||A||
  double tol;       // convergence: |fit - fit_prev| < tol
  int max_sweeps;
  int second_order;
};

// Work item of the grouped kernels: the problem and the first output row (contraction:
// BATCH_RUN_ROWS rows from m0; multi-TTV: 256 output elements from m0).
struct BTile {
  int prob;
  int m0;
};

hipError_t launch_b_begin(BState* st, BProb* pr, const BConf* conf, int count, hipStream_t s);
hipError_t launch_b_f32(const BProb* pr, const BState* st, int count, int mode_mask, hipStream_t s);
hipError_t launch_b_prep(const BProb* pr, const BState* st, int count, hipStream_t s);
hipError_t launch_b_gemm(int variant, const BProb* pr, const BState* st, const BTile* tiles,
                         int ntiles, int cmode, int out_op, int kind_mask, hipStream_t s);
hipError_t launch_b_ttv(const BProb* pr, const BState* st, const BTile* tiles, int ntiles, int mode,
                        int build_mp, hipStream_t s);
hipError_t launch_b_solve(const BProb* pr, BState* st, const BConf* conf, int count, int mode,
                          int maxR, hipStream_t s);
hipError_t launch_b_end(BState* st, const BConf* conf, int count, hipStream_t s);
hipError_t launch_b_norm(const BProb* pr, BState* st, const BConf* conf, int count, hipStream_t s);
int batch_gemm_rows(int variant);
hipError_t batch_prepare();

}  // namespace ppk
