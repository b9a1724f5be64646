// Device-side interface of the Tucker kernels (k_tucker.hip) and the host plan helpers.
#pragma once

#include "common.h"

namespace ppk {

struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t M, N, K;
  int64_t sam, sak;  // A(m, k) = A[m * sam + k * sak]
  int64_t sbk, sbn;  // B(k, n) = B[k * sbk + n * sbn]
  int64_t ldc;
  double alpha, beta;
  int ks;            // K split over workgroups (>= 1); ks > 1 needs alpha 1, beta 0, ldc N
  double* part;      //   and ks x nb x M x N doubles of partial sums here
  int nb;            // batch of products sharing A (>= 1): B_x = B + x sbb, C_x = C + x M N
  int64_t sbb;       //   (nb > 1 needs ldc N)
};
// Minimum k-values per split of launch_gemm_f64.
constexpr int64_t kGemmSplitMin = 32;
hipError_t launch_gemm_f64(const GemmArgs& g, hipStream_t s);

struct RRArgs {
  int R;
  const double* B;   // R x R, V^T V
  const double* H;   // R x R, V^T W V
  const double* P;   // R x R, V^T A_prev (NULL: no sign alignment)
  double* T;         // R x R out: V T are the Ritz vectors, decreasing order
  double* lam;       // R out: Ritz values, decreasing
  int* status;       // [0] 1 if V^T V was not positive definite, [1] Jacobi sweeps
  // launch_rr_small only (B, H and P are then not read): V and C (rows x R) give
  // B = V^T V and H = V^T C, Ap (rows x R, may be null) gives P = V^T Ap; the Ritz update's
  // outputs (U, the next basis Vout = V, the residual); C is the sum of npart slots of
  // pstride doubles at cpart (null: C itself).
  const double* V;
  const double* C;
  const double* Ap;
  int64_t rows;
  double* U;
  double* Vout;
  double* residual;
  const double* cpart;
  int npart;
  int64_t pstride;
};
// The whole subspace step after C = W V (projections, Rayleigh-Ritz, Ritz update, residual)
// in one workgroup, for R <= 16 and rows R <= kRRSmallElems (V, C, A_prev held in LDS).
constexpr int64_t kRRSmallElems = 2048;
constexpr int kRRSmallParts = 32;  // partial slots of C it adds at most
bool rr_small_fits(int64_t rows, int R);
hipError_t launch_rr_small(const RRArgs& a, hipStream_t s);
hipError_t launch_rayleigh_ritz(const RRArgs& a, hipStream_t s);
// U = V T, CT = C T, V <- CT diag(lam)^-1 and *residual = max_j ||CT_j - lam_j U_j|| / |lam_0|;
// part holds ceil(rows / 32) x R doubles.
constexpr int kRitzRows = 32;
hipError_t launch_ritz_update(double* V, const double* C, const double* T, const double* lam,
                              double* U, double* part, int64_t rows, int R, double* residual,
                              hipStream_t s);
hipError_t launch_sign_by_max(double* V, int64_t rows, int R, hipStream_t s);
struct TuckerCombine {
  double* out;              // rows x cols
  const double* base;       // rows x cols, or null
  const double* term[7];    // rows x cols each, rank digit pos[t] moved last
  int pos[7];
  int nterms;
  int nd;                   // rank digits (N - 1)
  int R;
  int64_t rows, cols;       // s_n, R^(N-1)
  int64_t rpow[9];          // R^k
};
hipError_t launch_tucker_combine(const TuckerCombine& a, hipStream_t s);
// The same sum with every term contracted in place: term t of output (x, c) is
// sum_{k < klen[t]} op[t][x nstride[t] + rest + k kstride[t]] F[t][k R + r], where (rest, r)
// is c with the rank digit at pos[t] taken out (r) and the others kept in order (rest).
// For small operators, where one launch beats a contraction launch per term.  Each output
// element takes pp_rhs_lanes(rows cols) lanes (1 to 16, at least 98304 lanes in all when
// 16 per element reach it).
struct TuckerPPRhs {
  double* out;
  const double* base;
  const double* op[7];
  const double* F[7];       // klen[t] x R
  int64_t klen[7], kstride[7], nstride[7];
  int pos[7];
  int nterms;
  int nd;
  int R;
  int64_t rows, cols;
  int64_t rpow[9];
};
int pp_rhs_lanes(int64_t elems);
hipError_t launch_tucker_pp_rhs(const TuckerPPRhs& a, hipStream_t s);
// Total multiply-adds below which the in-place form is used.
constexpr int64_t kPPRhsInPlaceMax = int64_t(1) << 25;
hipError_t launch_core_stats(const double* Gn, const double* Go, int64_t n, double* out,
                             hipStream_t s);
// End of a factor update: A = U (skipped when A is null), dA = U - Ap, and out[0], out[1] =
// ||U||^2, ||U - Ap||^2 summed in the order of launch_core_stats(U, Ap).
hipError_t launch_mode_end(const double* U, const double* Ap, double* A, double* dA, int64_t n,
                           double* out, hipStream_t s);
// C = Y (Y^T V) for a small TTMc Y (s x m, row-major), V (s x R): the columns of Y in chunks
// of w, one workgroup each, whose s x R results go to part[chunk] and are added in chunk
// order by a second launch.  w_apply_width gives w (about 32 chunks, more when LDS bounds
// w), or 0 when a chunk (s x w), V and Z = Y_chunk^T V (w x R) do not fit the workgroup's
// LDS.
int w_apply_width(int64_t s, int64_t m, int R);
hipError_t launch_w_apply(const double* Y, const double* V, int64_t s, int64_t m, int R, int w,
                          double* part, double* C, hipStream_t st);
// the same without the second launch: C is left as the (m + w - 1) / w slots of s x R in part
hipError_t launch_w_apply_parts(const double* Y, const double* V, int64_t s, int64_t m, int R,
                                int w, double* part, hipStream_t st);
// out1 = out2 = in (n doubles)
hipError_t launch_copy2(double* out1, double* out2, const double* in, int64_t n, hipStream_t s);
// First-level contraction at small rank on the vector units: C (M x R, row-major) with
// C[p Q + q][r] = sum_k T[(p K + k) Q + q] F[k R + r] (T of P x K x Q, Q > 1; F of K x R,
// row-major).  ttm_small_r_fits says when it is used in place of the matrix-core kernel
// (R <= 8, odd Q > 1, M >= 2^20).
bool ttm_small_r_fits(int64_t M, int64_t K, int64_t Q, int R);
hipError_t launch_ttm_small_r(const double* T, const double* F, int64_t M, int64_t K, int64_t Q,
                              int R, double* C, hipStream_t s);
// The same for few rows over a long k: C[m][r] = sum_k T[(k / after) M after + m after +
// k mod after] F[k R + r] (after = K: rows contiguous; K a multiple of after), k split
// over workgroups whose M x R parts go to part and are added in order by a second
// launch.  ttm_rows_small_r_parts gives the number of parts (at most max_parts), or 0
// when the kernel does not apply (R <= 8, M R <= 2048, K >= 2^20, max_parts >= 256).
int ttm_rows_small_r_parts(int64_t M, int64_t K, int R, int max_parts);
hipError_t launch_ttm_rows_small_r(const double* T, const double* F, int64_t M, int64_t K,
                                   int64_t after, int R, int nparts, double* part, double* C,
                                   hipStream_t s);

}  // namespace ppk

// first-level contraction geometry and the multiplier of the strided loads' divisions
// (ppals.cpp)
ppk::Level1Geom l1_geom(int64_t P, int64_t K, int64_t Q, int R, int l1dt);
void l1_magic(uint32_t d, uint64_t* mag, int* sh);
