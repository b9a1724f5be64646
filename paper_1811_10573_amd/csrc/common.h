// Shared definitions for the gfx950 kernels and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#define PP_MAXN 8
#define PP_MAXR 128

namespace ppk {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

enum Dt { DT_F64 = 0, DT_F32 = 1, DT_BF16 = 2 };

// Operand of a first-level contraction, laid out for direct MFMA use.
// K is split into chunks of KC k-values; inside a chunk, step t (KSTEP k-values
// per MFMA) and n-block c (16 columns) hold 64 lanes x E elements contiguously,
// so one wave reads its operand for (t, c) as a single linear 64-lane access.
struct Level1Geom {
  int64_t M;       // rows of the output (P * Q)
  int64_t K;       // contracted extent
  int64_t Q;       // extent of the uncontracted modes after the contracted block
  int64_t Kpad;    // K rounded up to a multiple of KC
  int R;           // output columns (rank)
  int NB;          // 16-column blocks per column slice (1..4)
  int nslices;     // column slices (rank > 64)
  int kc_mode;     // 1: contracted block is the fastest (Q == 1) -> K-contiguous rows
  int ksplit;      // split of K across workgroups
  int64_t kchunk;  // k-values per split (multiple of KC)
  // Strided rows and contracted index (direct operator build, FP64/FP32, scalar loads).
  // When strided != 0, row m = (m0 * mrad + m1) * mrad2 + m2 (m1 < mrad, m2 < mrad2)
  // starts at X offset m0 * ms0 + m1 * ms1 + m2 * ms2, and k = (k0 * kr1 + k1) * kr2 + k2
  // (k1 < kr1, k2 < kr2) adds k0 * ks0 + k1 * ks1 + k2 * ks2.  kmag1/ksh1 and kmag2/ksh2
  // divide by kr1 and kr2: q = (n * kmag) >> (32 + ksh), exact for n < 2^31.
  int strided;
  int64_t mrad, ms0, ms1, mrad2, ms2;
  uint32_t kr1, kr2;
  uint64_t kmag1, kmag2;
  int ksh1, ksh2;
  int64_t ks0, ks1, ks2;
};

// Khatri-Rao descriptor: value(k, r) = prod_f A_f[digit_f(k)][r], first factor slowest.
struct KrpDesc {
  const double* A[PP_MAXN];
  int64_t dim[PP_MAXN];
  int nf;
  int R;
};

// One column-wise contraction ("multi-TTV") job:
//   out[p][q][r] (+)= sum_{x in split} T[p][x][q][r] * F[x][r]
struct TtvJob {
  const void* T;       // source, FP64 or FP32 elements
  const double* F;     // weights, X x R doubles
  double* out;         // destination (FP64), P x Q x R per split slot
  int64_t P, X, Q;
  int64_t out_split_stride;  // elements between split slots of out
  int xsplit;
  int jblocks;
  int G;               // x-groups per workgroup
  int Jb;              // j-width per group (j = q*R + r)
  int64_t blocks;      // workgroups of this job
  int t_is_f32;
  int kind;            // TTV_SCALAR, TTV_SLAB, TTV_ROWS or TTV_ROWS2 (vector kernel, 256 threads)
  int lanes;           // TTV_SLAB: active lanes per wave (VEC * lanes is a multiple of R)
  int xs;              // TTV_ROWS: x-rows per split
  int f_vec;           // TTV_SLAB: F is 16-byte aligned (vector weight loads)
};
// Job kinds.  TTV_SCALAR: the general kernel (any P, X, Q).  TTV_SLAB (Q == 1): each
// (p, x-split) is a contiguous slab whose flat index is also F's, streamed with 16-byte
// loads by lanes whose rank indices stay fixed.  TTV_ROWS (Q*R a multiple of the vector
// width): each x-row of Q*R elements is streamed with 16-byte loads, F's rows of the
// split staged in LDS.
// TTV_ROWS2: TTV_ROWS with 8-byte vectors (two FP32 elements), for FP32 rows whose Q*R is
// even but not a multiple of four (16-byte vectors would straddle rows).
enum { TTV_SCALAR = 0, TTV_SLAB = 1, TTV_ROWS = 2, TTV_ROWS2 = 3 };
constexpr int TTV_VTHREADS = 256;
constexpr int TTV_SLAB_PB = 2;  // slabs per TTV_SLAB workgroup (they share the weight loads)

#define PP_MAX_JOBS 8
// Threads per multi-TTV workgroup: 12 waves, so at most two workgroups (six waves per
// SIMD) fit on a compute unit and the small per-mode kernels of the other stream find
// free wave slots and registers while a contraction streams.
constexpr int TTV_THREADS = 768;
struct TtvBatch {
  TtvJob job[PP_MAX_JOBS];
  int njobs;
  int R;
  const int* gate;     // if set and *gate == 0 the launch does nothing
};

}  // namespace ppk

// ---------------------------------------------------------------------------
// Launchers (defined in the .hip files, called from the host library)
// ---------------------------------------------------------------------------
namespace ppk {
hipError_t launch_prep_operand(const KrpDesc& krp, const Level1Geom& g, int dt, void* out,
                               hipStream_t s);
hipError_t launch_level1(const void* X, int dt, const void* B, const Level1Geom& g, void* C,
                         void* partial, hipStream_t s, hipEvent_t after_gemm = nullptr);
hipError_t launch_krp_f64(const KrpDesc& krp, int64_t K, double* out, hipStream_t s);
hipError_t launch_ttv(const TtvBatch& b, hipStream_t s);
hipError_t launch_combine(double* out, int64_t count, int R, const double* base,
                          const double* partial, int nslots, int64_t slot_stride,
                          const double* A, const double* W, hipStream_t s);
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s);
hipError_t launch_copy(double* out, const double* a, int64_t n, hipStream_t s);
hipError_t launch_copy_bytes(void* out, const void* in, size_t bytes, hipStream_t s);
// End of an operator build in one launch: A_p^(n) := A^(n) for every mode (Ap holds the
// modes back to back, mode n from off[n]), dA := 0 and U := 0, and the counters zeroed.
struct BuildReset {
  const double* A[PP_MAXN];
  double* Ap;
  int64_t off[PP_MAXN + 1];
  int N;
  double* dA;
  int64_t ndA;
  double* U;
  int64_t nU;
  int* ints[2];
  int nints[2];
};
hipError_t launch_build_reset(const BuildReset& r, hipStream_t s);
hipError_t launch_fill(double* out, double v, int64_t n, hipStream_t s);
hipError_t launch_reduce_splits_to(void* out, int out_f32, const void* partial, int part_f32,
                                   int nsplit, int64_t count, hipStream_t s);

struct ModeArgs {
  int N, R;
  int n;              // mode whose Gamma/Cholesky to prepare (-1: none)
  int prev;           // mode to finish (-1: none)
  int pp;             // 1: PP sweep (W term, dA reference A_p)
  int second_order;
  int write_fit;      // 1: compute the fit after finishing prev (last mode)
  int sweep_kind;
  int64_t prev_rows;  // s_prev
  double normX2;
  double* S;          // N x R x R (caller)
  double* U;          // N x R x R (ws)
  double* gamma;      // R x R (ws) Gamma of mode n
  double* L;          // R x R (ws) Cholesky factor (lower, row-major)
  double* gamma_save; // R x R (ws) Gamma used by the last solve (for the fit)
  double* W;          // R x R (ws)
  double* rowpart;    // rows x 4 partial norms of prev (ws)
  double* scal;       // scratch scalars (ws)
  void* rec;          // ppals_sweep_record* (device)
  int* status;        // int32 per-mode Cholesky status (ws)
};
hipError_t launch_mode_begin(const ModeArgs& a, hipStream_t s);

// Fast tail (rank <= 64): head kernel on an auxiliary stream, fused solve.
struct HeadArgs {
  int N, R;
  int n;              // mode to prepare
  int pp, second_order;
  int gamma_ready;    // Gamma^(n) (and W^(n)) already formed by the Gram kernel of mode n-1
  double* S;          // N x R x R
  double* U;          // N x R x R
  double* gamma;
  double* L;
  double* W;
  double* pack;       // solve operands: L D^-1 (transposed), D^-1 L, 1 / diag L
  int* status;
  const int* gate;    // if set and *gate == 0 the launch does nothing
};
struct GramArgs {
  int R, mode, nblk;
  int64_t rows;
  const double* A;
  const double* dA;        // NULL -> S only
  double* S_out;
  double* U_out;
  const double* blockpart; // solve partials (nblk x 5)
  const int* status;
  void* rec;
  int write_fit, sweep_kind;
  double normX2;
  const int* gate;         // if set and *gate == 0 the launch does nothing
  // optional: Gamma^(next) and W^(next) of the following mode, tile by tile (gamma_out NULL: off)
  int N, next, wterm;
  const double* S_all;     // N x R x R (the slot of this mode is being written)
  const double* U_all;
  double* gamma_out;
  double* W_out;
  // optional (write_fit set): once the record is complete, file it in ring[*ring_ctr],
  // advance the position and take Algorithm 3's threshold test for the sweep that follows:
  // *gate_out = 1 while every relative change is below eps, else 0 (sweep kind -1)
  void* ring;
  int* ring_ctr;
  int* gate_out;
  double eps;
  // optional: row ranges per tile (<= 1: one), with, in the fused PP-correction launch,
  // their partial tiles (tiles x nsplit x 512 doubles) and per-tile counters (zero between
  // launches)
  int nsplit;
  double* gpart;
  int* gctr;
};
struct FusedSolveArgs {
  int R;
  int64_t rows;
  const double* base;      // M_p^(n) or NULL
  const double* part;      // partial slots (FP64)
  int nslots;
  int64_t slot_stride;
  const double* W;         // second-order matrix or NULL
  const double* pack;      // written by the head: L D^-1 (transposed), D^-1 L, 1 / diag L
  const double* gamma;
  double* A;
  const double* Aref;      // NULL -> old A
  double* dA;              // NULL -> not stored
  double* blockpart;       // nblk x 5 partial sums
  const int* status;
  int write_fit;
  const int* gate;         // if set and *gate == 0 the launch does nothing
  double step;             // update step size lambda: A_new = A + lambda (M Gamma^-1 - A)
};
hipError_t launch_head(const HeadArgs& h, hipStream_t s);
hipError_t launch_solve_fused(const FusedSolveArgs& a, hipStream_t s);
int solve_fused_blocks(int64_t rows);
// tail_order: the wave count (and so the summation order) of the fused PP-correction
// launch's Gram role, so that both give the same bits
hipError_t launch_gram_tiles(const GramArgs& a, hipStream_t s, bool tail_order = false);
// The contraction jobs of a PP mode, the Grams of the previous mode (g may be NULL) and
// the head of this mode in one launch; ctr is a device int that is zero between launches.
bool ttv_tail_fusable(const TtvBatch& b);
hipError_t launch_ttv_tail(const TtvBatch& b, const GramArgs* g, const HeadArgs& h, int* ctr,
                           hipStream_t s);
hipError_t launch_set_int(int* p, int v, hipStream_t s);
hipError_t launch_set_int2(int* p, int v, int* q, int w, hipStream_t s);
hipError_t launch_pp_gate_ring(void* rec, int N, double eps, int* gate, void* ring, int* ctr,
                               hipStream_t s);
hipError_t launch_rec_store(const void* rec, void* ring, const int* ctr, hipStream_t s);

// learned PP controller (k_mlp.hip)
constexpr int MLP_MAX_IN = 16;
constexpr int MLP_MAX_HIDDEN = 1024;
hipError_t launch_mlp_forward(const float* p, int d, int H, const float* X, int64_t B, float* y,
                              float* hcache, hipStream_t s);
hipError_t launch_mlp_backward(const float* p, int d, int H, const float* X, const float* hcache,
                               const float* y, const float* t, int64_t B, float* g, float* loss,
                               hipStream_t s);
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int64_t P, float lr,
                           float beta1, float beta2, float eps, float c1, float c2, hipStream_t s);
hipError_t launch_mlp_decide(const float* p, int H, int N, void* rec, int sweep, double log10_tau,
                             hipStream_t s);
hipError_t launch_rhs_err(const double* Mt, const double* M, int64_t count, double* out,
                          hipStream_t s);
hipError_t launch_rhs_err_max(const double* sums, int N, double* err, hipStream_t s);

struct SolveArgs {
  int R;
  int64_t rows;
  const double* M;       // rows x R FP64 right-hand side
  const float* M32;      // alternatively FP32 right-hand side (standalone gram_solve)
  const double* L;       // R x R
  const double* gamma;   // R x R
  double* A;             // rows x R, in/out
  const double* Aref;    // reference for dA (A_p in PP); NULL -> old A
  double* dA;            // rows x R output of A_new - ref (may be NULL)
  double* rowpart;       // rows x 4: ||g||^2, ||dA||^2, ||a||^2, <m, a>
  const int* status;     // Cholesky status (2 -> leave A unchanged)
  double step;           // update step size lambda: A_new = A + lambda (M Gamma^-1 - A)
};
hipError_t launch_solve_rows(const SolveArgs& a, hipStream_t s);
// S_out = A^T A; if dA: U_out = A^T dA (R x R each)
hipError_t launch_gram(const double* A, const double* dA, int64_t rows, int R, double* S_out,
                       double* U_out, hipStream_t s);
hipError_t launch_norm2(const void* X, int dt, int64_t n, double* partial, int nblocks,
                        double* out, hipStream_t s);
hipError_t launch_cast_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s);
hipError_t launch_residual2(const void* X, int dt, const double* const* A, const int64_t* dims,
                            int N, int R, double* partial, int nblocks, double* out,
                            hipStream_t s);
hipError_t launch_finish_gram_solve(const double* rowpart, int64_t rows, double* grad_out,
                                    int32_t* status_out, const int* status, hipStream_t s);
hipError_t launch_chol_standalone(const double* gamma, int R, double* L, int* status,
                                  hipStream_t s);
}  // namespace ppk
