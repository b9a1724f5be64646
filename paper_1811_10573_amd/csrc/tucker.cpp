// Tucker-ALS and PP-Tucker-ALS for order-3 tensors (Algorithms 2 and 4), FP64.
//
// Every TTM runs on the first-level MFMA contraction kernel: a P x K x Q tensor
// contracted over its middle index with a K x R factor, written P x Q x R.  The three
// modes of an order-3 tensor are all reachable that way without transposing X, and
// the rank indices of each TTMc come out in a fixed order per mode (documented with
// tucker_ttmc).  The factor update is a subspace iteration on W = Y_(n) Y_(n)^T whose
// products W V are applied as Y_(n) (Y_(n)^T V), two more first-level contractions;
// the small R x R algebra (Rayleigh-Ritz with Jacobi rotations) is one workgroup.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ppals.h"
#include "common.h"
#include "tucker.h"

namespace ppk {
ppals_status set_error(ppals_status st, const std::string& msg);
}

using namespace ppk;

#define THIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(PPALS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)
#define TCHK(expr)                    \
  do {                                \
    ppals_status st_ = (expr);        \
    if (st_ != PPALS_OK) return st_;  \
  } while (0)

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Contr {  // a first-level contraction P x K x Q (K contracted)
  int64_t P, K, Q;
};

}  // namespace

struct tucker_plan {
  int64_t s[3];
  int R;
  double tol = 1e-12;
  int max_iters = 500;
  int hosvd_iters = 5000;
  // workspace regions (byte offsets)
  size_t o_T3, o_T1, o_op01, o_op02, o_op12, o_Yp[3], o_Y, o_Ta, o_Tb, o_Gn, o_Ap[3], o_dA[3],
      o_Aold, o_V, o_C, o_U, o_Z, o_B, o_H, o_P, o_T, o_lam, o_info, o_stats, o_prep, o_part,
      o_gpart, o_Zx, o_rpart;
  size_t slot = 0;  // bytes between the basis slots V, C, A_prev
  size_t ws_bytes = 0;
  bool built = false;
  bool dA_zero[3] = {true, true, true};
  bool pp_optimistic = true;  // PP sweeps: one unchecked subspace iteration per mode first
  size_t o_Astart[3];
  void* built_ws = nullptr;
};

namespace {

struct TCtx {
  tucker_plan* p;
  char* ws;
  hipStream_t s;
  double* d(size_t off) const { return reinterpret_cast<double*>(ws + off); }
};

// Contractions the plan runs, for the workspace size of the operand and partial buffers.
std::vector<Contr> all_contractions(const tucker_plan* p) {
  const int64_t s0 = p->s[0], s1 = p->s[1], s2 = p->s[2], R = p->R;
  std::vector<Contr> v = {
      {s0 * s1, s2, 1},   // X x_3            -> (x1, x2, r3)
      {1, s0, s1 * s2},   // X x_1            -> (x2, x3, r1)
      {s0, s1, s2},       // X x_2            -> (x1, x3, r2)
      {s0, s1, R},        // (x1,x2,r3) x x2  -> (x1, r3, r2)
      {1, s0, s1 * R},    // (x1,x2,r3) x x1  -> (x2, r3, r1)
      {1, s1, s2 * R},    // (x2,x3,r1) x x2  -> (x3, r1, r2)
      {s0, s2, R},        // (x1,x3,r2) x x3  -> (x1, r2, r3)
      {s1, s2, R},        // (x2,x3,r1) x x3  -> (x2, r1, r3)
      {1, s0, s2 * R},    // (x1,x3,r2) x x1  -> (x3, r2, r1)
      {1, s2, R * R},     // core from (x3, r1, r2)
  };
  for (int n = 0; n < 3; ++n) {
    v.push_back({1, p->s[n], R * R});  // Y_(n)^T V
    v.push_back({p->s[n], R * R, 1});  // Y_(n) Z
  }
  v.push_back({s0, s1 * s2, 1});       // HOSVD: X_(1) Z
  v.push_back({1, s0 * s1, s2});       // HOSVD: X_(3) Z
  return v;
}

size_t prep_elems(const Level1Geom& g) { return (size_t)g.nslices * g.Kpad * 16 * g.NB; }
size_t part_elems(const Level1Geom& g) {
  return g.ksplit > 1 ? (size_t)g.ksplit * g.M * g.R : 0;
}

// out (P x Q x R) = sum_k T(p, k, q) F(k, r)
ppals_status ttm(const TCtx& c, const double* T, Contr k, const double* F, double* out) {
  const Level1Geom g = l1_geom(k.P, k.K, k.Q, c.p->R, DT_F64);
  KrpDesc krp;
  memset(&krp, 0, sizeof(krp));
  krp.nf = 1;
  krp.R = c.p->R;
  krp.A[0] = F;
  krp.dim[0] = k.K;
  void* B = c.ws + c.p->o_prep;
  THIPCHK(launch_prep_operand(krp, g, DT_F64, B, c.s));
  THIPCHK(launch_level1(T, DT_F64, B, g, out, c.ws + c.p->o_part, c.s));
  return PPALS_OK;
}

GemmArgs gemm_args(const double* A, const double* B, double* C, int64_t M, int64_t N, int64_t K) {
  GemmArgs g;
  memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.C = C;
  g.M = M;
  g.N = N;
  g.K = K;
  g.ldc = N;
  g.alpha = 1.0;
  g.beta = 0.0;
  g.ks = 1;
  g.nb = 1;
  return g;
}

constexpr int kMaxGemmSplit = 32;

// The projections of the Rayleigh-Ritz step in one launch: V^T V, V^T C and (nb = 3)
// V^T A_prev into the consecutive R x R blocks B, H, P.  V, C and A_prev are the
// consecutive slots of the basis region.
ppals_status projections(const TCtx& c, int64_t rows, int nb) {
  const int R = c.p->R;
  GemmArgs g = gemm_args(c.d(c.p->o_V), c.d(c.p->o_V), c.d(c.p->o_B), R, R, rows);
  g.sam = 1;
  g.sak = R;
  g.sbk = R;
  g.sbn = 1;
  g.nb = nb;
  g.sbb = (int64_t)(c.p->slot / sizeof(double));
  g.ks = (int)std::min<int64_t>(kMaxGemmSplit, std::max<int64_t>(1, rows / kGemmSplitMin));
  g.part = c.d(c.p->o_gpart);
  THIPCHK(launch_gemm_f64(g, c.s));
  return PPALS_OK;
}

// The product X_(1) Z of the HOSVD of the middle mode: C[x2][r] = sum over (x1, x3) of
// X[x1][x2][x3] Z[x1 s3 + x3][r], a first-level contraction whose rows (x2) and
// contracted index (x1, x3) reach X through strided offsets.
Level1Geom middle_unfolding_geom(const tucker_plan* p) {
  const int64_t s0 = p->s[0], s1 = p->s[1], s2 = p->s[2];
  Level1Geom g = l1_geom(s1, s0 * s2, 1, p->R, DT_F64);
  g.kc_mode = 0;
  g.Q = 1;
  g.strided = 1;
  g.mrad = s1;  // row m = x2: offset x2 s3
  g.ms0 = 0;
  g.ms1 = s2;
  g.mrad2 = 1;
  g.ms2 = 0;
  g.kr1 = 1;    // k = x1 s3 + x3: offset x1 s2 s3 + x3
  g.kr2 = (uint32_t)s2;
  l1_magic(g.kr1, &g.kmag1, &g.ksh1);
  l1_magic(g.kr2, &g.kmag2, &g.ksh2);
  g.ks0 = s1 * s2;
  g.ks1 = 0;
  g.ks2 = 1;
  return g;
}

// out (M x R) = first-level contraction of T with the K x R factor F under geometry g
ppals_status ttm_geom(const TCtx& c, const double* T, const Level1Geom& g, const double* F,
                      double* out) {
  KrpDesc krp;
  memset(&krp, 0, sizeof(krp));
  krp.nf = 1;
  krp.R = c.p->R;
  krp.A[0] = F;
  krp.dim[0] = g.K;
  void* B = c.ws + c.p->o_prep;
  THIPCHK(launch_prep_operand(krp, g, DT_F64, B, c.s));
  THIPCHK(launch_level1(T, DT_F64, B, g, out, c.ws + c.p->o_part, c.s));
  return PPALS_OK;
}

// C = W V for the subspace iteration of mode n: through a TTMc Y (W = Y_(n) Y_(n)^T,
// Y given) or, for the HOSVD (Y null), through X itself (W = X_(n) X_(n)^T) with the
// intermediate Z = X_(n)^T V in the scratch region Zx.
ppals_status apply_w(const TCtx& c, int n, const double* Y, const double* X, const double* V,
                     double* C) {
  tucker_plan* p = c.p;
  const int64_t s0 = p->s[0], s1 = p->s[1], s2 = p->s[2], R = p->R;
  const int64_t sn = p->s[n];
  if (Y) {
    double* Z = c.d(p->o_Z);
    TCHK(ttm(c, Y, {1, sn, R * R}, V, Z));  // Z = Y^T V   (R^2 x R)
    TCHK(ttm(c, Y, {sn, R * R, 1}, Z, C));  // C = Y Z     (s_n x R)
    return PPALS_OK;
  }
  double* Zx = c.d(p->o_Zx);
  if (n == 0) {
    TCHK(ttm(c, X, {1, s0, s1 * s2}, V, Zx));  // (x2, x3, r)
    TCHK(ttm(c, X, {s0, s1 * s2, 1}, Zx, C));  // (x1, r)
  } else if (n == 2) {
    TCHK(ttm(c, X, {s0 * s1, s2, 1}, V, Zx));  // (x1, x2, r)
    TCHK(ttm(c, X, {1, s0 * s1, s2}, Zx, C));  // (x3, r)
  } else {
    TCHK(ttm(c, X, {s0, s1, s2}, V, Zx));      // (x1, x3, r)
    TCHK(ttm_geom(c, X, middle_unfolding_geom(p), Zx, C));  // (x2, r)
  }
  return PPALS_OK;
}

struct IterInfo {
  double residual;
  int32_t rr_bad;
  int32_t jacobi_sweeps;
};

// One subspace iteration on the basis V of the workspace: C = W V, the projections, the
// Rayleigh-Ritz step and the Ritz update (U, residual into info, next basis in V).
// Enqueues only.  has_prev: A_prev is in the basis region's third slot.
ppals_status subspace_step(const TCtx& c, int n, const double* Y, const double* X, bool has_prev,
                           IterInfo* info) {
  tucker_plan* p = c.p;
  const int R = p->R;
  const int64_t sn = p->s[n];
  double* V = c.d(p->o_V);
  double* C = c.d(p->o_C);
  TCHK(apply_w(c, n, Y, X, V, C));  // C = W V
  TCHK(projections(c, sn, has_prev ? 3 : 2));
  RRArgs rr;
  rr.R = R;
  rr.B = c.d(p->o_B);
  rr.H = c.d(p->o_H);
  rr.P = has_prev ? c.d(p->o_P) : nullptr;
  rr.T = c.d(p->o_T);
  rr.lam = c.d(p->o_lam);
  rr.status = &info->rr_bad;
  THIPCHK(launch_rayleigh_ritz(rr, c.s));
  // Ritz vectors U, the residual, and the next basis V <- W U diag(lam)^-1
  THIPCHK(launch_ritz_update(V, C, rr.T, rr.lam, c.d(p->o_U), c.d(p->o_rpart), sn, R,
                             &info->residual, c.s));
  return PPALS_OK;
}

// Subspace iteration for the R leading eigenvectors of W (s_n x s_n), W = Y_(n) Y_(n)^T
// for a TTMc Y or, with Y null, X_(n) X_(n)^T (the HOSVD).  V starts from V0; A_prev (may
// be null) orients the columns.  Result into A_out.
ppals_status subspace(const TCtx& c, int n, const double* Y, const double* X, const double* V0,
                      const double* A_prev, double* A_out, int max_iters, int32_t* info,
                      double* residual) {
  tucker_plan* p = c.p;
  const int R = p->R;
  const int64_t sn = p->s[n];
  double* V = c.d(p->o_V);
  double* C = c.d(p->o_C);
  double* U = c.d(p->o_U);
  double* T = c.d(p->o_T);
  double* lam = c.d(p->o_lam);
  double* Aold = c.d(p->o_Aold);
  IterInfo* dinfo = reinterpret_cast<IterInfo*>(c.ws + p->o_info) + n;
  if (A_prev && A_prev != Aold) THIPCHK(launch_copy(Aold, A_prev, sn * R, c.s));
  THIPCHK(launch_copy(V, V0, sn * R, c.s));
  IterInfo hinfo;
  memset(&hinfo, 0, sizeof(hinfo));
  int it = 0, bad = 0;
  bool conv = false;
  while (it < max_iters) {
    ++it;
    TCHK(subspace_step(c, n, Y, X, A_prev != nullptr, dinfo));
    THIPCHK(hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, c.s));
    THIPCHK(hipStreamSynchronize(c.s));
    bad |= hinfo.rr_bad;
    if (hinfo.residual <= p->tol) {
      conv = true;
      break;
    }
  }
  (void)V;
  (void)C;
  (void)T;
  (void)lam;
  THIPCHK(launch_copy(A_out, U, sn * R, c.s));
  if (!A_prev) THIPCHK(launch_sign_by_max(A_out, sn, R, c.s));
  if (info) {
    info[0] = it;
    info[1] = conv ? 1 : 0;
    info[2] = bad;
  }
  if (residual) *residual = hinfo.residual;
  return PPALS_OK;
}

// The TTMc Y^(n) needed by mode n of a sweep.  For an ALS sweep with the order-3
// tree: mode 0 and 1 from T3 = X x_3 A^(3)T (computed at mode 0), mode 2 from
// T1 = X x_1 A^(1)T.
ppals_status als_ttmc(const TCtx& c, const double* X, double* const* A, int n, bool make_t3,
                      double* Y) {
  tucker_plan* p = c.p;
  const int64_t s0 = p->s[0], s1 = p->s[1], s2 = p->s[2], R = p->R;
  double* T3 = c.d(p->o_T3);
  double* T1 = c.d(p->o_T1);
  if (n == 0) {
    if (make_t3) TCHK(ttm(c, X, {s0 * s1, s2, 1}, A[2], T3));
    TCHK(ttm(c, T3, {s0, s1, R}, A[1], Y));  // (x1, r3, r2)
  } else if (n == 1) {
    if (make_t3) TCHK(ttm(c, X, {s0 * s1, s2, 1}, A[2], T3));
    TCHK(ttm(c, T3, {1, s0, s1 * R}, A[0], Y));  // (x2, r3, r1)
  } else {
    TCHK(ttm(c, X, {1, s0, s1 * s2}, A[0], T1));
    TCHK(ttm(c, T1, {1, s1, s2 * R}, A[1], Y));  // (x3, r1, r2)
  }
  return PPALS_OK;
}

// Core from Y^(3) (x3, r1, r2) and A^(3): G (r1, r2, r3); stats[6..7] = ||G||^2, ||G - G_old||^2;
// G_old <- G.
ppals_status finish_core(const TCtx& c, const double* Y3, const double* A3, double* G,
                         bool commit = true) {
  tucker_plan* p = c.p;
  const int64_t R = p->R;
  double* Gn = c.d(p->o_Gn);
  TCHK(ttm(c, Y3, {1, p->s[2], R * R}, A3, Gn));
  THIPCHK(launch_core_stats(Gn, G, R * R * R, c.d(p->o_stats) + 6, c.s));
  if (commit) THIPCHK(launch_copy(G, Gn, R * R * R, c.s));
  return PPALS_OK;
}

void fill_record(const tucker_plan* p, const double* stats, double normX2, int kind,
                 tucker_sweep_record* rec) {
  rec->kind = kind;
  for (int n = 0; n < 3; ++n) {
    const double a2 = stats[2 * n], d2 = stats[2 * n + 1];
    rec->rel_change[n] = a2 > 0.0 ? std::sqrt(d2) / std::sqrt(a2) : 0.0;
  }
  const double g2 = stats[6];
  rec->core_norm = std::sqrt(g2);
  rec->f_norm = std::sqrt(stats[7]);
  rec->fit = 1.0 - std::sqrt(std::max(0.0, normX2 - g2)) / std::sqrt(normX2);
  (void)p;
}

ppals_status check_common(tucker_plan* p, void* ws) {
  if (!p) return set_error(PPALS_E_ARG, "NULL plan");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
    return set_error(PPALS_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  return PPALS_OK;
}

ppals_status check_factors(const tucker_plan* p, double* const* A) {
  if (!A) return set_error(PPALS_E_ARG, "NULL factor array");
  for (int n = 0; n < 3; ++n)
    if (!A[n]) return set_error(PPALS_E_ARG, "NULL factor " + std::to_string(n));
  (void)p;
  return PPALS_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-order PP TTMc of mode n into Y from the operators and dA.
ppals_status pp_rhs_impl(const TCtx& c, int n, double* Y) {
  tucker_plan* p = c.p;
  const int64_t s0 = p->s[0], s1 = p->s[1], s2 = p->s[2], R = p->R;
  double* op01 = c.d(p->o_op01);  // (x1, x2, r3)
  double* op02 = c.d(p->o_op02);  // (x1, x3, r2)
  double* op12 = c.d(p->o_op12);  // (x2, x3, r1)
  double* Ta = c.d(p->o_Ta);
  double* Tb = c.d(p->o_Tb);
  const double* dA[3] = {c.d(p->o_dA[0]), c.d(p->o_dA[1]), c.d(p->o_dA[2])};
  const double* ta = nullptr;  // same rank order as Y_p^(n)
  const double* tb = nullptr;  // rank indices swapped
  if (n == 0) {
    if (!p->dA_zero[1]) { TCHK(ttm(c, op01, {s0, s1, R}, dA[1], Ta)); ta = Ta; }       // (x1, r3, r2)
    if (!p->dA_zero[2]) { TCHK(ttm(c, op02, {s0, s2, R}, dA[2], Tb)); tb = Tb; }       // (x1, r2, r3)
  } else if (n == 1) {
    if (!p->dA_zero[0]) { TCHK(ttm(c, op01, {1, s0, s1 * R}, dA[0], Ta)); ta = Ta; }   // (x2, r3, r1)
    if (!p->dA_zero[2]) { TCHK(ttm(c, op12, {s1, s2, R}, dA[2], Tb)); tb = Tb; }       // (x2, r1, r3)
  } else {
    if (!p->dA_zero[1]) { TCHK(ttm(c, op12, {1, s1, s2 * R}, dA[1], Ta)); ta = Ta; }   // (x3, r1, r2)
    if (!p->dA_zero[0]) { TCHK(ttm(c, op02, {1, s0, s2 * R}, dA[0], Tb)); tb = Tb; }   // (x3, r2, r1)
  }
  THIPCHK(launch_pp_tucker_combine(Y, c.d(p->o_Yp[n]), ta, tb, p->s[n], (int)R, c.s));
  return PPALS_OK;
}

}  // namespace

extern "C" {

ppals_status tucker_plan_create(const int64_t dims[3], int32_t rank, tucker_plan** out) {
  if (!dims || !out) return set_error(PPALS_E_ARG, "NULL argument");
  *out = nullptr;
  if (rank < 1 || rank > TUCKER_MAX_RANK)
    return set_error(PPALS_E_UNSUPPORTED, "Tucker rank must be in [1, 64]");
  for (int n = 0; n < 3; ++n) {
    if (dims[n] < 1) return set_error(PPALS_E_ARG, "dims must be >= 1");
    if (dims[n] < rank)
      return set_error(PPALS_E_UNSUPPORTED, "Tucker rank must not exceed any dimension");
  }
  if ((double)dims[0] * (double)dims[2] > 2147483647.0 - 64.0)
    return set_error(PPALS_E_UNSUPPORTED, "s1 * s3 must stay below 2^31 - 64 (strided HOSVD product)");
  tucker_plan* p = new tucker_plan();
  for (int n = 0; n < 3; ++n) p->s[n] = dims[n];
  p->R = rank;
  const int64_t s0 = dims[0], s1 = dims[1], s2 = dims[2], R = rank;
  const int64_t smax = std::max(s0, std::max(s1, s2));
  size_t off = 0;
  auto take = [&](size_t elems) {
    const size_t o = off;
    off += al256(std::max<size_t>(elems, 1) * sizeof(double));
    return o;
  };
  p->o_T3 = take(s0 * s1 * R);
  p->o_T1 = take(s1 * s2 * R);
  p->o_op01 = take(s0 * s1 * R);
  p->o_op02 = take(s0 * s2 * R);
  p->o_op12 = take(s1 * s2 * R);
  for (int n = 0; n < 3; ++n) p->o_Yp[n] = take(dims[n] * R * R);
  p->o_Y = take(smax * R * R);
  p->o_Ta = take(smax * R * R);
  p->o_Tb = take(smax * R * R);
  p->o_Gn = take(R * R * R);
  for (int n = 0; n < 3; ++n) p->o_Ap[n] = take(dims[n] * R);
  for (int n = 0; n < 3; ++n) p->o_dA[n] = take(dims[n] * R);
  // basis slots V, C, A_prev at equal spacing (one batched projection launch)
  p->slot = al256((size_t)smax * R * sizeof(double));
  p->o_V = take(smax * R);
  p->o_C = take(smax * R);
  p->o_Aold = take(smax * R);
  p->o_U = take(smax * R);
  p->o_Z = take(R * R * R);
  // B, H, P consecutive R x R blocks
  p->o_B = take(3 * R * R);
  p->o_H = p->o_B + (size_t)R * R * sizeof(double);
  p->o_P = p->o_H + (size_t)R * R * sizeof(double);
  p->o_rpart = take(((smax + kRitzRows - 1) / kRitzRows) * R);
  p->o_T = take(R * R);
  p->o_lam = take(R);
  p->o_info = take(8);  // an iteration record per mode
  for (int n = 0; n < 3; ++n) p->o_Astart[n] = take(dims[n] * R);
  p->o_stats = take(8);
  size_t prep = 1, part = 1;
  for (const Contr& k : all_contractions(p)) {
    const Level1Geom g = l1_geom(k.P, k.K, k.Q, p->R, DT_F64);
    prep = std::max(prep, prep_elems(g));
    part = std::max(part, part_elems(g));
  }
  {
    const Level1Geom g = middle_unfolding_geom(p);
    prep = std::max(prep, prep_elems(g));
    part = std::max(part, part_elems(g));
  }
  p->o_prep = take(prep);
  p->o_part = take(std::max<size_t>(part, 1024));
  p->o_gpart = take((size_t)kMaxGemmSplit * 3 * R * R);
  // HOSVD intermediate X_(n)^T V: the largest of s2 s3, s1 s3, s1 s2 times R
  p->o_Zx = take(std::max(s1 * s2, std::max(s0 * s2, s0 * s1)) * R);
  p->ws_bytes = off;
  *out = p;
  return PPALS_OK;
}

void tucker_plan_destroy(tucker_plan* plan) { delete plan; }

size_t tucker_workspace_bytes(const tucker_plan* plan) { return plan ? plan->ws_bytes : 0; }

ppals_status tucker_set_solver(tucker_plan* plan, double tol, int32_t max_iters,
                               int32_t hosvd_max_iters) {
  if (!plan) return set_error(PPALS_E_ARG, "NULL plan");
  if (!(tol > 0.0) || max_iters < 1 || hosvd_max_iters < 1)
    return set_error(PPALS_E_ARG, "need tol > 0 and iteration limits >= 1");
  plan->tol = tol;
  plan->max_iters = max_iters;
  plan->hosvd_iters = hosvd_max_iters;
  return PPALS_OK;
}

ppals_status tucker_ttmc(tucker_plan* plan, void* ws, const double* X, double* const* A,
                         int32_t mode, double* Y, hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  if (!X || !Y) return set_error(PPALS_E_ARG, "NULL argument");
  if (mode < 0 || mode > 2) return set_error(PPALS_E_ARG, "mode must be 0, 1 or 2");
  TCtx c{plan, (char*)ws, stream};
  return als_ttmc(c, X, A, mode, true, Y);
}

ppals_status tucker_factor_update(tucker_plan* plan, void* ws, const double* Y, int32_t mode,
                                  const double* A_prev, double* A_out, int32_t* info,
                                  double* residual, hipStream_t stream) {
  TCHK(check_common(plan, ws));
  if (!Y || !A_prev || !A_out) return set_error(PPALS_E_ARG, "NULL argument");
  if (mode < 0 || mode > 2) return set_error(PPALS_E_ARG, "mode must be 0, 1 or 2");
  TCtx c{plan, (char*)ws, stream};
  double* Aold = c.d(plan->o_Aold);
  THIPCHK(launch_copy(Aold, A_prev, plan->s[mode] * plan->R, stream));
  return subspace(c, mode, Y, nullptr, Aold, Aold, A_out, plan->max_iters, info, residual);
}

ppals_status tucker_hosvd(tucker_plan* plan, void* ws, const double* X, double* const* V0,
                          double* const* A, double* G, int32_t* info, hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  TCHK(check_factors(plan, V0));
  if (!X || !G) return set_error(PPALS_E_ARG, "NULL argument");
  TCtx c{plan, (char*)ws, stream};
  for (int n = 0; n < 3; ++n)
    TCHK(subspace(c, n, nullptr, X, V0[n], nullptr, A[n], plan->hosvd_iters,
                  info ? info + 3 * n : nullptr, nullptr));
  const int64_t s0 = plan->s[0], s1 = plan->s[1], s2 = plan->s[2], R = plan->R;
  double* T1 = c.d(plan->o_T1);
  double* Y = c.d(plan->o_Y);
  TCHK(ttm(c, X, {1, s0, s1 * s2}, A[0], T1));    // (x2, x3, r1)
  TCHK(ttm(c, T1, {1, s1, s2 * R}, A[1], Y));     // (x3, r1, r2)
  TCHK(ttm(c, Y, {1, s2, R * R}, A[2], G));       // (r1, r2, r3)
  THIPCHK(hipStreamSynchronize(stream));
  plan->built = false;
  return PPALS_OK;
}

ppals_status tucker_als_sweep(tucker_plan* plan, void* ws, const double* X, double* const* A,
                              double* G, double normX2, tucker_sweep_record* rec,
                              hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  if (!X || !G || !rec) return set_error(PPALS_E_ARG, "NULL argument");
  if (!(normX2 > 0.0)) return set_error(PPALS_E_ARG, "normX2 must be positive");
  const double t0 = now_ms();
  TCtx c{plan, (char*)ws, stream};
  memset(rec, 0, sizeof(*rec));
  double* Y = c.d(plan->o_Y);
  double* Aold = c.d(plan->o_Aold);
  double* stats = c.d(plan->o_stats);
  const int R = plan->R;
  for (int n = 0; n < 3; ++n) {
    TCHK(als_ttmc(c, X, A, n, n == 0, Y));
    THIPCHK(launch_copy(Aold, A[n], plan->s[n] * R, stream));
    int32_t info[3];
    TCHK(subspace(c, n, Y, nullptr, Aold, Aold, A[n], plan->max_iters, info,
                  &rec->ritz_residual[n]));
    rec->iters[n] = info[0];
    rec->converged[n] = info[1];
    rec->rr_status[n] = info[2];
    THIPCHK(launch_core_stats(A[n], Aold, plan->s[n] * R, stats + 2 * n, stream));
  }
  TCHK(finish_core(c, Y, A[2], G));
  double h[8];
  THIPCHK(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, stream));
  THIPCHK(hipStreamSynchronize(stream));
  fill_record(plan, h, normX2, PPALS_SWEEP_ALS, rec);
  rec->ms = now_ms() - t0;
  return PPALS_OK;
}

ppals_status tucker_pp_build(tucker_plan* plan, void* ws, const double* X, double* const* A,
                             hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  if (!X) return set_error(PPALS_E_ARG, "NULL argument");
  TCtx c{plan, (char*)ws, stream};
  const int64_t s0 = plan->s[0], s1 = plan->s[1], s2 = plan->s[2], R = plan->R;
  double* op01 = c.d(plan->o_op01);
  double* op02 = c.d(plan->o_op02);
  double* op12 = c.d(plan->o_op12);
  for (int n = 0; n < 3; ++n) {
    THIPCHK(launch_copy(c.d(plan->o_Ap[n]), A[n], plan->s[n] * R, stream));
    THIPCHK(launch_fill(c.d(plan->o_dA[n]), 0.0, plan->s[n] * R, stream));
    plan->dA_zero[n] = true;
  }
  TCHK(ttm(c, X, {s0 * s1, s2, 1}, A[2], op01));          // (x1, x2, r3)
  TCHK(ttm(c, X, {s0, s1, s2}, A[1], op02));              // (x1, x3, r2)
  TCHK(ttm(c, X, {1, s0, s1 * s2}, A[0], op12));          // (x2, x3, r1)
  TCHK(ttm(c, op01, {s0, s1, R}, A[1], c.d(plan->o_Yp[0])));      // (x1, r3, r2)
  TCHK(ttm(c, op01, {1, s0, s1 * R}, A[0], c.d(plan->o_Yp[1])));  // (x2, r3, r1)
  TCHK(ttm(c, op12, {1, s1, s2 * R}, A[1], c.d(plan->o_Yp[2])));  // (x3, r1, r2)
  plan->built = true;
  plan->built_ws = ws;
  plan->pp_optimistic = true;
  return PPALS_OK;
}

ppals_status tucker_pp_rhs(tucker_plan* plan, void* ws, int32_t mode, double* Y,
                           hipStream_t stream) {
  TCHK(check_common(plan, ws));
  if (!Y) return set_error(PPALS_E_ARG, "NULL argument");
  if (mode < 0 || mode > 2) return set_error(PPALS_E_ARG, "mode must be 0, 1 or 2");
  if (!plan->built || plan->built_ws != ws)
    return set_error(PPALS_E_STATE, "tucker_pp_rhs before tucker_pp_build on this workspace");
  TCtx c{plan, (char*)ws, stream};
  return pp_rhs_impl(c, mode, Y);
}

ppals_status tucker_pp_sweep(tucker_plan* plan, void* ws, double* const* A, double* G,
                             double normX2, int32_t kind, tucker_sweep_record* rec,
                             hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  if (!G || !rec) return set_error(PPALS_E_ARG, "NULL argument");
  if (!(normX2 > 0.0)) return set_error(PPALS_E_ARG, "normX2 must be positive");
  if (kind != PPALS_SWEEP_PP_INIT && kind != PPALS_SWEEP_PP_APPROX)
    return set_error(PPALS_E_ARG, "kind must be PP_INIT or PP_APPROX");
  if (!plan->built || plan->built_ws != ws)
    return set_error(PPALS_E_STATE, "tucker_pp_sweep before tucker_pp_build on this workspace");
  const double t0 = now_ms();
  TCtx c{plan, (char*)ws, stream};
  memset(rec, 0, sizeof(*rec));
  double* Y = c.d(plan->o_Y);
  double* Aold = c.d(plan->o_Aold);
  double* stats = c.d(plan->o_stats);
  const int R = plan->R;
  IterInfo* dinfo = reinterpret_cast<IterInfo*>(c.ws + plan->o_info);
  int n0 = 0;  // first mode of the synchronised pass
  if (plan->pp_optimistic) {
    // One subspace iteration per mode with no host synchronisation; the residuals are
    // read once at the end.  If a mode did not converge, that mode and the later ones are
    // restored and redone below with a check after every iteration (same launches in the
    // same order, so the result does not depend on the path).
    bool zero_start[3];
    for (int n = 0; n < 3; ++n) {
      zero_start[n] = plan->dA_zero[n];
      THIPCHK(launch_copy(c.d(plan->o_Astart[n]), A[n], plan->s[n] * R, stream));
    }
    for (int n = 0; n < 3; ++n) {
      TCHK(pp_rhs_impl(c, n, Y));
      THIPCHK(launch_copy(Aold, A[n], plan->s[n] * R, stream));
      THIPCHK(launch_copy(c.d(plan->o_V), Aold, plan->s[n] * R, stream));
      TCHK(subspace_step(c, n, Y, nullptr, true, dinfo + n));
      THIPCHK(launch_copy(A[n], c.d(plan->o_U), plan->s[n] * R, stream));
      double* dA = c.d(plan->o_dA[n]);
      const double* Ap = c.d(plan->o_Ap[n]);
      THIPCHK(launch_sub(dA, A[n], Ap, plan->s[n] * R, stream));
      plan->dA_zero[n] = false;
      THIPCHK(launch_core_stats(A[n], Ap, plan->s[n] * R, stats + 2 * n, stream));
    }
    TCHK(finish_core(c, Y, A[2], G, false));
    IterInfo hi[3];
    THIPCHK(hipMemcpyAsync(hi, dinfo, sizeof(hi), hipMemcpyDeviceToHost, stream));
    THIPCHK(hipStreamSynchronize(stream));
    n0 = 3;
    for (int n = 2; n >= 0; --n)
      if (!(hi[n].residual <= plan->tol)) n0 = n;
    for (int n = 0; n < n0; ++n) {
      rec->iters[n] = 1;
      rec->converged[n] = 1;
      rec->rr_status[n] = hi[n].rr_bad;
      rec->ritz_residual[n] = hi[n].residual;
    }
    if (n0 == 3) {
      THIPCHK(launch_copy(G, c.d(plan->o_Gn), (int64_t)R * R * R, stream));
    } else {
      plan->pp_optimistic = false;
      for (int n = n0; n < 3; ++n) {
        THIPCHK(launch_copy(A[n], c.d(plan->o_Astart[n]), plan->s[n] * R, stream));
        THIPCHK(launch_sub(c.d(plan->o_dA[n]), A[n], c.d(plan->o_Ap[n]), plan->s[n] * R, stream));
        plan->dA_zero[n] = zero_start[n];
      }
    }
  }
  if (n0 < 3) {
    for (int n = n0; n < 3; ++n) {
      TCHK(pp_rhs_impl(c, n, Y));
      THIPCHK(launch_copy(Aold, A[n], plan->s[n] * R, stream));
      int32_t info[3];
      TCHK(subspace(c, n, Y, nullptr, Aold, Aold, A[n], plan->max_iters, info,
                    &rec->ritz_residual[n]));
      rec->iters[n] = info[0];
      rec->converged[n] = info[1];
      rec->rr_status[n] = info[2];
      double* dA = c.d(plan->o_dA[n]);
      const double* Ap = c.d(plan->o_Ap[n]);
      THIPCHK(launch_sub(dA, A[n], Ap, plan->s[n] * R, stream));
      plan->dA_zero[n] = false;
      THIPCHK(launch_core_stats(A[n], Ap, plan->s[n] * R, stats + 2 * n, stream));
    }
    TCHK(finish_core(c, Y, A[2], G));
    // back to the unsynchronised pass once a sweep needs a single iteration everywhere
    plan->pp_optimistic = rec->iters[0] == 1 && rec->iters[1] == 1 && rec->iters[2] == 1;
  }
  double h[8];
  THIPCHK(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, stream));
  THIPCHK(hipStreamSynchronize(stream));
  fill_record(plan, h, normX2, kind, rec);
  rec->ms = now_ms() - t0;
  return PPALS_OK;
}

ppals_status tucker_run(tucker_plan* plan, void* ws, const double* X, double* const* A,
                        double* G, double eps, int32_t sweeps, double delta,
                        const int32_t* replay, int32_t replay_len, tucker_sweep_record* recs,
                        int32_t* n_out, hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  if (!X || !G || !recs || !n_out) return set_error(PPALS_E_ARG, "NULL argument");
  if (sweeps < 0) return set_error(PPALS_E_ARG, "sweeps must be >= 0");
  if (!(eps >= 0.0)) return set_error(PPALS_E_ARG, "eps must be >= 0");
  *n_out = 0;
  const int64_t count = plan->s[0] * plan->s[1] * plan->s[2];
  const int64_t R3 = (int64_t)plan->R * plan->R * plan->R;
  double* stats = reinterpret_cast<double*>((char*)ws + plan->o_stats);
  // ||X||^2 with the multi-workgroup reduction (partials in the level-1 partial region)
  THIPCHK(launch_norm2(X, DT_F64, count, reinterpret_cast<double*>((char*)ws + plan->o_part), 1024,
                       stats, stream));
  THIPCHK(launch_core_stats(G, G, R3, stats + 2, stream));
  double h[4];
  THIPCHK(hipMemcpyAsync(h, stats, sizeof(h), hipMemcpyDeviceToHost, stream));
  THIPCHK(hipStreamSynchronize(stream));
  const double normX2 = h[0];
  if (!(normX2 > 0.0)) return set_error(PPALS_E_ARG, "X must be nonzero");
  const double normX = std::sqrt(normX2);
  int n = 0;
  if (replay) {
    const int len = std::min<int>(replay_len, sweeps);
    for (int k = 0; k < len; ++k) {
      const int kind = replay[k];
      if (kind == PPALS_SWEEP_ALS) {
        TCHK(tucker_als_sweep(plan, ws, X, A, G, normX2, &recs[n], stream));
      } else if (kind == PPALS_SWEEP_PP_INIT) {
        TCHK(tucker_pp_build(plan, ws, X, A, stream));
        TCHK(tucker_pp_sweep(plan, ws, A, G, normX2, kind, &recs[n], stream));
      } else if (kind == PPALS_SWEEP_PP_APPROX) {
        TCHK(tucker_pp_sweep(plan, ws, A, G, normX2, kind, &recs[n], stream));
      } else {
        return set_error(PPALS_E_ARG, "unknown sweep kind in replay");
      }
      *n_out = ++n;
    }
    return PPALS_OK;
  }
  double rel[3] = {1.0, 1.0, 1.0};  // dA = A initially
  double f_norm = std::sqrt(h[2]);
  auto stopped = [&]() { return delta > 0.0 && n > 0 && recs[n - 1].f_norm <= delta * normX; };
  while (n < sweeps && !stopped()) {
    if (rel[0] < eps && rel[1] < eps && rel[2] < eps && f_norm < eps * normX) {
      TCHK(tucker_pp_build(plan, ws, X, A, stream));
      int kind = PPALS_SWEEP_PP_INIT;
      while (n < sweeps && f_norm < eps * normX && !stopped()) {
        TCHK(tucker_pp_sweep(plan, ws, A, G, normX2, kind, &recs[n], stream));
        f_norm = recs[n].f_norm;
        for (int i = 0; i < 3; ++i) rel[i] = recs[n].rel_change[i];
        *n_out = ++n;
        kind = PPALS_SWEEP_PP_APPROX;
      }
      if (n >= sweeps || stopped()) break;
    }
    TCHK(tucker_als_sweep(plan, ws, X, A, G, normX2, &recs[n], stream));
    f_norm = recs[n].f_norm;
    for (int i = 0; i < 3; ++i) rel[i] = recs[n].rel_change[i];
    *n_out = ++n;
  }
  return PPALS_OK;
}

}  // extern "C"
