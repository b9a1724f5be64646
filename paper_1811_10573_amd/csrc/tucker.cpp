// Tucker-ALS and PP-Tucker-ALS for tensors of order 3 to 8 (Algorithms 2 and 4), FP64.
//
// Every TTM is a first-level contraction (k_level1.hip).  A partly contracted tensor is
// kept as its remaining original modes, in order, followed by the rank indices made so
// far; contracting original mode m is then a P x K x Q contraction (P: the remaining modes
// before m; K = s_m; Q: the remaining modes after m times the ranks) whose new rank index
// lands last.  Contracting modes in increasing order gives every TTMc its canonical
// layout: the kept mode(s) first, then the rank indices in increasing mode order.
//
// The factor update is a subspace iteration on W = Y_(n) Y_(n)^T whose products W V are
// applied as Y_(n) (Y_(n)^T V), two more first-level contractions; the small R x R algebra
// (Rayleigh-Ritz with Jacobi rotations) is one workgroup (k_tucker.hip).
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

constexpr int TMAX = PPALS_MAX_ORDER;

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

struct Contr {  // a first-level contraction P x K x Q (K contracted)
  int64_t P, K, Q;
};

// Layout of a partly contracted tensor: the remaining original modes (increasing) and
// the number of rank indices appended after them.
struct Lay {
  std::vector<int> modes;
  int nr = 0;
};

// What a schedule would launch, gathered without launching (workspace sizes).
struct Collector {
  size_t prep = 1, part = 1024;  // elements of the operand and split-partial regions
  int64_t tmp = 1;               // largest intermediate of a contraction chain
  int64_t lvl[8] = {1, 1, 1, 1, 1, 1, 1, 1};  // largest node of the operator tree per depth
};

}  // namespace

struct tucker_plan {
  int N = 0;
  int64_t s[TMAX] = {0};
  int R = 0;
  int64_t rpow[TMAX + 1] = {0};  // R^k
  double tol = 1e-12;
  int max_iters = 500;
  int hosvd_iters = 5000;
  // workspace regions (byte offsets)
  size_t o_pre[2], o_tmp[2];       // prefix chain and chain temporaries
  size_t o_F[3];                   // X x_c A_p^(c), c = 0, 1, 2 (operator build)
  size_t o_lvl[8] = {0};           // operator tree: one node of each depth >= 2 at a time
  size_t o_op[TMAX][TMAX];         // Y_p^(i,n), i < n
  size_t o_Yp[TMAX], o_Y, o_term[TMAX], o_Gn;
  size_t o_Ap[TMAX], o_dA[TMAX], o_Astart[TMAX];
  size_t o_dAprep[TMAX];           // dA^(i) in the first-level operand order (dA_geom)
  size_t o_V, o_C, o_Aold, o_U, o_Z, o_B, o_H, o_P, o_T, o_lam, o_info, o_stats;
  size_t o_prep, o_part, o_gpart, o_rpart;
  size_t slot = 0;  // bytes between the basis slots V, C, A_prev
  size_t ws_bytes = 0;
  bool built = false;
  bool dA_zero[TMAX];
  bool pp_optimistic = true;  // PP sweeps: one unchecked subspace iteration per mode first
  void* built_ws = nullptr;
};

namespace {

struct TCtx {
  tucker_plan* p;
  char* ws;
  hipStream_t s;
  Collector* col = nullptr;  // set: gather sizes only, launch nothing
  double* d(size_t off) const { return reinterpret_cast<double*>(ws + off); }
};

int64_t numel(const tucker_plan* p, const Lay& L) {
  int64_t v = p->rpow[L.nr];
  for (int m : L.modes) v *= p->s[m];
  return v;
}

// Contracting original mode m of a tensor with layout L, and the layout after it.
Contr contr_of(const tucker_plan* p, const Lay& L, int m) {
  Contr k{1, p->s[m], p->rpow[L.nr]};
  bool after = false;
  for (int q : L.modes) {
    if (q == m) after = true;
    else if (after) k.Q *= p->s[q];
    else k.P *= p->s[q];
  }
  return k;
}
Lay lay_after(const Lay& L, int m) {
  Lay o;
  for (int q : L.modes)
    if (q != m) o.modes.push_back(q);
  o.nr = L.nr + 1;
  return o;
}
Lay lay_all(const tucker_plan* p) {
  Lay L;
  for (int m = 0; m < p->N; ++m) L.modes.push_back(m);
  return L;
}

size_t prep_elems(const Level1Geom& g) { return (size_t)g.nslices * g.Kpad * 16 * g.NB; }
size_t part_elems(const Level1Geom& g) {
  return g.ksplit > 1 ? (size_t)g.ksplit * g.M * g.R : 0;
}

// out (M x R) = first-level contraction of T with the K x R factor F under geometry g
ppals_status ttm_geom(const TCtx& c, const double* T, const Level1Geom& g, const double* F,
                      double* out) {
  if (c.col) {
    c.col->prep = std::max(c.col->prep, prep_elems(g));
    c.col->part = std::max(c.col->part, part_elems(g));
    return PPALS_OK;
  }
  if (!g.strided && ttm_small_r_fits(g.M, g.K, g.Q, c.p->R)) {
    THIPCHK(launch_ttm_small_r(T, F, g.M, g.K, g.Q, c.p->R, out, c.s));
    return PPALS_OK;
  }
  // Few rows over a long k: rows contiguous (Q = 1), or the inner-mode unfolding of
  // inner_unfolding_geom (row stride `after` = ms1, k = c_before after + c_after).  The
  // part region holds ksplit x M x R doubles (sized from this geometry).
  const bool inner = g.strided && g.ms0 == 0 && g.ms2 == 0 && g.mrad2 == 1 && g.ks1 == 0 &&
                     g.ks2 == 1 && g.ms1 >= 1 && g.ks0 == g.M * g.ms1 && g.kr1 == 1 &&
                     (int64_t)g.kr2 == g.ms1;
  const int64_t after = inner ? g.ms1 : g.K;
  const int nparts = (inner || (!g.strided && g.Q == 1)) && g.ksplit > 1
                         ? ttm_rows_small_r_parts(g.M, g.K, c.p->R, g.ksplit) : 0;
  if (nparts > 0) {
    THIPCHK(launch_ttm_rows_small_r(T, F, g.M, g.K, after, c.p->R, nparts,
                                    reinterpret_cast<double*>(c.ws + c.p->o_part), out, c.s));
    return PPALS_OK;
  }
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

ppals_status ttm(const TCtx& c, const double* T, Contr k, const double* F, double* out) {
  return ttm_geom(c, T, l1_geom(k.P, k.K, k.Q, c.p->R, DT_F64), F, out);
}

// Operand order of dA^(i) kept between its update and the correction terms that read it:
// the order of a contraction over s_i whose trailing extent is not 1.  The operand order
// depends only on K, R and whether that extent is 1.
Level1Geom dA_geom(const tucker_plan* p, int i) { return l1_geom(1, p->s[i], 2, p->R, DT_F64); }
bool same_operand_order(const Level1Geom& a, const Level1Geom& b) {
  return a.K == b.K && a.Kpad == b.Kpad && a.nslices == b.nslices && a.NB == b.NB &&
         a.kc_mode == b.kc_mode;
}
ppals_status prep_dA(const TCtx& c, int i) {
  if (c.col) return PPALS_OK;
  KrpDesc krp;
  memset(&krp, 0, sizeof(krp));
  krp.nf = 1;
  krp.R = c.p->R;
  krp.A[0] = c.d(c.p->o_dA[i]);
  krp.dim[0] = c.p->s[i];
  THIPCHK(launch_prep_operand(krp, dA_geom(c.p, i), DT_F64, c.ws + c.p->o_dAprep[i], c.s));
  return PPALS_OK;
}

// Contract the modes ms (increasing) of src (layout L) with the factors F[m]: the result
// goes to dst, the intermediate steps alternate between the two temporaries.
ppals_status chain(const TCtx& c, const double* src, Lay L, const std::vector<int>& ms,
                   const double* const* F, double* dst) {
  const double* cur = src;
  for (size_t k = 0; k < ms.size(); ++k) {
    const bool last = k + 1 == ms.size();
    double* out = last ? dst : c.d(c.p->o_tmp[k & 1]);
    TCHK(ttm(c, cur, contr_of(c.p, L, ms[k]), F[ms[k]], out));
    L = lay_after(L, ms[k]);
    if (!last && c.col) c.col->tmp = std::max(c.col->tmp, numel(c.p, L));
    cur = out;
  }
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
  if (c.col) return PPALS_OK;
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

// The product X_(n) Z of the HOSVD for a mode n strictly inside: C[x_n][r] = sum over the
// other modes of X[.., x_n, ..] Z[(before, after)][r], a first-level contraction whose rows
// (x_n) and contracted index (the modes before n, then the modes after n) reach X through
// strided offsets.
Level1Geom inner_unfolding_geom(const tucker_plan* p, int n) {
  int64_t before = 1, after = 1;
  for (int m = 0; m < n; ++m) before *= p->s[m];
  for (int m = n + 1; m < p->N; ++m) after *= p->s[m];
  Level1Geom g = l1_geom(p->s[n], before * after, 1, p->R, DT_F64);
  g.kc_mode = 0;
  g.Q = 1;
  g.strided = 1;
  g.mrad = p->s[n];  // row m = x_n: offset x_n * after
  g.mrad2 = 1;
  g.ms0 = 0;
  g.ms1 = after;
  g.ms2 = 0;
  g.kr1 = 1;         // k = c_before * after + c_after: offset c_before s_n after + c_after
  g.kr2 = (uint32_t)after;
  l1_magic(g.kr1, &g.kmag1, &g.ksh1);
  l1_magic(g.kr2, &g.kmag2, &g.ksh2);
  g.ks0 = p->s[n] * after;
  g.ks1 = 0;
  g.ks2 = 1;
  return g;
}

// C = W V for the subspace iteration of mode n: through a TTMc Y (W = Y_(n) Y_(n)^T, Y
// given) or, for the HOSVD (Y null), through X itself (W = X_(n) X_(n)^T) with the
// intermediate Z = X_(n)^T V in a chain temporary.
// With npart non-null the chunked product may leave C as *npart <= kRRSmallParts slots in
// the partial region (*npart = 0: C written).
// X: the tensor with layout XL (null: X itself, every mode), mode n contracted around;
// n is the first remaining mode of XL unless XL is null.
ppals_status apply_w(const TCtx& c, int n, const double* Y, const double* X, const double* V,
                     double* C, int* npart = nullptr, const Lay* XL = nullptr) {
  tucker_plan* p = c.p;
  const int N = p->N;
  const int64_t sn = p->s[n], RN1 = p->rpow[N - 1];
  if (npart) *npart = 0;
  if (Y) {
    const int w = w_apply_width(sn, RN1, p->R);
    if (w > 0) {  // one pass over the small TTMc: C = Y (Y^T V) chunk by chunk
      const int64_t nchunk = (RN1 + w - 1) / w;
      if (c.col) {
        c.col->part = std::max(c.col->part, (size_t)(nchunk * sn * p->R));
        return PPALS_OK;
      }
      if (npart && nchunk <= kRRSmallParts) {
        THIPCHK(launch_w_apply_parts(Y, V, sn, RN1, p->R, w, c.d(p->o_part), c.s));
        *npart = (int)nchunk;
      } else {
        THIPCHK(launch_w_apply(Y, V, sn, RN1, p->R, w, c.d(p->o_part), C, c.s));
      }
      return PPALS_OK;
    }
    double* Z = c.d(p->o_Z);
    TCHK(ttm(c, Y, {1, sn, RN1}, V, Z));  // Z = Y^T V   (R^(N-1) x R)
    TCHK(ttm(c, Y, {sn, RN1, 1}, Z, C));  // C = Y Z     (s_n x R)
    return PPALS_OK;
  }
  double* Zx = c.d(p->o_tmp[0]);
  const Lay L = XL ? *XL : lay_all(p);
  const Contr k = contr_of(p, L, n);
  if (c.col) c.col->tmp = std::max(c.col->tmp, k.P * k.Q * p->R);
  TCHK(ttm(c, X, k, V, Zx));  // (other modes, r)
  const int64_t others = k.P * k.Q;
  if (k.P == 1) TCHK(ttm(c, X, {sn, others, 1}, Zx, C));       // n first
  else if (k.Q == 1) TCHK(ttm(c, X, {1, others, sn}, Zx, C));  // n last, no ranks after
  else TCHK(ttm_geom(c, X, inner_unfolding_geom(p, n), Zx, C));
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
                           IterInfo* info, const Lay* XL = nullptr) {
  tucker_plan* p = c.p;
  const int R = p->R;
  const int64_t sn = p->s[n];
  double* V = c.d(p->o_V);
  double* C = c.d(p->o_C);
  const bool small = rr_small_fits(sn, R);
  int npart = 0;
  TCHK(apply_w(c, n, Y, X, V, C, small ? &npart : nullptr, XL));  // C = W V
  if (c.col) return PPALS_OK;
  RRArgs rr;
  memset(&rr, 0, sizeof(rr));
  if (small) {  // projections, Rayleigh-Ritz and Ritz update in one workgroup
    rr.R = R;
    rr.V = V;
    rr.Vout = V;
    rr.C = C;
    rr.Ap = has_prev ? c.d(p->o_Aold) : nullptr;
    rr.rows = sn;
    rr.T = c.d(p->o_T);
    rr.lam = c.d(p->o_lam);
    rr.status = &info->rr_bad;
    rr.U = c.d(p->o_U);
    rr.residual = &info->residual;
    if (npart > 0) {
      rr.cpart = c.d(p->o_part);
      rr.npart = npart;
      rr.pstride = sn * R;
    }
    THIPCHK(launch_rr_small(rr, c.s));
    return PPALS_OK;
  }
  TCHK(projections(c, sn, has_prev ? 3 : 2));
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

// Subspace iteration for the R leading eigenvectors of W (s_n x s_n), W = Y_(n) Y_(n)^T for
// a TTMc Y or, with Y null, X_(n) X_(n)^T (the HOSVD).  V starts from V0; A_prev (may be
// null) orients the columns.  Result into A_out.  Synchronises once per iteration.
ppals_status subspace(const TCtx& c, int n, const double* Y, const double* X, const double* V0,
                      const double* A_prev, double* A_out, int max_iters, int32_t* info,
                      double* residual, const Lay* XL = nullptr) {
  tucker_plan* p = c.p;
  if (c.col) {
    IterInfo dummy;
    return subspace_step(c, n, Y, X, A_prev != nullptr, &dummy, XL);
  }
  const int R = p->R;
  const int64_t sn = p->s[n];
  double* Aold = c.d(p->o_Aold);
  IterInfo* dinfo = reinterpret_cast<IterInfo*>(c.ws + p->o_info) + n;
  if (A_prev && A_prev != Aold) THIPCHK(launch_copy(Aold, A_prev, sn * R, c.s));
  THIPCHK(launch_copy(c.d(p->o_V), V0, sn * R, c.s));
  IterInfo hinfo;
  memset(&hinfo, 0, sizeof(hinfo));
  int it = 0, bad = 0;
  bool conv = false;
  while (it < max_iters) {
    ++it;
    TCHK(subspace_step(c, n, Y, X, A_prev != nullptr, dinfo, XL));
    THIPCHK(hipMemcpyAsync(&hinfo, dinfo, sizeof(hinfo), hipMemcpyDeviceToHost, c.s));
    THIPCHK(hipStreamSynchronize(c.s));
    bad |= hinfo.rr_bad;
    if (hinfo.residual <= p->tol) {
      conv = true;
      break;
    }
  }
  THIPCHK(launch_copy(A_out, c.d(p->o_U), sn * R, c.s));
  if (!A_prev) THIPCHK(launch_sign_by_max(A_out, sn, R, c.s));
  if (info) {
    info[0] = it;
    info[1] = conv ? 1 : 0;
    info[2] = bad;
  }
  if (residual) *residual = hinfo.residual;
  return PPALS_OK;
}

// The prefix chain P_n = X x_0 A^(0)T .. x_(n-1) A^(n-1)T, held in o_pre[n % 2], layout
// (x_n, .., x_(N-1), r_0, .., r_(n-1)).
Lay prefix_lay(const tucker_plan* p, int n) {
  Lay L;
  for (int m = n; m < p->N; ++m) L.modes.push_back(m);
  L.nr = n;
  return L;
}

// Y^(n) of an ALS sweep from the prefix P_n (X for n = 0), the later modes contracted
// with their current factors.  For n = N - 1 the prefix itself is Y^(N-1): *Y points to it.
ppals_status als_ttmc(const TCtx& c, const double* X, const double* const* A, int n,
                      const double** Y) {
  tucker_plan* p = c.p;
  const int N = p->N;
  if (n == N - 1) {
    *Y = c.d(p->o_pre[n & 1]);
    return PPALS_OK;
  }
  const double* src = n == 0 ? X : c.d(p->o_pre[n & 1]);
  std::vector<int> ms;
  for (int m = n + 1; m < N; ++m) ms.push_back(m);
  TCHK(chain(c, src, prefix_lay(p, n), ms, A, c.d(p->o_Y)));
  *Y = c.d(p->o_Y);
  return PPALS_OK;
}

// P_(n+1) = P_n x_n A^(n)T (P_0 = X).
ppals_status extend_prefix(const TCtx& c, const double* X, const double* const* A, int n) {
  tucker_plan* p = c.p;
  const double* src = n == 0 ? X : c.d(p->o_pre[n & 1]);
  const Lay L = prefix_lay(p, n);
  return ttm(c, src, contr_of(p, L, n), A[n], c.d(p->o_pre[(n + 1) & 1]));
}

// Core from Y^(N-1) (x_(N-1), r_0 .. r_(N-2)) and A^(N-1): G (r_0 .. r_(N-1)); stats[2N],
// stats[2N+1] = ||G||^2, ||G - G_old||^2; G_old <- G when commit.
ppals_status finish_core(const TCtx& c, const double* Y, const double* A_last, double* G,
                         bool commit = true) {
  tucker_plan* p = c.p;
  const int N = p->N;
  const int64_t RN = p->rpow[N];
  double* Gn = c.d(p->o_Gn);
  TCHK(ttm(c, Y, {1, p->s[N - 1], p->rpow[N - 1]}, A_last, Gn));
  if (c.col) return PPALS_OK;
  THIPCHK(launch_core_stats(Gn, G, RN, c.d(p->o_stats) + 2 * N, c.s));
  if (commit) THIPCHK(launch_copy(G, Gn, RN, c.s));
  return PPALS_OK;
}

void fill_record(const tucker_plan* p, const double* stats, double normX2, int kind,
                 tucker_sweep_record* rec) {
  const int N = p->N;
  rec->kind = kind;
  for (int n = 0; n < N; ++n) {
    const double a2 = stats[2 * n], d2 = stats[2 * n + 1];
    rec->rel_change[n] = a2 > 0.0 ? std::sqrt(d2) / std::sqrt(a2) : 0.0;
  }
  const double g2 = stats[2 * N];
  rec->core_norm = std::sqrt(g2);
  rec->f_norm = std::sqrt(stats[2 * N + 1]);
  rec->fit = 1.0 - std::sqrt(std::max(0.0, normX2 - g2)) / std::sqrt(normX2);
}

ppals_status check_common(tucker_plan* p, void* ws) {
  if (!p) return set_error(PPALS_E_ARG, "NULL plan");
  if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255))
    return set_error(PPALS_E_WORKSPACE, "workspace NULL or not 256-byte aligned");
  return PPALS_OK;
}

ppals_status check_factors(const tucker_plan* p, double* const* A) {
  if (!A) return set_error(PPALS_E_ARG, "NULL factor array");
  for (int n = 0; n < p->N; ++n)
    if (!A[n]) return set_error(PPALS_E_ARG, "NULL factor " + std::to_string(n));
  return PPALS_OK;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Position of mode i among the rank indices of Y^(n) (the modes other than n, increasing).
int rank_pos(int i, int n) { return i < n ? i : i - 1; }

// Y_p^(i,n) (i != n) contracted over x_i with an s_i x R factor: result (x_n, ranks of
// the modes other than i and n, r_i).
Contr op_contr(const tucker_plan* p, int i, int n) {
  const int64_t RN2 = p->rpow[p->N - 2];
  if (i < n) return {1, p->s[i], p->s[n] * RN2};  // operator (x_i, x_n, ..)
  return {p->s[n], p->s[i], RN2};                 // operator (x_n, x_i, ..)
}

TuckerCombine combine_args(const tucker_plan* p, int n, double* out, const double* base) {
  TuckerCombine a;
  memset(&a, 0, sizeof(a));
  a.out = out;
  a.base = base;
  a.nd = p->N - 1;
  a.R = p->R;
  a.rows = p->s[n];
  a.cols = p->rpow[p->N - 1];
  for (int k = 0; k <= TMAX; ++k) a.rpow[k] = p->rpow[k];
  return a;
}

// out = base + the terms Y_p^(i,n) x_i F_i^T (terms in list order, F_i an s_i x R matrix)
// in one in-place launch when its multiply-adds stay below kPPRhsInPlaceMax (*done), else
// nothing (the caller contracts term by term).
ppals_status pp_rhs_in_place(const TCtx& c, int n, const int* is, const double* const* F, int nt,
                             const double* base, double* out, bool* done) {
  tucker_plan* p = c.p;
  const int N = p->N;
  const int64_t RN2 = p->rpow[N - 2], cols = p->rpow[N - 1];
  int64_t work = 0;
  for (int t = 0; t < nt; ++t) work += p->s[is[t]] * p->s[n] * cols;
  *done = work <= kPPRhsInPlaceMax;
  if (!*done || c.col) return PPALS_OK;
  TuckerPPRhs a;
  memset(&a, 0, sizeof(a));
  a.out = out;
  a.base = base;
  a.nd = N - 1;
  a.R = p->R;
  a.rows = p->s[n];
  a.cols = cols;
  for (int k = 0; k <= TMAX; ++k) a.rpow[k] = p->rpow[k];
  for (int t = 0; t < nt; ++t) {
    const int i = is[t];
    a.op[t] = c.d(p->o_op[std::min(i, n)][std::max(i, n)]);
    a.F[t] = F[t];
    a.klen[t] = p->s[i];
    if (i < n) {  // operator (x_i, x_n, ..)
      a.kstride[t] = p->s[n] * RN2;
      a.nstride[t] = RN2;
    } else {      // operator (x_n, x_i, ..)
      a.kstride[t] = RN2;
      a.nstride[t] = p->s[i] * RN2;
    }
    a.pos[t] = rank_pos(i, n);
  }
  a.nterms = nt;
  THIPCHK(launch_tucker_pp_rhs(a, c.s));
  return PPALS_OK;
}

// First-order PP TTMc of mode n into Y from the operators and dA (Section 3.2.2):
// Y~^(n) = Y_p^(n) + sum_{i != n} Y_p^(i,n) x_i dA^(i)T; terms whose dA is still the zero
// of the build are skipped.
ppals_status pp_rhs_impl(const TCtx& c, int n, double* Y) {
  tucker_plan* p = c.p;
  const int N = p->N;
  {
    int is[TMAX];
    const double* F[TMAX];
    int nt = 0;
    for (int i = 0; i < N; ++i) {
      if (i == n || p->dA_zero[i]) continue;
      is[nt] = i;
      F[nt] = c.d(p->o_dA[i]);
      ++nt;
    }
    bool done = false;
    TCHK(pp_rhs_in_place(c, n, is, F, nt, c.d(p->o_Yp[n]), Y, &done));
    if (done) return PPALS_OK;
  }
  TuckerCombine a = combine_args(p, n, Y, c.d(p->o_Yp[n]));
  for (int i = 0; i < N; ++i) {
    if (i == n || p->dA_zero[i]) continue;
    double* T = c.d(p->o_term[a.nterms]);
    const Contr k = op_contr(p, i, n);
    const Level1Geom g = l1_geom(k.P, k.K, k.Q, p->R, DT_F64);
    const double* op = c.d(p->o_op[std::min(i, n)][std::max(i, n)]);
    if (same_operand_order(g, dA_geom(p, i))) {
      if (c.col) {
        c.col->part = std::max(c.col->part, part_elems(g));
      } else {
        THIPCHK(launch_level1(op, DT_F64, c.ws + p->o_dAprep[i], g, T, c.ws + p->o_part, c.s));
      }
    } else {
      TCHK(ttm_geom(c, op, g, c.d(p->o_dA[i]), T));
    }
    a.term[a.nterms] = T;
    a.pos[a.nterms] = rank_pos(i, n);
    ++a.nterms;
  }
  if (c.col) return PPALS_OK;
  THIPCHK(launch_tucker_combine(a, c.s));
  return PPALS_OK;
}

// Operator tree below a node T (layout L, d modes contracted): the operators in ops contract
// the modes other than i and n in increasing order, and their first d are the node's.
// Operators that contract the same next mode share that child node (in o_lvl[d + 1]);
// children are made depth first, so one buffer per depth suffices (the tree of the PP
// operators, Section 3.2.3).
ppals_status build_subtree(const TCtx& c, const double* T, const Lay& L, int d,
                           const std::vector<std::pair<int, int>>& ops, const double* const* Ap) {
  tucker_plan* p = c.p;
  const int N = p->N;
  auto next_mode = [&](const std::pair<int, int>& o) {
    int k = 0;
    for (int m = 0; m < N; ++m)
      if (m != o.first && m != o.second && k++ == d) return m;
    return -1;
  };
  std::vector<int> done(ops.size(), 0);
  for (size_t a = 0; a < ops.size(); ++a) {
    if (done[a]) continue;
    const int m = next_mode(ops[a]);
    std::vector<std::pair<int, int>> group;
    for (size_t b = a; b < ops.size(); ++b)
      if (!done[b] && next_mode(ops[b]) == m) {
        group.push_back(ops[b]);
        done[b] = 1;
      }
    const Contr k = contr_of(p, L, m);
    if (d + 1 == N - 2) {  // the operator itself (one per group: its modes are fixed)
      const std::pair<int, int> o = group.front();
      TCHK(ttm(c, T, k, Ap[m], c.d(p->o_op[o.first][o.second])));
      continue;
    }
    const Lay Lc = lay_after(L, m);
    if (c.col) c.col->lvl[d + 1] = std::max(c.col->lvl[d + 1], numel(p, Lc));
    double* child = c.d(p->o_lvl[d + 1]);
    TCHK(ttm(c, T, k, Ap[m], child));
    TCHK(build_subtree(c, child, Lc, d + 1, group, Ap));
  }
  return PPALS_OK;
}

// PP operator build (Algorithm 4): with A_p = A, Y_p^(i,n) for every pair i < n, the other
// modes contracted in increasing order; the first of them is 0, 1 or 2, so three passes
// over X (F_c = X x_c A_p^(c)T) serve every operator, and the later contractions follow
// the operator tree (build_subtree).  Y_p^(n) from an operator.
ppals_status build_impl(const TCtx& c, const double* X, double* const* A) {
  tucker_plan* p = c.p;
  const int N = p->N;
  const double* Ap[TMAX];
  for (int n = 0; n < N; ++n) {
    if (!c.col) {
      THIPCHK(launch_copy(c.d(p->o_Ap[n]), A[n], p->s[n] * p->R, c.s));
      THIPCHK(launch_fill(c.d(p->o_dA[n]), 0.0, p->s[n] * p->R, c.s));
    }
    Ap[n] = c.d(p->o_Ap[n]);
  }
  for (int c0 = 0; c0 < 3; ++c0) {
    const Lay L = lay_all(p);
    TCHK(ttm(c, X, contr_of(p, L, c0), Ap[c0], c.d(p->o_F[c0])));
    std::vector<std::pair<int, int>> ops;
    for (int i = 0; i < N; ++i)
      for (int n = i + 1; n < N; ++n) {
        int first = 0;
        while (first == i || first == n) ++first;
        if (first == c0) ops.push_back({i, n});
      }
    if (N == 3) {  // the operator is F_c itself
      for (const auto& o : ops)
        if (!c.col)
          THIPCHK(launch_copy(c.d(p->o_op[o.first][o.second]), c.d(p->o_F[c0]),
                              p->s[o.first] * p->s[o.second] * p->R, c.s));
      continue;
    }
    TCHK(build_subtree(c, c.d(p->o_F[c0]), lay_after(L, c0), 1, ops, Ap));
  }
  for (int n = 0; n < N; ++n) {
    const int i = n == 0 ? 1 : 0;  // Y_p^(n) = Y_p^(0,n) x_0 A_p^(0)T (n = 0: Y_p^(0,1) x_1)
    bool done = false;
    TCHK(pp_rhs_in_place(c, n, &i, &Ap[i], 1, nullptr, c.d(p->o_Yp[n]), &done));
    if (done) continue;
    TuckerCombine a = combine_args(p, n, c.d(p->o_Yp[n]), nullptr);
    double* T = c.d(p->o_term[0]);
    TCHK(ttm(c, c.d(p->o_op[std::min(i, n)][std::max(i, n)]), op_contr(p, i, n), Ap[i], T));
    a.term[0] = T;
    a.pos[0] = rank_pos(i, n);
    a.nterms = 1;
    if (!c.col) THIPCHK(launch_tucker_combine(a, c.s));
  }
  return PPALS_OK;
}

// HOSVD core: G = X x_0 A^(0)T .. x_(N-1) A^(N-1)T.
ppals_status hosvd_core(const TCtx& c, const double* X, const double* const* A, double* G) {
  std::vector<int> ms;
  for (int m = 0; m < c.p->N; ++m) ms.push_back(m);
  return chain(c, X, lay_all(c.p), ms, A, G);
}

// Interlaced HOSVD (Section 2.4): A^(n) from the prefix Z^(n) = P_n (X for n = 0, then
// P_(n+1) = P_n x_n A^(n)T), whose first mode is n; the core from P_(N-1).  info as in
// tucker_hosvd.
ppals_status hosvd_interlaced_impl(const TCtx& c, const double* X, double* const* V0,
                                   double* const* A, double* G, int32_t* info) {
  tucker_plan* p = c.p;
  const int N = p->N;
  for (int n = 0; n < N; ++n) {
    const double* Z = n == 0 ? X : c.d(p->o_pre[n & 1]);
    const Lay L = prefix_lay(p, n);
    TCHK(subspace(c, n, nullptr, Z, c.col ? nullptr : V0[n], nullptr, c.col ? nullptr : A[n],
                  p->hosvd_iters, info ? info + 3 * n : nullptr, nullptr, &L));
    if (n < N - 1) TCHK(extend_prefix(c, X, A, n));
  }
  return ttm(c, c.d(p->o_pre[(N - 1) & 1]), {1, p->s[N - 1], p->rpow[N - 1]},
             c.col ? nullptr : A[N - 1], G);
}

// ALS sweep schedule (also run in collecting mode for the workspace sizes).
ppals_status als_impl(const TCtx& c, const double* X, double* const* A, double* G,
                      tucker_sweep_record* rec) {
  tucker_plan* p = c.p;
  const int N = p->N;
  const int R = p->R;
  double* Aold = c.d(p->o_Aold);
  double* stats = c.d(p->o_stats);
  const double* Y = nullptr;
  for (int n = 0; n < N; ++n) {
    TCHK(als_ttmc(c, X, A, n, &Y));
    if (!c.col) THIPCHK(launch_copy(Aold, A[n], p->s[n] * R, c.s));
    int32_t info[3] = {0, 0, 0};
    TCHK(subspace(c, n, Y, nullptr, Aold, Aold, A[n], p->max_iters, info,
                  rec ? &rec->ritz_residual[n] : nullptr));
    if (rec) {
      rec->iters[n] = info[0];
      rec->converged[n] = info[1];
      rec->rr_status[n] = info[2];
    }
    if (!c.col) THIPCHK(launch_core_stats(A[n], Aold, p->s[n] * R, stats + 2 * n, c.s));
    if (n < N - 1) TCHK(extend_prefix(c, X, A, n));
  }
  return finish_core(c, Y, A[N - 1], G);
}

}  // namespace

extern "C" {

ppals_status tucker_plan_create(int32_t order, const int64_t* dims, int32_t rank,
                                tucker_plan** out) {
  if (!dims || !out) return set_error(PPALS_E_ARG, "NULL argument");
  *out = nullptr;
  if (order < 3 || order > TMAX) return set_error(PPALS_E_UNSUPPORTED, "order must be in [3, 8]");
  if (rank < 1 || rank > TUCKER_MAX_RANK)
    return set_error(PPALS_E_UNSUPPORTED, "Tucker rank must be in [1, 64]");
  double total = 1.0;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1) return set_error(PPALS_E_ARG, "dims must be >= 1");
    if (dims[n] < rank)
      return set_error(PPALS_E_UNSUPPORTED, "Tucker rank must not exceed any dimension");
    total *= (double)dims[n];
  }
  for (int n = 1; n < order - 1; ++n)
    if (total / (double)dims[n] > 2147483647.0 - 64.0)
      return set_error(PPALS_E_UNSUPPORTED,
                       "the product of the other dimensions of an inner mode must stay below "
                       "2^31 - 64 (strided HOSVD product)");
  if (std::pow((double)rank, order) > 1.0e12)
    return set_error(PPALS_E_UNSUPPORTED, "R^N too large");
  tucker_plan* p = new tucker_plan();
  p->N = order;
  p->R = rank;
  for (int n = 0; n < order; ++n) {
    p->s[n] = dims[n];
    p->dA_zero[n] = true;
  }
  p->rpow[0] = 1;
  for (int k = 1; k <= TMAX; ++k) p->rpow[k] = p->rpow[k - 1] * (k <= order ? rank : 1);
  const int N = order;
  const int64_t R = rank;
  int64_t smax = 0;
  for (int n = 0; n < N; ++n) smax = std::max(smax, dims[n]);
  // gather the schedules' sizes without launching
  Collector col;
  {
    TCtx c{p, nullptr, nullptr, &col};
    double* fake[TMAX];
    for (int n = 0; n < N; ++n) fake[n] = nullptr;
    const double* some = reinterpret_cast<const double*>(p);  // any non-null Y: sweep form
    for (int n = 0; n < N; ++n) {
      apply_w(c, n, nullptr, nullptr, nullptr, nullptr);  // HOSVD
      apply_w(c, n, some, nullptr, nullptr, nullptr);     // sweeps
    }
    hosvd_core(c, nullptr, fake, nullptr);
    hosvd_interlaced_impl(c, nullptr, fake, fake, nullptr, nullptr);
    for (int n = 0; n < N; ++n) {  // tucker_ttmc
      std::vector<int> ms;
      for (int m = 0; m < N; ++m)
        if (m != n) ms.push_back(m);
      chain(c, nullptr, lay_all(p), ms, fake, nullptr);
    }
    als_impl(c, nullptr, fake, nullptr, nullptr);
    build_impl(c, nullptr, fake);
    for (int n = 0; n < N; ++n) p->dA_zero[n] = false;  // every correction term
    for (int n = 0; n < N; ++n) pp_rhs_impl(c, n, nullptr);
    for (int n = 0; n < N; ++n) p->dA_zero[n] = true;
  }
  int64_t pre = 1;  // largest prefix P_n, n >= 1
  for (int n = 1; n < N; ++n) pre = std::max(pre, numel(p, prefix_lay(p, n)));
  size_t off = 0;
  auto take = [&](size_t elems) {
    const size_t o = off;
    off += al256(std::max<size_t>(elems, 1) * sizeof(double));
    return o;
  };
  for (int k = 0; k < 2; ++k) p->o_pre[k] = take(pre);
  for (int k = 0; k < 2; ++k) p->o_tmp[k] = take(col.tmp);
  for (int c0 = 0; c0 < 3; ++c0) p->o_F[c0] = take(numel(p, lay_after(lay_all(p), c0)));
  for (int d = 0; d < 8; ++d) p->o_lvl[d] = d >= 2 && d <= N - 3 ? take(col.lvl[d]) : 0;
  for (int i = 0; i < N; ++i)
    for (int n = i + 1; n < N; ++n) p->o_op[i][n] = take(dims[i] * dims[n] * p->rpow[N - 2]);
  for (int n = 0; n < N; ++n) p->o_Yp[n] = take(dims[n] * p->rpow[N - 1]);
  p->o_Y = take(smax * p->rpow[N - 1]);
  for (int t = 0; t < N - 1; ++t) p->o_term[t] = take(smax * p->rpow[N - 1]);
  p->o_Gn = take(p->rpow[N]);
  for (int n = 0; n < N; ++n) p->o_Ap[n] = take(dims[n] * R);
  for (int n = 0; n < N; ++n) p->o_dA[n] = take(dims[n] * R);
  for (int n = 0; n < N; ++n) p->o_Astart[n] = take(dims[n] * R);
  for (int n = 0; n < N; ++n) p->o_dAprep[n] = take(prep_elems(dA_geom(p, n)));
  // basis slots V, C, A_prev at equal spacing (one batched projection launch)
  p->slot = al256((size_t)smax * R * sizeof(double));
  p->o_V = take(smax * R);
  p->o_C = take(smax * R);
  p->o_Aold = take(smax * R);
  p->o_U = take(smax * R);
  p->o_Z = take(p->rpow[N - 1] * R);
  // B, H, P consecutive R x R blocks
  p->o_B = take(3 * R * R);
  p->o_H = p->o_B + (size_t)R * R * sizeof(double);
  p->o_P = p->o_H + (size_t)R * R * sizeof(double);
  p->o_T = take(R * R);
  p->o_lam = take(R);
  p->o_info = take(2 * TMAX);  // an iteration record per mode
  p->o_stats = take(2 * TMAX + 2);
  p->o_rpart = take(((smax + kRitzRows - 1) / kRitzRows) * R);
  p->o_prep = take(col.prep);
  p->o_part = take(col.part);
  p->o_gpart = take((size_t)kMaxGemmSplit * 3 * R * R);
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
  if (mode < 0 || mode >= plan->N) return set_error(PPALS_E_ARG, "mode out of range");
  TCtx c{plan, (char*)ws, stream};
  std::vector<int> ms;
  for (int m = 0; m < plan->N; ++m)
    if (m != mode) ms.push_back(m);
  return chain(c, X, lay_all(plan), ms, A, Y);
}

ppals_status tucker_factor_update(tucker_plan* plan, void* ws, const double* Y, int32_t mode,
                                  const double* A_prev, double* A_out, int32_t* info,
                                  double* residual, hipStream_t stream) {
  TCHK(check_common(plan, ws));
  if (!Y || !A_prev || !A_out) return set_error(PPALS_E_ARG, "NULL argument");
  if (mode < 0 || mode >= plan->N) return set_error(PPALS_E_ARG, "mode out of range");
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
  for (int n = 0; n < plan->N; ++n)
    TCHK(subspace(c, n, nullptr, X, V0[n], nullptr, A[n], plan->hosvd_iters,
                  info ? info + 3 * n : nullptr, nullptr));
  TCHK(hosvd_core(c, X, A, G));
  THIPCHK(hipStreamSynchronize(stream));
  plan->built = false;
  return PPALS_OK;
}

ppals_status tucker_hosvd_interlaced(tucker_plan* plan, void* ws, const double* X,
                                    double* const* V0, double* const* A, double* G,
                                    int32_t* info, hipStream_t stream) {
  TCHK(check_common(plan, ws));
  TCHK(check_factors(plan, A));
  TCHK(check_factors(plan, V0));
  if (!X || !G) return set_error(PPALS_E_ARG, "NULL argument");
  TCtx c{plan, (char*)ws, stream};
  TCHK(hosvd_interlaced_impl(c, X, V0, A, G, info));
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
  TCHK(als_impl(c, X, A, G, rec));
  double h[2 * TMAX + 2];
  THIPCHK(hipMemcpyAsync(h, c.d(plan->o_stats), sizeof(double) * (2 * plan->N + 2),
                         hipMemcpyDeviceToHost, stream));
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
  TCHK(build_impl(c, X, A));
  for (int n = 0; n < plan->N; ++n) plan->dA_zero[n] = true;
  plan->built = true;
  plan->built_ws = ws;
  plan->pp_optimistic = true;
  return PPALS_OK;
}

ppals_status tucker_pp_rhs(tucker_plan* plan, void* ws, int32_t mode, double* Y,
                           hipStream_t stream) {
  TCHK(check_common(plan, ws));
  if (!Y) return set_error(PPALS_E_ARG, "NULL argument");
  if (mode < 0 || mode >= plan->N) return set_error(PPALS_E_ARG, "mode out of range");
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
  const int N = plan->N;
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
    bool zero_start[TMAX];
    for (int n = 0; n < N; ++n) {
      zero_start[n] = plan->dA_zero[n];
      THIPCHK(launch_copy(c.d(plan->o_Astart[n]), A[n], plan->s[n] * R, stream));
    }
    for (int n = 0; n < N; ++n) {
      TCHK(pp_rhs_impl(c, n, Y));
      THIPCHK(launch_copy2(Aold, c.d(plan->o_V), A[n], plan->s[n] * R, stream));
      TCHK(subspace_step(c, n, Y, nullptr, true, dinfo + n));
      // A = U, dA = A - A_p, the norms; dA in operand order for the later modes' terms
      THIPCHK(launch_mode_end(c.d(plan->o_U), c.d(plan->o_Ap[n]), A[n], c.d(plan->o_dA[n]),
                              plan->s[n] * R, stats + 2 * n, stream));
      TCHK(prep_dA(c, n));
      plan->dA_zero[n] = false;
    }
    TCHK(finish_core(c, Y, A[N - 1], G, false));
    IterInfo hi[TMAX];
    THIPCHK(hipMemcpyAsync(hi, dinfo, sizeof(IterInfo) * N, hipMemcpyDeviceToHost, stream));
    THIPCHK(hipStreamSynchronize(stream));
    n0 = N;
    for (int n = N - 1; n >= 0; --n)
      if (!(hi[n].residual <= plan->tol)) n0 = n;
    for (int n = 0; n < n0; ++n) {
      rec->iters[n] = 1;
      rec->converged[n] = 1;
      rec->rr_status[n] = hi[n].rr_bad;
      rec->ritz_residual[n] = hi[n].residual;
    }
    if (n0 == N) {
      THIPCHK(launch_copy(G, c.d(plan->o_Gn), plan->rpow[N], stream));
    } else {
      plan->pp_optimistic = false;
      for (int n = n0; n < N; ++n) {
        THIPCHK(launch_copy(A[n], c.d(plan->o_Astart[n]), plan->s[n] * R, stream));
        THIPCHK(launch_sub(c.d(plan->o_dA[n]), A[n], c.d(plan->o_Ap[n]), plan->s[n] * R, stream));
        TCHK(prep_dA(c, n));
        plan->dA_zero[n] = zero_start[n];
      }
    }
  }
  if (n0 < N) {
    for (int n = n0; n < N; ++n) {
      TCHK(pp_rhs_impl(c, n, Y));
      THIPCHK(launch_copy(Aold, A[n], plan->s[n] * R, stream));
      int32_t info[3];
      TCHK(subspace(c, n, Y, nullptr, Aold, Aold, A[n], plan->max_iters, info,
                    &rec->ritz_residual[n]));
      rec->iters[n] = info[0];
      rec->converged[n] = info[1];
      rec->rr_status[n] = info[2];
      THIPCHK(launch_mode_end(A[n], c.d(plan->o_Ap[n]), nullptr, c.d(plan->o_dA[n]),
                              plan->s[n] * R, stats + 2 * n, stream));
      TCHK(prep_dA(c, n));
      plan->dA_zero[n] = false;
    }
    TCHK(finish_core(c, Y, A[N - 1], G));
    // back to the unsynchronised pass once a sweep needs a single iteration everywhere
    bool ones = true;
    for (int n = 0; n < N; ++n) ones = ones && rec->iters[n] == 1;
    plan->pp_optimistic = ones;
  }
  double h[2 * TMAX + 2];
  THIPCHK(hipMemcpyAsync(h, stats, sizeof(double) * (2 * N + 2), hipMemcpyDeviceToHost, stream));
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
  const int N = plan->N;
  int64_t count = 1;
  for (int n = 0; n < N; ++n) count *= plan->s[n];
  double* stats = reinterpret_cast<double*>((char*)ws + plan->o_stats);
  // ||X||^2 with the multi-workgroup reduction (partials in the level-1 partial region)
  THIPCHK(launch_norm2(X, DT_F64, count, reinterpret_cast<double*>((char*)ws + plan->o_part), 1024,
                       stats, stream));
  THIPCHK(launch_core_stats(G, G, plan->rpow[N], stats + 2, stream));
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
  double rel[TMAX];
  for (int i = 0; i < N; ++i) rel[i] = 1.0;  // dA = A initially
  double f_norm = std::sqrt(h[2]);
  auto stopped = [&]() { return delta > 0.0 && n > 0 && recs[n - 1].f_norm <= delta * normX; };
  auto small = [&]() {
    for (int i = 0; i < N; ++i)
      if (!(rel[i] < eps)) return false;
    return true;
  };
  while (n < sweeps && !stopped()) {
    if (small() && f_norm < eps * normX) {
      TCHK(tucker_pp_build(plan, ws, X, A, stream));
      int kind = PPALS_SWEEP_PP_INIT;
      while (n < sweeps && f_norm < eps * normX && !stopped()) {
        TCHK(tucker_pp_sweep(plan, ws, A, G, normX2, kind, &recs[n], stream));
        f_norm = recs[n].f_norm;
        for (int i = 0; i < N; ++i) rel[i] = recs[n].rel_change[i];
        *n_out = ++n;
        kind = PPALS_SWEEP_PP_APPROX;
      }
      if (n >= sweeps || stopped()) break;
    }
    TCHK(tucker_als_sweep(plan, ws, X, A, G, normX2, &recs[n], stream));
    f_norm = recs[n].f_norm;
    for (int i = 0; i < N; ++i) rel[i] = recs[n].rel_change[i];
    *n_out = ++n;
  }
  return PPALS_OK;
}

}  // extern "C"
