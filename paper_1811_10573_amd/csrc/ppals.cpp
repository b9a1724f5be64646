// Host side of the library: plans (dimension-tree schedules and workspace
// layout), the C ABI entry points and the native PP-CP-ALS driver.
//
// Schedules
//  * ALS sweep (Algorithm 1) with a binary dimension tree (Section 2.5).  For
//    N = 3 the tree contracts X with A^(3) (first-level GEMM) to get M^(1,2),
//    from which M^(1) and M^(2) follow by column-wise TTVs; then X with A^(1)
//    gives M^(2,3) and M^(3).  For N >= 4 the first two levels are combined
//    (Section 3.2.3, memory footprint): X is contracted with the Khatri-Rao
//    product of the trailing half of the modes, then of the leading half, and
//    each half is split recursively with TTVs.
//  * PP operator build (Section 3.2.3): level 2 holds the three tensors
//    X x_w A^(w), w in {1,2,3} (first-level GEMMs); level l >= 3 contracts one
//    mode of a level-(l-1) tensor; the leaves are the C(N,2) operators
//    M_p^(i,j).  M_p^(n) is one more TTV from a leaf.
//  * PP sweep (Algorithm 3 inner loop): per mode one batched TTV launch for the
//    N-1 first-order terms, one combine (M_p^(n) + partials + A^(n) W^(n)), the
//    FP64 solve and the Grams.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/ppals.h"
#include "common.h"

using namespace ppk;

static thread_local std::string g_err;
static ppals_status fail(ppals_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

// Waits for the stream by polling it: the driver's wait may put the thread to sleep, and
// the wake-up after each of the run loop's host decisions then costs up to hundreds of
// microseconds, depending on the host.
static hipError_t sync_spin(hipStream_t s) {
  for (;;) {
    const hipError_t e = hipStreamQuery(s);
    if (e != hipErrorNotReady) return e;
  }
}

// The k-th mode (k = 0 .. N-2) of mode n's PP-correction jobs, in the order their
// operators are read: the operator shared with the previous mode first, the one shared
// with the next mode last, so that consecutive modes read the operator they share back to
// back and the memory-side cache can serve the second read.
static inline int pp_job_mode(int N, int n, int k) { return ((n - 1 - k) % N + N) % N; }
namespace ppk {
// error reporting for the other host translation units (the batched engine)
ppals_status set_error(ppals_status st, const std::string& msg) { return fail(st, msg); }
}  // namespace ppk
#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(PPALS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

extern "C" const char* ppals_last_error(void) { return g_err.c_str(); }

namespace {

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct L1Step {
  int lo, hi;           // contracted modes [lo, hi); -1, -1 for a strided step
  std::vector<int> cmodes;  // strided step: the contracted modes, increasing
  Level1Geom geom;
  int out_buf;          // intermediate buffer id (bulk dtype), or -1: write FP64 M
  std::vector<int> kept;
};

struct TtvStep {
  int src_buf;                  // buffer id of the source intermediate
  std::vector<int> src_modes;   // modes of the source (sorted)
  int bpos, blen;               // contracted block inside src_modes
  int64_t P, X, Q;
  TtvJob job;                   // launch configuration (pointers filled at run time)
  int out_buf;                  // intermediate id, or -1 for the FP64 M buffer
  int out_mode;                 // if out_buf == -1: the mode whose M this is
  std::vector<int> kept;
};

enum OpKind { OP_L1 = 0, OP_TTV = 1, OP_SOLVE = 2 };
struct Op {
  OpKind kind;
  int idx;   // into l1 / ttv vectors, or the mode for SOLVE
};

struct BufDesc {
  size_t off = 0, bytes = 0;
};

}  // namespace

struct ppals_plan {
  int N = 0, R = 0;
  int64_t dims[PPALS_MAX_ORDER] = {0};
  int tdt = DT_F64, l1dt = DT_F64, bulk = DT_F64;
  int second_order = 1;
  int64_t max_s = 0, sum_s = 0;

  std::vector<L1Step> l1;
  std::vector<TtvStep> ttv;
  std::vector<BufDesc> bufs;       // intermediates (bulk dtype)
  std::vector<Op> dt_ops;          // ALS sweep
  std::vector<Op> pp_ops;          // operator build (L1 + TTV to leaves)
  std::vector<int> mp_ttv;         // per mode: TTV step producing M_p^(n) (out to mp buffer)
  int leaf_buf[PPALS_MAX_ORDER][PPALS_MAX_ORDER];
  // A first-level step of the operator build whose tensor the ALS sweep's tree also
  // contracts, with factors that are final by then: a build right after an ALS sweep copies
  // it from the tree's buffer (reuse_src) instead of contracting X again.  -1: none.
  int reuse_l1 = -1, reuse_src = -1;
  // per mode PP correction batch configuration
  TtvBatch ppb[PPALS_MAX_ORDER];
  int pp_slots[PPALS_MAX_ORDER];

  // workspace offsets
  size_t off_B = 0, sz_B = 0;          // level-1 operand
  size_t off_l1part = 0, sz_l1part = 0;
  size_t off_F = 0, sz_F = 0;          // FP64 Khatri-Rao block for multi-mode TTV
  size_t off_tpart = 0, sz_tpart = 0;  // FP64 TTV partial slots
  size_t off_M = 0;                    // FP64 max_s x R
  size_t off_Mp = 0, off_Ap = 0, off_dA = 0;  // FP64 sum_s x R each
  size_t off_U = 0;                    // N R^2
  size_t off_gamma = 0, off_L = 0, off_W = 0, off_pack = 0;
  size_t off_rowpart = 0;              // max_s x 4
  size_t off_scal = 0;                 // 64 doubles
  size_t off_status = 0;               // ints
  size_t off_norm = 0;                 // 4096 doubles
  size_t off_ppart = 0, sz_ppart = 0;  // PP partial slots
  size_t off_blockpart = 0;  // fused-solve per-block partial sums
  size_t off_Mx = 0, off_Mt = 0, off_errsum = 0;  // right-hand-side error measurement
  size_t off_gate = 0;                              // gate of PP sweeps enqueued ahead (int),
                                                    // then the ring position (int, +16 bytes)
                                                    // and the fused tail's counter (int, +32)
  size_t off_ring = 0;                              // records of sweeps enqueued ahead
  size_t off_gpart = 0, off_gctr = 0;  // Gram tiles' row-range partials and counters
  const int* cur_gate = nullptr;  // set while the gated PP sweep is being captured
  // while a PP sweep enqueued ahead is captured: its threshold test (eps); whether mode 0's
  // fused launch takes it (and finishes the sweep before), or a gate kernel does
  bool la_cur = false, la_gate_fused = false;
  double la_eps_cur = 0.0;
  bool fast = false;                   // rank <= 64: fused head/solve tail
  int combine = 1;                     // leading PP tree levels combined (1: the plain tree)
  bool combine_auto = false;           // chosen by the cost model
  std::string combine_model = "null";  // modelled build time per candidate (ms), JSON
  hipStream_t aux = nullptr;           // stream for the head kernel (default priority)
  ppals_sweep_record* pinned_rec = nullptr;  // pinned host staging of the sweep record
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  size_t ws_bytes = 0;
  std::vector<size_t> mode_off;        // element offsets of mode n in sum_s x R arrays

  // state
  bool ops_built = false;
  int sweeps_since_build = 0;
  // dA^(n) = 0 for every mode since the last build (set by the build, cleared by the first
  // sweep after it and by every other writer of dA)
  bool dA_zero = false;
  // update step size lambda of the step-size variant (1: Algorithm 1)
  double step = 1.0;

  // learned controller for leaving the PP phase (ppals_set_controller)
  bool ctl_set = false;
  ppals_controller ctl{};

  // PP-approximated sweep captured once in a HIP graph by ppals_run (rank <= 64 path)
  hipStream_t cap_stream = nullptr;  // capture stream (default priority)
  hipGraph_t pp_graph = nullptr;
  hipGraphExec_t pp_exec = nullptr;
  // ALS sweeps and PP-initialisation sweeps (operator build + first PP sweep), replayed
  struct SweepGraph {
    hipGraph_t g = nullptr;
    hipGraphExec_t e = nullptr;
    const void *ws = nullptr, *rec = nullptr, *S = nullptr, *X = nullptr, *Xb = nullptr;
    const double* A[PPALS_MAX_ORDER] = {nullptr};
    double normX2 = 0.0;
  } als_g, init_g, init_rg;  // init_rg: the build that copies the reused step
  // the same sweep behind the device-side threshold test, for sweeps enqueued ahead
  hipGraph_t la_graph = nullptr;
  hipGraphExec_t la_exec = nullptr;
  void* la_ws = nullptr;
  const void* la_recp = nullptr;
  const double* la_S = nullptr;
  const double* la_A[PPALS_MAX_ORDER] = {nullptr};
  double la_normX2 = 0.0, la_eps = 0.0;
  const void* g_ws = nullptr;
  const void* g_rec = nullptr;
  const double* g_S = nullptr;
  const double* g_A[PPALS_MAX_ORDER] = {nullptr};
  double g_normX2 = 0.0;
  // PP-approximated sweeps enqueued ahead of the host's decision by ppals_run
  static constexpr int kLookahead = 8;
  ppals_sweep_record* la_rec = nullptr;  // pinned host records, kLookahead slots
  hipEvent_t la_e0[kLookahead] = {nullptr}, la_e1[kLookahead] = {nullptr};

  // optional per-kernel-class timing with HIP events on the launch stream
  bool prof = false;
  struct Pending { int cls; hipEvent_t a, b; double flops, bytes; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
  ppals_kernel_stat stats[PPALS_PROF_CLASSES];

  std::string describe;
};

namespace {

int esize(int dt) { return dt == DT_F64 ? 8 : (dt == DT_F32 ? 4 : 2); }

int64_t prod_dims(const ppals_plan* p, const std::vector<int>& modes, int a, int b) {
  int64_t r = 1;
  for (int i = a; i < b; ++i) r *= p->dims[modes[i]];
  return r;
}

// Work decomposition of one multi-TTV job (T is P x X x Q x R with elements of es bytes).
// The vector kinds stream 16-byte vectors; the scalar kind covers every other shape.
// Workgroups of the slab kind wanted per multi-TTV launch (the row kind, whose workgroups
// stream more, takes 2/5 as many).  Measured on 800^3, R = 50: more, smaller workgroups
// of the slab kind shorten the tail of a launch; one round of large workgroups is slower.
constexpr int64_t kTtvRound = 3200;
constexpr int kGramSplitMax = 4;  // row ranges per Gram tile in PP sweeps
// Row ranges of a PP sweep's Gram tiles for a factor of `rows` rows: ranges of at least 192
// rows, at most kGramSplitMax.
int gram_ranges(int64_t rows) {
  return (int)std::max<int64_t>(1, std::min<int64_t>(kGramSplitMax, rows / 192));
}

// target: workgroups wanted for this job (slab kind; 2/5 of it for the row kind).
void ttv_config(TtvJob& J, int64_t P, int64_t X, int64_t Q, int R, int es, int64_t target) {
  memset(&J, 0, sizeof(J));
  J.P = P;
  J.X = X;
  J.Q = Q;
  const int64_t QR = Q * R;
  const int VEC = 16 / es;
  const int g = R / std::gcd(R, VEC);  // lanes per whole number of rank rows
  if (Q == 1 && (X * R) % VEC == 0 && g <= 64) {
    J.kind = TTV_SLAB;
    J.lanes = (64 / g) * g;
    const int64_t niter = X * R / ((int64_t)VEC * J.lanes);
    const int64_t cap = std::max<int64_t>(1, niter / 32);
    const int64_t groups = (P + TTV_SLAB_PB - 1) / TTV_SLAB_PB;
    J.xsplit = (int)std::max<int64_t>(1, std::min<int64_t>((target + groups - 1) / groups, cap));
    J.jblocks = 1;
    J.blocks = groups * J.xsplit;
    J.out_split_stride = P * QR;
    return;
  }
  // rows of 16-byte vectors, or for FP32 rows of even length 8-byte vectors
  const bool rows16 = QR % VEC == 0 && QR >= (int64_t)VEC * 64;
  const bool rows8 = !rows16 && es == 4 && QR % 2 == 0 && QR >= 2 * 64;
  if (rows16 || rows8) {
    const int RV = rows16 ? VEC : 2;
    J.kind = rows16 ? TTV_ROWS : TTV_ROWS2;
    J.jblocks = (int)((QR + (int64_t)RV * TTV_VTHREADS - 1) / ((int64_t)RV * TTV_VTHREADS));
    const int64_t base = P * J.jblocks;
    int64_t xsplit = (target * 2 / 5 + base - 1) / base;
    xsplit = std::max<int64_t>(1, std::min<int64_t>(xsplit, X / 8));
    int64_t xs = (X + xsplit - 1) / xsplit;
    xs = std::min<int64_t>(xs, 8192 / R);  // F rows staged in at most 64 KB of LDS
    xs = std::max<int64_t>(xs, 1);
    J.xs = (int)xs;
    J.xsplit = (int)((X + xs - 1) / xs);
    J.blocks = base * J.xsplit;
    J.out_split_stride = P * QR;
    return;
  }
  J.kind = TTV_SCALAR;
  if (QR >= TTV_THREADS) {
    J.Jb = TTV_THREADS;
    J.G = 1;
    J.jblocks = (int)((QR + TTV_THREADS - 1) / TTV_THREADS);
  } else {
    J.Jb = (int)QR;
    J.G = (int)(TTV_THREADS / QR);
    J.jblocks = 1;
  }
  const int64_t base = P * J.jblocks;
  const int64_t starget = 512;  // 768-thread workgroups of the scalar kernel
  int64_t xs = (starget + base - 1) / base;
  const int64_t maxs = std::max<int64_t>(1, X / (8 * (int64_t)J.G));
  xs = std::max<int64_t>(1, std::min(xs, maxs));
  J.xsplit = (int)xs;
  J.blocks = base * xs;
  J.out_split_stride = P * QR;
}

constexpr int64_t kL1Workgroups = 1536;

}  // namespace

// Geometry of a first-level contraction of a P x K x Q tensor (K contracted) with a
// K x R operand in the given dtype tier.
Level1Geom l1_geom(int64_t P, int64_t K, int64_t Q, int R, int l1dt) {
  Level1Geom g;
  memset(&g, 0, sizeof(g));
  g.M = P * Q;
  g.K = K;
  g.Q = Q;
  g.R = R;
  const int nbt = (R + 15) / 16;
  g.nslices = (nbt + 3) / 4;
  g.NB = (nbt + g.nslices - 1) / g.nslices;
  const int KC = l1dt == DT_BF16 ? 64 : 32;
  g.Kpad = (K + KC - 1) / KC * KC;
  g.kc_mode = (Q == 1) ? 1 : 0;
  int BM;
  if (l1dt == DT_F64) BM = 128;
  else if (l1dt == DT_F32) BM = 256;
  else BM = g.kc_mode ? 256 : 128;
  const int64_t mtiles = (g.M + BM - 1) / BM;
  const int64_t nchunks = g.Kpad / KC;
  // Split K when the row tiles alone give too few workgroups: aim at two rounds of the
  // 768 workgroups that run at once (256 compute units, three per unit at the occupancy of
  // the FP32 kernel).  Measured at 160^4, R = 64 (25600 row tiles of 256, K = 25600):
  // 600 workgroups 1.04 / 0.91 ms, 1500 workgroups 0.94 / 0.82 ms.
  int64_t ks = (kL1Workgroups + mtiles * g.nslices - 1) / (mtiles * g.nslices);
  ks = std::max<int64_t>(1, std::min(ks, nchunks / 4));
  const int64_t cps = (nchunks + ks - 1) / ks;
  g.kchunk = cps * KC;
  g.ksplit = (int)((g.K + g.kchunk - 1) / g.kchunk);
  return g;
}

namespace {

Level1Geom l1_config(const ppals_plan* p, int lo, int hi) {
  int64_t P = 1, K = 1, Q = 1;
  for (int i = 0; i < lo; ++i) P *= p->dims[i];
  for (int i = lo; i < hi; ++i) K *= p->dims[i];
  for (int i = hi; i < p->N; ++i) Q *= p->dims[i];
  return l1_geom(P, K, Q, p->R, p->l1dt);
}

int new_buf(ppals_plan* p, size_t bytes) {
  BufDesc b;
  b.bytes = bytes;
  p->bufs.push_back(b);
  return (int)p->bufs.size() - 1;
}

int add_l1(ppals_plan* p, int lo, int hi, int out_buf) {
  L1Step s;
  s.lo = lo;
  s.hi = hi;
  s.geom = l1_config(p, lo, hi);
  s.out_buf = out_buf;
  for (int i = 0; i < p->N; ++i)
    if (i < lo || i >= hi) s.kept.push_back(i);
  p->l1.push_back(s);
  return (int)p->l1.size() - 1;
}

int add_ttv(ppals_plan* p, int src_buf, const std::vector<int>& src_modes, int bpos, int blen,
            int out_buf, int out_mode) {
  TtvStep t;
  t.src_buf = src_buf;
  t.src_modes = src_modes;
  t.bpos = bpos;
  t.blen = blen;
  t.P = prod_dims(p, src_modes, 0, bpos);
  t.X = prod_dims(p, src_modes, bpos, bpos + blen);
  t.Q = prod_dims(p, src_modes, bpos + blen, (int)src_modes.size());
  ttv_config(t.job, t.P, t.X, t.Q, p->R, esize(p->bulk), kTtvRound / 2);
  t.out_buf = out_buf;
  t.out_mode = out_mode;
  for (int i = 0; i < (int)src_modes.size(); ++i)
    if (i < bpos || i >= bpos + blen) t.kept.push_back(src_modes[i]);
  p->ttv.push_back(t);
  return (int)p->ttv.size() - 1;
}

size_t node_bytes(const ppals_plan* p, const std::vector<int>& modes) {
  int64_t n = p->R;
  for (int m : modes) n *= p->dims[m];
  return (size_t)n * esize(p->bulk);
}

// Recursive part of the ALS dimension tree: `buf` holds M^(modes) (|modes| >= 2).
void dt_recurse(ppals_plan* p, int buf, const std::vector<int>& modes, std::vector<int>& depth_buf,
                int depth) {
  const int k = (int)modes.size();
  const int m = (k + 1) / 2;
  std::vector<int> left(modes.begin(), modes.begin() + m), right(modes.begin() + m, modes.end());
  for (int side = 0; side < 2; ++side) {
    const std::vector<int>& keep = side == 0 ? left : right;
    // left child contracts the trailing block, right child the leading block
    const int bpos = side == 0 ? m : 0;
    const int blen = side == 0 ? k - m : m;
    if (keep.size() == 1) {
      const int t = add_ttv(p, buf, modes, bpos, blen, -1, keep[0]);
      p->dt_ops.push_back({OP_TTV, t});
      p->dt_ops.push_back({OP_SOLVE, keep[0]});
    } else {
      if ((int)depth_buf.size() <= depth) depth_buf.push_back(new_buf(p, 0));
      const int ob = depth_buf[depth];
      p->bufs[ob].bytes = std::max(p->bufs[ob].bytes, node_bytes(p, keep));
      const int t = add_ttv(p, buf, modes, bpos, blen, ob, -1);
      p->dt_ops.push_back({OP_TTV, t});
      dt_recurse(p, ob, keep, depth_buf, depth + 1);
    }
  }
}

void build_dt(ppals_plan* p) {
  const int N = p->N;
  std::vector<int> depth_buf;
  depth_buf.push_back(new_buf(p, 0));
  const int b0 = depth_buf[0];
  auto root_child = [&](int lo, int hi) {
    std::vector<int> keep;
    for (int i = 0; i < N; ++i)
      if (i < lo || i >= hi) keep.push_back(i);
    p->bufs[b0].bytes = std::max(p->bufs[b0].bytes, node_bytes(p, keep));
    const int s = add_l1(p, lo, hi, b0);
    p->dt_ops.push_back({OP_L1, s});
    dt_recurse(p, b0, keep, depth_buf, 1);
  };
  if (N == 3) {
    root_child(2, 3);   // M^(1,2) = X x_3 A^(3)  -> M^(1), M^(2)
    root_child(0, 1);   // M^(2,3) = X x_1 A^(1)  -> (M^(2) unused) M^(3)
  } else {
    const int h = (N + 1) / 2;
    root_child(h, N);
    root_child(0, h);
  }
}

// For N == 3 the second root child {2,3} would produce M^(2) a second time; keep
// only the first SOLVE of each mode and, by backward liveness, the contractions
// that feed a kept op.
void prune_dt(ppals_plan* p) {
  const int nops = (int)p->dt_ops.size();
  std::vector<int> first_solve(p->N, -1);
  for (int i = 0; i < nops; ++i)
    if (p->dt_ops[i].kind == OP_SOLVE && first_solve[p->dt_ops[i].idx] < 0)
      first_solve[p->dt_ops[i].idx] = i;
  std::vector<bool> keep(nops, false);
  std::vector<int> readers(p->bufs.size(), 0);  // kept readers of a buffer's current value
  bool need_M = false;
  for (int i = nops - 1; i >= 0; --i) {
    const Op& o = p->dt_ops[i];
    if (o.kind == OP_SOLVE) {
      keep[i] = first_solve[o.idx] == i;
      if (keep[i]) need_M = true;
    } else if (o.kind == OP_TTV) {
      const TtvStep& t = p->ttv[o.idx];
      if (t.out_buf < 0) {
        keep[i] = need_M;
        need_M = false;
      } else {
        keep[i] = readers[t.out_buf] > 0;
        readers[t.out_buf] = 0;
      }
      if (keep[i]) readers[t.src_buf]++;
    } else {
      const L1Step& l = p->l1[o.idx];
      keep[i] = readers[l.out_buf] > 0;
      readers[l.out_buf] = 0;
    }
  }
  std::vector<Op> out;
  for (int i = 0; i < nops; ++i)
    if (keep[i]) out.push_back(p->dt_ops[i]);
  p->dt_ops.swap(out);
}

}  // namespace

// Multiplier and shift of the division by d used by the strided first-level loads:
// q = (n * mag) >> (32 + sh) with sh = ceil(log2 d) and mag = ceil(2^(32+sh) / d) is
// floor(n / d) for every n < 2^32 (Granlund and Montgomery, division by invariant
// integers); the kernel keeps n < 2^31 so that n * mag fits in 64 bits.
void l1_magic(uint32_t d, uint64_t* mag, int* sh) {
  int l = 0;
  while ((1ull << l) < d) ++l;
  const unsigned __int128 num = (unsigned __int128)1 << (32 + l);
  *mag = (uint64_t)((num + d - 1) / d);
  *sh = l;
}

namespace {

// Node of the PP tree at paper level lv (2 <= lv <= N - 1) for the pair (i, j), i < j <= lv
// (0-based): the tensor with modes i, j and the tail lv + 1 .. N - 1, straight from X by
// contracting the other lv - 1 modes (all <= lv) with their Khatri-Rao product.  At
// lv = N - 1 it is the operator M_p^(i,j); at lv = 2 it is a first-level node of the tree.
// A contiguous block of contracted modes is a plain first-level step; otherwise the
// contracted modes form up to three blocks (before i, between i and j, after j) and the
// step reads X through strided offsets: rows (x_i, x_j, tail), k over the three blocks.
int add_direct_node(ppals_plan* p, int lv, int i, int j, int out_buf) {
  const int N = p->N;
  std::vector<int> cm;
  for (int m = 0; m <= lv; ++m)
    if (m != i && m != j) cm.push_back(m);
  bool contiguous = true;
  for (size_t a = 1; a < cm.size(); ++a) contiguous = contiguous && cm[a] == cm[a - 1] + 1;
  if (contiguous) return add_l1(p, cm.front(), cm.back() + 1, out_buf);
  auto prod = [&](int lo, int hi) {  // dims[lo..hi)
    int64_t v = 1;
    for (int m = lo; m < hi; ++m) v *= p->dims[m];
    return v;
  };
  L1Step s;
  s.lo = s.hi = -1;
  s.cmodes = cm;
  s.kept = {i, j};
  for (int m = lv + 1; m < N; ++m) s.kept.push_back(m);
  s.out_buf = out_buf;
  const int64_t tail = prod(lv + 1, N);
  const int64_t n1 = prod(0, i), n2 = prod(i + 1, j), n3 = prod(j + 1, lv + 1);
  const int64_t K = n1 * n2 * n3, M = p->dims[i] * p->dims[j] * tail;
  Level1Geom g = l1_geom(M, K, 1, p->R, p->l1dt);
  g.kc_mode = 0;
  g.Q = 1;
  g.strided = 1;
  g.mrad = p->dims[j];
  g.mrad2 = tail;
  g.ms0 = prod(i + 1, N);
  g.ms1 = prod(j + 1, N);
  g.ms2 = 1;
  g.kr1 = (uint32_t)n2;
  g.kr2 = (uint32_t)n3;
  l1_magic(g.kr1, &g.kmag1, &g.ksh1);
  l1_magic(g.kr2, &g.kmag2, &g.ksh2);
  g.ks0 = prod(i, N);
  g.ks1 = prod(j, N);
  g.ks2 = tail;
  s.geom = g;
  p->l1.push_back(s);
  return (int)p->l1.size() - 1;
}

// Operator build with the first l levels combined (Section 3.2.3): the C(l + 2, 2) nodes
// of paper level l + 1 each contract l modes of X at once, the later levels contract one
// mode of a parent each.  Modelled time, per node, from the rates the first-level kernel
// and the multi-TTV reach here: a contraction of X at 0.6 of the tier's MFMA peak (0.45
// when the contracted modes are not one block and the loads are strided) or 0.6 of 8 TB/s
// for reading X and writing the node, whichever is slower; a tree contraction at 0.55 of
// 8 TB/s for reading its parent and writing the node.
double model_build_ms(const ppals_desc* d, int l) {
  const int N = d->order;
  double nX = 1.0;
  for (int m = 0; m < N; ++m) nX *= (double)d->dims[m];
  const double peak = d->level1_dtype == PPALS_FP64 ? 78.6e12 : (d->level1_dtype == PPALS_FP32 ? 157.3e12 : 2500e12);
  const double xsz = d->level1_dtype == PPALS_FP64 ? 8.0 : (d->level1_dtype == PPALS_FP32 ? 4.0 : 2.0);
  const double bulk = d->tensor_dtype == PPALS_FP64 ? 8.0 : 4.0;
  const double R = d->rank;
  double t = 0.0;
  for (int lv = l + 1; lv <= N - 1; ++lv) {
    double tail = 1.0;
    for (int m = lv + 1; m < N; ++m) tail *= (double)d->dims[m];
    for (int i = 0; i <= lv; ++i)
      for (int j = i + 1; j <= lv; ++j) {
        if (lv == l + 1) {
          // contracted modes {0..lv} minus {i, j}: one block unless i, j split them
          const bool block = (i == 0 && j == 1) || (j == lv && i == lv - 1) || (i == 0 && j == lv);
          const double f = 2.0 * nX * R / ((block || lv == 2 ? 0.6 : 0.45) * peak);
          // X read once, the node (modes i, j, the tail, the rank) written once
          const double node = (double)d->dims[i] * d->dims[j] * tail * R;
          const double b = (nX * xsz + node * bulk) / (0.6 * 8e12);
          t += std::max(f, b);
        } else {
          // parent: modes i, j, the mode w the tree rule contracts (build_pp: lv while
          // j < lv, else lv - 1, or lv - 2 when i = lv - 1), and the tail
          const int w = j < lv ? lv : (i == lv - 1 ? lv - 2 : lv - 1);
          const double child = (double)d->dims[i] * d->dims[j] * tail * R * bulk;
          const double parent = child * (double)d->dims[w];
          t += (parent + child) / (0.55 * 8e12);
        }
      }
  }
  return t * 1e3;
}

// Levels to combine: requested (clamped to N - 2) or, for -1, the candidate with the least
// modelled time.  Returns -1 if combining needs the FP64/FP32 first level, -2 if a strided
// node would exceed the 31-bit contracted extent; est receives the model per candidate.
int choose_combine(const ppals_desc* d, int req, std::vector<double>* est) {
  const int N = d->order;
  auto fits = [&](int l) {
    const int lv = l + 1;
    for (int i = 0; i <= lv; ++i)
      for (int j = i + 1; j <= lv; ++j) {
        double K = 1.0;
        for (int m = 0; m <= lv; ++m)
          if (m != i && m != j) K *= (double)d->dims[m];
        if (K > 2147483647.0 - 64.0) return false;
      }
    return true;
  };
  for (int l = 1; l <= N - 2; ++l) est->push_back(model_build_ms(d, l));
  if (req == -1) {
    if (d->level1_dtype == PPALS_BF16) return 1;
    int best = 1;
    for (int l = 2; l <= N - 2; ++l)
      if (fits(l) && (*est)[l - 1] < (*est)[best - 1]) best = l;
    return best;
  }
  const int l = std::min(req, N - 2);
  if (l >= 2 && d->level1_dtype == PPALS_BF16) return -1;
  if (l >= 2 && !fits(l)) return -2;
  return l;
}

void build_pp(ppals_plan* p) {
  const int N = p->N;
  // node store: mode list -> buffer id
  std::vector<std::pair<std::vector<int>, int>> nodes;
  auto find = [&](const std::vector<int>& m) {
    for (auto& e : nodes)
      if (e.first == m) return e.second;
    return -1;
  };
  for (int i = 0; i < N; ++i)
    for (int j = 0; j < N; ++j) p->leaf_buf[i][j] = -1;
  // Paper numbering (modes 1-based in the text; 0-based here).  The nodes of level
  // first = combine + 1 come straight from X (combine modes contracted at once; 1 is the
  // plain tree), the later levels from their parents by one contraction each.
  const int first = p->combine + 1;
  for (int l = first; l <= N - 1; ++l) {
    std::vector<int> tail;
    for (int m = l + 2; m <= N; ++m) tail.push_back(m - 1);
    for (int i = 1; i <= l + 1; ++i)
      for (int j = i + 1; j <= l + 1; ++j) {
        int w = (j <= l) ? l + 1 : std::max(i == l - 1 ? -1 : l - 1, i == l ? -1 : l);
        std::vector<int> child = {i - 1, j - 1};
        child.insert(child.end(), tail.begin(), tail.end());
        std::vector<int> parent = child;
        parent.push_back(w - 1);
        std::sort(parent.begin(), parent.end());
        const int ob = new_buf(p, node_bytes(p, child));
        if (l == first) {
          p->pp_ops.push_back({OP_L1, add_direct_node(p, l, i - 1, j - 1, ob)});
        } else {
          const int pb = find(parent);
          const int pos = (int)(std::find(parent.begin(), parent.end(), w - 1) - parent.begin());
          const int t = add_ttv(p, pb, parent, pos, 1, ob, -1);
          p->pp_ops.push_back({OP_TTV, t});
        }
        nodes.push_back({child, ob});
        if (l == N - 1) p->leaf_buf[i - 1][j - 1] = ob;
      }
  }
  // M_p^(n) from a leaf (M_p^(1) from M_p^(1,2) contracting mode 2; others from M_p^(1,n))
  p->mp_ttv.assign(N, -1);
  for (int n = 0; n < N; ++n) {
    if (n == 0) {
      p->mp_ttv[n] = add_ttv(p, p->leaf_buf[0][1], {0, 1}, 1, 1, -2, 0);
    } else {
      p->mp_ttv[n] = add_ttv(p, p->leaf_buf[0][n], {0, n}, 0, 1, -2, n);
    }
  }
  // per-mode correction batches
  for (int n = 0; n < N; ++n) {
    TtvBatch& b = p->ppb[n];
    memset(&b, 0, sizeof(b));
    b.R = p->R;
    int nj = 0, slots = 0;
    for (int k = 0; k < N - 1; ++k) {
      const int i = pp_job_mode(N, n, k);
      TtvJob& J = b.job[nj++];
      const int64_t tg = kTtvRound / (N - 1);
      if (i < n) ttv_config(J, 1, p->dims[i], p->dims[n], p->R, esize(p->bulk), tg);  // op (i,n): contract leading
      else ttv_config(J, p->dims[n], p->dims[i], 1, p->R, esize(p->bulk), tg);        // op (n,i): contract trailing
      J.out_split_stride = p->dims[n] * (int64_t)p->R;
      slots += J.xsplit;
    }
    b.njobs = nj;
    p->pp_slots[n] = slots;
  }
}

void layout(ppals_plan* p) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += align256(std::max<size_t>(bytes, 1));
    return o;
  };
  const int R = p->R;
  // level-1 operand and split partials
  size_t szB = 0, szP = 0;
  for (auto& s : p->l1) {
    const Level1Geom& g = s.geom;
    szB = std::max(szB, (size_t)g.nslices * g.Kpad * 16 * g.NB * esize(p->l1dt));
    if (g.ksplit > 1) szP = std::max(szP, (size_t)g.ksplit * g.M * R * esize(p->bulk));
  }
  // TTV partials and KRP blocks
  size_t szF = 0, szT = 0;
  for (auto& t : p->ttv) {
    if (t.blen > 1) szF = std::max(szF, (size_t)t.X * R * 8);
    szT = std::max(szT, (size_t)t.job.xsplit * t.P * t.Q * R * 8);
  }
  {
    // the M_p^(n) contractions of a build run in one launch, each with its own slots
    size_t szMp = 0;
    for (int n = 0; n < p->N; ++n) {
      const TtvStep& t = p->ttv[p->mp_ttv[n]];
      szMp += (size_t)t.job.xsplit * t.P * t.Q * R * 8;
    }
    szT = std::max(szT, szMp);
  }
  size_t szPP = 0;
  for (int n = 0; n < p->N; ++n) szPP = std::max(szPP, (size_t)p->pp_slots[n] * p->dims[n] * R * 8);
  p->off_B = take(szB); p->sz_B = szB;
  p->off_l1part = take(szP); p->sz_l1part = szP;
  p->off_F = take(szF); p->sz_F = szF;
  p->off_tpart = take(szT); p->sz_tpart = szT;
  p->off_ppart = take(szPP); p->sz_ppart = szPP;
  p->off_M = take((size_t)p->max_s * R * 8);
  p->off_Mp = take((size_t)p->sum_s * R * 8);
  p->off_Ap = take((size_t)p->sum_s * R * 8);
  p->off_dA = take((size_t)p->sum_s * R * 8);
  p->off_U = take((size_t)p->N * R * R * 8);
  p->off_gamma = take((size_t)R * R * 8);
  p->off_L = take((size_t)R * R * 8);
  p->off_pack = take((2 * (size_t)R * R + R) * 8);
  p->off_W = take((size_t)R * R * 8);
  p->off_rowpart = take((size_t)p->max_s * 4 * 8);
  p->off_scal = take(64 * 8);
  p->off_status = take(64 * 4);
  p->off_norm = take(4096 * 8);
  {
    const int64_t nb = solve_fused_blocks(p->max_s);
    p->off_blockpart = take((size_t)nb * 5 * 8);
  }
  p->off_Mx = take((size_t)p->sum_s * R * 8);
  p->off_Mt = take((size_t)p->max_s * R * 8);
  p->off_errsum = take((size_t)2 * PPALS_MAX_ORDER * 8);
  p->off_gate = take(64);
  p->off_ring = take(sizeof(ppals_sweep_record) * (ppals_plan::kLookahead + 1));
  {
    const int nbr = (R + 15) / 16;
    p->off_gpart = take((size_t)nbr * nbr * kGramSplitMax * 512 * sizeof(double));
    p->off_gctr = take((size_t)nbr * nbr * sizeof(int));
  }
  for (auto& b : p->bufs) b.off = take(b.bytes);
  p->ws_bytes = off;
}

// A first-level step of the ALS sweep whose contracted modes are all solved before it in
// the sweep, and whose buffer nothing later in the sweep writes, holds at the end of the
// sweep the same tensor as the build step with the same contracted modes (the factors it
// used are the ones a build right after the sweep takes as A_p).  For order 3 this is
// X x_1 A^(1) = M_p^(2,3) (modes 1-based).
void find_reuse(ppals_plan* p) {
  const int nops = (int)p->dt_ops.size();
  for (int k = nops - 1; k >= 0 && p->reuse_l1 < 0; --k) {
    const Op& o = p->dt_ops[k];
    if (o.kind != OP_L1) continue;
    const L1Step& d = p->l1[o.idx];
    bool ok = true;
    for (int m = d.lo; m < d.hi && ok; ++m) {
      bool solved = false;
      for (int q = 0; q < k; ++q)
        solved = solved || (p->dt_ops[q].kind == OP_SOLVE && p->dt_ops[q].idx == m);
      ok = solved;
    }
    for (int q = k + 1; q < nops && ok; ++q) {
      const Op& w = p->dt_ops[q];
      if (w.kind == OP_L1 && p->l1[w.idx].out_buf == d.out_buf) ok = false;
      if (w.kind == OP_TTV && p->ttv[w.idx].out_buf == d.out_buf) ok = false;
    }
    if (!ok) continue;
    for (const Op& q : p->pp_ops) {
      if (q.kind != OP_L1) continue;
      const L1Step& b = p->l1[q.idx];
      if (b.lo == d.lo && b.hi == d.hi && b.kept == d.kept) {
        p->reuse_l1 = q.idx;
        p->reuse_src = d.out_buf;
        break;
      }
    }
  }
}

std::string json_ops(const ppals_plan* p, const std::vector<Op>& ops, double* flops_l1,
                     double* flops_ttv) {
  std::string s = "[";
  char tmp[512];
  bool first = true;
  *flops_l1 = 0;
  *flops_ttv = 0;
  for (const Op& o : ops) {
    if (!first) s += ",";
    first = false;
    if (o.kind == OP_L1) {
      const L1Step& st = p->l1[o.idx];
      const double f = 2.0 * (double)st.geom.M * (double)st.geom.K * p->R;
      *flops_l1 += f;
      std::string kept, contr;
      for (size_t i = 0; i < st.kept.size(); ++i) kept += (i ? "," : "") + std::to_string(st.kept[i]);
      if (st.cmodes.empty()) {
        contr = std::to_string(st.lo) + "," + std::to_string(st.hi);
      } else {
        for (size_t i = 0; i < st.cmodes.size(); ++i) contr += (i ? "," : "") + std::to_string(st.cmodes[i]);
      }
      snprintf(tmp, sizeof(tmp),
               "{\"op\":\"level1\",\"contract\":[%s],\"kept\":[%s],\"M\":%lld,\"K\":%lld,"
               "\"Q\":%lld,\"ksplit\":%d,\"kc_mode\":%d,\"strided\":%d,\"flops\":%.0f}",
               contr.c_str(), kept.c_str(), (long long)st.geom.M, (long long)st.geom.K,
               (long long)st.geom.Q, st.geom.ksplit, st.geom.kc_mode, st.geom.strided, f);
    } else if (o.kind == OP_TTV) {
      const TtvStep& t = p->ttv[o.idx];
      const double f = 2.0 * (double)t.P * t.X * t.Q * p->R;
      *flops_ttv += f;
      std::string kept, src;
      for (size_t i = 0; i < t.kept.size(); ++i) kept += (i ? "," : "") + std::to_string(t.kept[i]);
      for (size_t i = 0; i < t.src_modes.size(); ++i) src += (i ? "," : "") + std::to_string(t.src_modes[i]);
      snprintf(tmp, sizeof(tmp),
               "{\"op\":\"ttv\",\"src\":[%s],\"contract_pos\":[%d,%d],\"kept\":[%s],\"P\":%lld,"
               "\"X\":%lld,\"Q\":%lld,\"xsplit\":%d,\"out_mode\":%d,\"flops\":%.0f}",
               src.c_str(), t.bpos, t.blen, kept.c_str(), (long long)t.P, (long long)t.X,
               (long long)t.Q, t.job.xsplit, t.out_mode, f);
    } else {
      snprintf(tmp, sizeof(tmp), "{\"op\":\"solve\",\"mode\":%d}", o.idx);
    }
    s += tmp;
  }
  s += "]";
  return s;
}

void make_describe(ppals_plan* p) {
  double a1, a2, b1, b2;
  std::string dt = json_ops(p, p->dt_ops, &a1, &a2);
  std::string pp = json_ops(p, p->pp_ops, &b1, &b2);
  double mpf = 0;
  for (int n = 0; n < p->N; ++n) {
    const TtvStep& t = p->ttv[p->mp_ttv[n]];
    mpf += 2.0 * (double)t.P * t.X * t.Q * p->R;
  }
  double approx = 0;
  for (int n = 0; n < p->N; ++n)
    for (int i = 0; i < p->N; ++i)
      if (i != n) approx += 2.0 * (double)p->dims[i] * p->dims[n] * p->R;
  char tmp[1024];
  snprintf(tmp, sizeof(tmp),
           "\"dt_level1_flops\":%.0f,\"dt_ttv_flops\":%.0f,\"pp_build_level1_flops\":%.0f,"
           "\"pp_build_tree_ttv_flops\":%.0f,\"pp_build_mp_flops\":%.0f,"
           "\"pp_approx_first_order_flops\":%.0f,\"workspace_bytes\":%zu,\"order\":%d,\"rank\":%d",
           a1, a2, b1, b2, mpf, approx, p->ws_bytes, p->N, p->R);
  std::string reuse = "null";
  if (p->reuse_l1 >= 0)
    reuse = "[" + std::to_string(p->l1[p->reuse_l1].lo) + "," + std::to_string(p->l1[p->reuse_l1].hi) + "]";
  // row ranges of the PP sweeps' Gram tiles per mode (rank <= 64 path only)
  std::string ranges = "[";
  for (int n = 0; n < p->N; ++n)
    ranges += (n ? "," : "") + std::to_string(p->fast ? gram_ranges(p->dims[n]) : 0);
  ranges += "]";
  size_t inter = 0;  // bulk bytes of the build's buffers that are not operators (tree nodes)
  for (size_t b = 0; b < p->bufs.size(); ++b) {
    bool leaf = false;
    for (int i = 0; i < p->N; ++i)
      for (int j = 0; j < p->N; ++j) leaf = leaf || p->leaf_buf[i][j] == (int)b;
    bool pp_node = false;
    for (const Op& o : p->pp_ops) {
      if (o.kind == OP_L1) pp_node = pp_node || p->l1[o.idx].out_buf == (int)b;
      if (o.kind == OP_TTV) pp_node = pp_node || p->ttv[o.idx].out_buf == (int)b;
    }
    if (pp_node && !leaf) inter += p->bufs[b].bytes;
  }
  p->describe = std::string("{") + tmp + ",\"dt_ops\":" + dt + ",\"pp_build_ops\":" + pp +
                ",\"pp_build\":\"" +
                (p->combine == 1 ? "tree" : (p->combine == p->N - 2 ? "direct" : "combined")) +
                "\",\"pp_build_levels\":" + std::to_string(p->combine) + ",\"pp_build_auto\":" +
                (p->combine_auto ? "true" : "false") + ",\"pp_build_model_ms\":" + p->combine_model +
                ",\"pp_build_intermediate_bytes\":" + std::to_string(inter) +
                ",\"pp_build_reused_after_als\":" + reuse + ",\"fused_tail\":" +
                (p->fast ? "true" : "false") + ",\"pp_gram_ranges\":" + ranges + "}";
}

// ---------------------------------------------------------------------------
// Run-time helpers
// ---------------------------------------------------------------------------
struct Ctx {
  ppals_plan* p;
  char* ws;
  hipStream_t s;
  template <typename T>
  T* at(size_t off) const { return reinterpret_cast<T*>(ws + off); }
  double* M() const { return at<double>(p->off_M); }
  double* Mp(int n) const { return at<double>(p->off_Mp) + p->mode_off[n]; }
  double* Ap(int n) const { return at<double>(p->off_Ap) + p->mode_off[n]; }
  double* dA(int n) const { return at<double>(p->off_dA) + p->mode_off[n]; }
  double* U() const { return at<double>(p->off_U); }
  void* buf(int b) const { return ws + p->bufs[b].off; }
};

const char* const kProfNames[PPALS_PROF_CLASSES] = {
    "level1_gemm", "pp_correct_ttv", "dt_ttv", "pp_combine", "mode_tail", "prep_operand",
    "pp_build_ttv", "split_reduce"};

hipEvent_t prof_event(ppals_plan* p) {
  if (!p->pool.empty()) {
    hipEvent_t e = p->pool.back();
    p->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one launch (or a short group of launches) of a kernel class.
struct Prof {
  ppals_plan* p;
  int cls;
  hipStream_t s;
  double flops, bytes;
  hipEvent_t a = nullptr;
  Prof(ppals_plan* p_, int cls_, hipStream_t s_, double f = 0, double b = 0)
      : p(p_), cls(cls_), s(s_), flops(f), bytes(b) {
    if (p->prof) {
      a = prof_event(p);
      if (a && hipEventRecord(a, s) != hipSuccess) a = nullptr;
    }
  }
  hipEvent_t end_event() {
    if (!p->prof || !a) return nullptr;
    hipEvent_t b = prof_event(p);
    if (!b) return nullptr;
    p->pending.push_back({cls, a, b, flops, bytes});
    a = nullptr;
    return b;
  }
  void end() {
    hipEvent_t b = end_event();
    if (b && hipEventRecord(b, s) != hipSuccess) p->pending.pop_back();
  }
};

// Fold finished event pairs into the statistics (the stream must have been synchronised).
void prof_resolve(ppals_plan* p) {
  for (auto& e : p->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      ppals_kernel_stat& st = p->stats[e.cls];
      st.launches += 1;
      st.total_ms += ms;
      st.flops += e.flops;
      st.bytes += e.bytes;
    }
    p->pool.push_back(e.a);
    p->pool.push_back(e.b);
  }
  p->pending.clear();
}

ppals_status run_l1(const Ctx& c, const L1Step& st, const void* X, const void* Xb,
                    double* const* A, void* out) {
  ppals_plan* p = c.p;
  KrpDesc krp;
  memset(&krp, 0, sizeof(krp));
  krp.R = p->R;
  if (!st.cmodes.empty()) {
    krp.nf = (int)st.cmodes.size();
    for (int f = 0; f < krp.nf; ++f) {
      krp.A[f] = A[st.cmodes[f]];
      krp.dim[f] = p->dims[st.cmodes[f]];
    }
  } else {
    krp.nf = st.hi - st.lo;
    for (int f = 0; f < krp.nf; ++f) {
      krp.A[f] = A[st.lo + f];
      krp.dim[f] = p->dims[st.lo + f];
    }
  }
  void* B = c.ws + p->off_B;
  {
    Prof pr(p, 5, c.s);
    HIPCHK(launch_prep_operand(krp, st.geom, p->l1dt, B, c.s));
    pr.end();
  }
  const void* xin = p->l1dt == DT_BF16 ? Xb : X;
  const Level1Geom& g = st.geom;
  const double flops = 2.0 * (double)g.M * (double)g.K * p->R;
  const double bytes = (double)g.M * g.K * esize(p->l1dt) + (double)g.K * p->R * esize(p->l1dt) +
                       (double)g.M * p->R * esize(p->bulk) * g.ksplit;
  Prof pr(p, 0, c.s, flops, bytes);
  HIPCHK(launch_level1(xin, p->l1dt, B, st.geom, out, c.ws + p->off_l1part, c.s, pr.end_event()));
  return PPALS_OK;
}

// Run a TTV step; out_fp64 (if non-null) receives the FP64 result (M buffers),
// otherwise the step's intermediate buffer gets the bulk-dtype result.
ppals_status run_ttv(const Ctx& c, const TtvStep& t, double* const* A, double* out_fp64,
                     int cls = 2, bool keep_partials = false) {
  ppals_plan* p = c.p;
  const double* F;
  if (t.blen == 1) {
    F = A[t.src_modes[t.bpos]];
  } else {
    KrpDesc krp;
    memset(&krp, 0, sizeof(krp));
    krp.nf = t.blen;
    krp.R = p->R;
    for (int f = 0; f < t.blen; ++f) {
      krp.A[f] = A[t.src_modes[t.bpos + f]];
      krp.dim[f] = p->dims[t.src_modes[t.bpos + f]];
    }
    double* Fb = c.at<double>(p->off_F);
    HIPCHK(launch_krp_f64(krp, t.X, Fb, c.s));
    F = Fb;
  }
  TtvBatch b;
  memset(&b, 0, sizeof(b));
  b.R = p->R;
  b.njobs = 1;
  b.job[0] = t.job;
  b.job[0].T = c.buf(t.src_buf);
  b.job[0].t_is_f32 = p->bulk == DT_F32;
  b.job[0].F = F;
  double* part = c.at<double>(p->off_tpart);
  b.job[0].out = part;
  const int64_t count = t.P * t.Q * p->R;
  {
    const double tb = (double)t.P * t.X * t.Q * p->R * esize(p->bulk);
    Prof pr(p, cls, c.s, 2.0 * (double)t.P * t.X * t.Q * p->R,
            tb + (double)count * 8 * t.job.xsplit + (double)t.X * p->R * 8);
    HIPCHK(launch_ttv(b, c.s));
    pr.end();
  }
  if (keep_partials) return PPALS_OK;
  if (out_fp64) {
    HIPCHK(launch_combine(out_fp64, count, p->R, nullptr, part, t.job.xsplit, count, nullptr,
                          nullptr, c.s));
  } else {
    HIPCHK(launch_reduce_splits_to(c.buf(t.out_buf), p->bulk == DT_F32, part, 0, t.job.xsplit,
                                   count, c.s));
  }
  return PPALS_OK;
}

ppals_status mode_begin(const Ctx& c, double* S, double normX2, ppals_sweep_record* rec, int n,
                        int prev, int pp, int write_fit, int kind) {
  ppals_plan* p = c.p;
  ModeArgs a;
  memset(&a, 0, sizeof(a));
  a.N = p->N;
  a.R = p->R;
  a.n = n;
  a.prev = prev;
  a.pp = pp;
  a.second_order = p->second_order;
  a.write_fit = write_fit;
  a.sweep_kind = kind;
  a.prev_rows = prev >= 0 ? p->dims[prev] : 0;
  a.normX2 = normX2;
  a.S = S;
  a.U = c.U();
  a.gamma = c.at<double>(p->off_gamma);
  a.L = c.at<double>(p->off_L);
  a.gamma_save = a.gamma;
  a.W = c.at<double>(p->off_W);
  a.rowpart = c.at<double>(p->off_rowpart);
  a.scal = c.at<double>(p->off_scal);
  a.rec = rec;
  a.status = c.at<int>(p->off_status);
  HIPCHK(launch_mode_begin(a, c.s));
  return PPALS_OK;
}

ppals_status solve_mode(const Ctx& c, double* const* A, double* S, int n, bool pp) {
  ppals_plan* p = c.p;
  SolveArgs a;
  memset(&a, 0, sizeof(a));
  a.R = p->R;
  a.rows = p->dims[n];
  a.M = c.M();
  a.L = c.at<double>(p->off_L);
  a.gamma = c.at<double>(p->off_gamma);
  a.A = A[n];
  a.Aref = pp ? c.Ap(n) : nullptr;
  a.dA = pp ? c.dA(n) : nullptr;
  a.rowpart = c.at<double>(p->off_rowpart);
  a.status = c.at<int>(p->off_status) + n;
  a.step = p->step;
  HIPCHK(launch_solve_rows(a, c.s));
  HIPCHK(launch_gram(A[n], pp ? c.dA(n) : nullptr, p->dims[n], p->R, S + (size_t)n * p->R * p->R,
                     pp ? c.U() + (size_t)n * p->R * p->R : nullptr, c.s));
  return PPALS_OK;
}

ppals_status check_common(const ppals_plan* p, const void* X, const void* Xb, double* const* A,
                          const void* ws) {
  if (!p) return fail(PPALS_E_ARG, "plan is NULL");
  if (!X) return fail(PPALS_E_ARG, "X is NULL");
  if (p->l1dt == DT_BF16 && !Xb) return fail(PPALS_E_ARG, "X_bf16 is NULL in the BF16 tier");
  if (!A) return fail(PPALS_E_ARG, "A is NULL");
  for (int n = 0; n < p->N; ++n)
    if (!A[n]) return fail(PPALS_E_ARG, "A[" + std::to_string(n) + "] is NULL");
  if (!ws) return fail(PPALS_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(PPALS_E_WORKSPACE, "workspace is not 256-byte aligned");
  return PPALS_OK;
}

HeadArgs head_args(const Ctx& c, double* S, int n, int pp) {
  ppals_plan* p = c.p;
  HeadArgs h;
  memset(&h, 0, sizeof(h));
  h.N = p->N;
  h.R = p->R;
  h.n = n;
  h.pp = pp;
  h.second_order = p->second_order;
  h.S = S;
  h.U = c.U();
  h.gamma = c.at<double>(p->off_gamma);
  h.L = c.at<double>(p->off_L);
  h.W = c.at<double>(p->off_W);
  h.pack = c.at<double>(p->off_pack);
  h.status = c.at<int>(p->off_status);
  h.gate = p->cur_gate;
  return h;
}

// Grams of the freshly solved factor n into S^(n) (and U^(n) in PP sweeps) plus the
// sweep record of mode n (and the fit after the last mode).
// PP sweeps' Grams (rank <= 64): the rows of each tile in up to kGramSplitMax ranges of at
// least 192 rows, so that the fused launch's Gram role, which runs beside the
// contraction's memory traffic, takes fewer dependent load rounds per workgroup.
void gram_split(const Ctx& c, GramArgs& g) {
  g.nsplit = gram_ranges(g.rows);
  g.gpart = c.at<double>(c.p->off_gpart);
  g.gctr = c.at<int>(c.p->off_gctr);
}

GramArgs gram_args(const Ctx& c, double* const* A, double* S, int n, int pp, double normX2,
                   ppals_sweep_record* rec, int write_fit, int kind) {
  ppals_plan* p = c.p;
  GramArgs g;
  memset(&g, 0, sizeof(g));
  g.R = p->R;
  g.mode = n;
  g.rows = p->dims[n];
  g.nblk = solve_fused_blocks(p->dims[n]);
  g.A = A[n];
  g.dA = pp ? c.dA(n) : nullptr;
  g.S_out = S + (size_t)n * p->R * p->R;
  g.U_out = c.U() + (size_t)n * p->R * p->R;
  g.blockpart = c.at<double>(p->off_blockpart);
  g.status = c.at<int>(p->off_status) + n;
  g.rec = rec;
  g.write_fit = write_fit;
  g.sweep_kind = kind;
  g.normX2 = normX2;
  g.gate = p->cur_gate;
  return g;
}

// Fast path: the Grams of the previous mode and the head of the next mode run on the
// auxiliary stream, forked from the main stream after the previous solve and joined
// before the next solve, so they overlap the next mode's contractions.
ppals_status tail_fork(const Ctx& c, const GramArgs* g, const HeadArgs* h) {
  ppals_plan* p = c.p;
  if (!p->aux) {
    HIPCHK(hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking));
    HIPCHK(hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming));
    HIPCHK(hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming));
  }
  HIPCHK(hipEventRecord(p->ev_fork, c.s));
  HIPCHK(hipStreamWaitEvent(p->aux, p->ev_fork, 0));
  if (g && h) {
    // the Gram kernel also forms Gamma^(n) and W^(n) of the next mode tile by tile, so the
    // head starts from them
    GramArgs g2 = *g;
    HeadArgs h2 = *h;
    g2.N = h->N;
    g2.next = h->n;
    g2.wterm = h->pp && h->second_order;
    g2.S_all = h->S;
    g2.U_all = h->U;
    g2.gamma_out = h->gamma;
    g2.W_out = h->W;
    h2.gamma_ready = 1;
    HIPCHK(launch_gram_tiles(g2, p->aux));
    HIPCHK(launch_head(h2, p->aux));
  } else {
    if (g) HIPCHK(launch_gram_tiles(*g, p->aux));
    if (h) HIPCHK(launch_head(*h, p->aux));
  }
  HIPCHK(hipEventRecord(p->ev_join, p->aux));
  return PPALS_OK;
}
ppals_status tail_join(const Ctx& c) {
  HIPCHK(hipStreamWaitEvent(c.s, c.p->ev_join, 0));
  return PPALS_OK;
}

ppals_status solve_fused(const Ctx& c, double* const* A, int n, const double* base,
                         const double* part, int nslots, bool pp, int write_fit) {
  ppals_plan* p = c.p;
  FusedSolveArgs a;
  memset(&a, 0, sizeof(a));
  a.R = p->R;
  a.rows = p->dims[n];
  a.base = base;
  a.part = part;
  a.nslots = nslots;
  a.slot_stride = p->dims[n] * (int64_t)p->R;
  a.W = (pp && p->second_order) ? c.at<double>(p->off_W) : nullptr;
  a.pack = c.at<double>(p->off_pack);
  a.gamma = c.at<double>(p->off_gamma);
  a.A = A[n];
  a.Aref = pp ? c.Ap(n) : nullptr;
  a.dA = pp ? c.dA(n) : nullptr;
  a.blockpart = c.at<double>(p->off_blockpart);
  a.status = c.at<int>(p->off_status) + n;
  a.write_fit = write_fit;
  a.gate = p->cur_gate;
  a.step = p->step;
  Prof pr(p, 4, c.s);
  HIPCHK(launch_solve_fused(a, c.s));
  pr.end();
  return PPALS_OK;
}

// End of a sweep: Grams and record of the last mode plus the fit (main stream).
ppals_status finish_sweep_fast(const Ctx& c, double* const* A, double* S, double normX2,
                               ppals_sweep_record* rec, int prev, int pp, int kind) {
  GramArgs g = gram_args(c, A, S, prev, pp, normX2, rec, 1, kind);
  if (pp) gram_split(c, g);
  Prof pr(c.p, 4, c.s);
  // PP sweeps: the summation order of the fused launches' Gram role, which computes the
  // same Grams for sweeps enqueued ahead
  HIPCHK(launch_gram_tiles(g, c.s, pp != 0));
  pr.end();
  return PPALS_OK;
}

ppals_status do_als_sweep(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                          double* S, double normX2, void* ws, ppals_sweep_record* rec,
                          hipStream_t s) {
  if (p->fast) {
    Ctx c{p, (char*)ws, s};
    int prev = -1, nslots = 0;
    bool forked = false;
    for (const Op& o : p->dt_ops) {
      ppals_status st = PPALS_OK;
      if (o.kind != OP_SOLVE && !forked) {
        const HeadArgs h = head_args(c, S, prev + 1, 0);
        if (prev >= 0) {
          const GramArgs g = gram_args(c, A, S, prev, 0, normX2, rec, 0, PPALS_SWEEP_ALS);
          st = tail_fork(c, &g, &h);
        } else {
          st = tail_fork(c, nullptr, &h);
        }
        forked = true;
      }
      if (st != PPALS_OK) return st;
      if (o.kind == OP_L1) {
        const L1Step& l = p->l1[o.idx];
        st = run_l1(c, l, X, Xb, A, c.buf(l.out_buf));
      } else if (o.kind == OP_TTV) {
        const TtvStep& t = p->ttv[o.idx];
        if (t.out_buf < 0) {
          st = run_ttv(c, t, A, nullptr, 2, /*keep_partials=*/true);
          nslots = t.job.xsplit;
        } else {
          st = run_ttv(c, t, A, nullptr);
        }
      } else {
        st = tail_join(c);
        if (st == PPALS_OK)
          st = solve_fused(c, A, o.idx, nullptr, c.at<double>(p->off_tpart), nslots, false,
                           o.idx == p->N - 1);
        prev = o.idx;
        forked = false;
      }
      if (st != PPALS_OK) return st;
    }
    return finish_sweep_fast(c, A, S, normX2, rec, prev, 0, PPALS_SWEEP_ALS);
  }
  Ctx c{p, (char*)ws, s};
  int prev = -1;
  for (const Op& o : p->dt_ops) {
    ppals_status st = PPALS_OK;
    if (o.kind == OP_L1) {
      const L1Step& l = p->l1[o.idx];
      st = run_l1(c, l, X, Xb, A, c.buf(l.out_buf));
    } else if (o.kind == OP_TTV) {
      const TtvStep& t = p->ttv[o.idx];
      st = run_ttv(c, t, A, t.out_buf < 0 ? c.M() : nullptr);
    } else {
      const int n = o.idx;
      Prof pr(p, 4, s);
      st = mode_begin(c, S, normX2, rec, n, prev, 0, 0, PPALS_SWEEP_ALS);
      if (st == PPALS_OK) st = solve_mode(c, A, S, n, false);
      pr.end();
      prev = n;
    }
    if (st != PPALS_OK) return st;
  }
  return mode_begin(c, S, normX2, rec, -1, prev, 0, 1, PPALS_SWEEP_ALS);
}

// reuse: the ALS sweep just before left the tensor of build step reuse_l1 in its buffer
// (same factors), so that step is a copy.
ppals_status do_pp_build(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                         void* ws, hipStream_t s, bool reuse = false) {
  Ctx c{p, (char*)ws, s};
  for (const Op& o : p->pp_ops) {
    ppals_status st = PPALS_OK;
    if (o.kind == OP_L1) {
      const L1Step& l = p->l1[o.idx];
      if (reuse && o.idx == p->reuse_l1)
        HIPCHK(launch_copy_bytes(c.buf(l.out_buf), c.buf(p->reuse_src), node_bytes(p, l.kept), s));
      else
        st = run_l1(c, l, X, Xb, A, c.buf(l.out_buf));
    } else {
      st = run_ttv(c, p->ttv[o.idx], A, nullptr, 6);
    }
    if (st != PPALS_OK) return st;
  }
  {
    // M_p^(n) for every mode: each contracts a leaf with one build-time factor, so the N
    // contractions are independent and share one launch (each job with its own partial
    // slots), followed by one slot reduction per mode.  Same jobs, same bits as N
    // launches.
    TtvBatch b;
    memset(&b, 0, sizeof(b));
    b.R = p->R;
    b.njobs = p->N;
    double* part = c.at<double>(p->off_tpart);
    int64_t off[PPALS_MAX_ORDER + 1];
    off[0] = 0;
    double fl = 0, by = 0;
    for (int n = 0; n < p->N; ++n) {
      const TtvStep& t = p->ttv[p->mp_ttv[n]];
      TtvJob& J = b.job[n];
      J = t.job;
      J.T = c.buf(t.src_buf);
      J.t_is_f32 = p->bulk == DT_F32;
      J.F = A[t.src_modes[t.bpos]];
      J.out = part + off[n];
      const int64_t count = t.P * t.Q * p->R;
      off[n + 1] = off[n] + count * t.job.xsplit;
      fl += 2.0 * (double)t.P * t.X * t.Q * p->R;
      by += (double)t.P * t.X * t.Q * p->R * esize(p->bulk) + (double)count * 8 * t.job.xsplit +
            (double)t.X * p->R * 8;
    }
    {
      Prof pr(p, 6, s, fl, by);
      HIPCHK(launch_ttv(b, s));
      pr.end();
    }
    for (int n = 0; n < p->N; ++n) {
      const TtvStep& t = p->ttv[p->mp_ttv[n]];
      const int64_t count = t.P * t.Q * p->R;
      HIPCHK(launch_combine(c.Mp(n), count, p->R, nullptr, part + off[n], t.job.xsplit, count,
                            nullptr, nullptr, s));
    }
  }
  {
    // A_p := A, dA := 0, U := 0 and the counters of the fused PP-correction launches (which
    // each leave them at zero again), in one launch
    BuildReset r{};
    r.N = p->N;
    int64_t o = 0;
    for (int n = 0; n < p->N; ++n) {
      r.A[n] = A[n];
      r.off[n] = o;
      o += (int64_t)p->dims[n] * p->R;
    }
    r.off[p->N] = o;
    r.Ap = c.Ap(0);
    r.dA = c.dA(0);
    r.ndA = o;
    r.U = c.U();
    r.nU = (int64_t)p->N * p->R * p->R;
    const int nbr = (p->R + 15) / 16;
    r.ints[0] = c.at<int>(p->off_gate) + 8;
    r.nints[0] = 1;
    r.ints[1] = c.at<int>(p->off_gctr);
    r.nints[1] = nbr * nbr;
    HIPCHK(launch_build_reset(r, s));
  }
  p->ops_built = true;
  p->sweeps_since_build = 0;
  p->dA_zero = true;
  return PPALS_OK;
}

ppals_status pp_correct(const Ctx& c, double* const* A, int n, double* out) {
  ppals_plan* p = c.p;
  TtvBatch b = p->ppb[n];
  double* part = c.at<double>(p->off_ppart);
  int64_t slot_off = 0;
  int nj = 0;
  for (int k = 0; k < p->N - 1; ++k) {
    const int i = pp_job_mode(p->N, n, k);
    TtvJob& J = b.job[nj++];
    const int lo = std::min(i, n), hi = std::max(i, n);
    J.T = c.buf(p->leaf_buf[lo][hi]);
    J.t_is_f32 = p->bulk == DT_F32;
    J.F = c.dA(i);
    J.out = part + slot_off;
    slot_off += (int64_t)J.xsplit * J.out_split_stride;
  }
  const int64_t count = p->dims[n] * (int64_t)p->R;
  {
    double fl = 0, by = 0;
    for (int i = 0; i < p->N; ++i) {
      if (i == n) continue;
      const double e = (double)p->dims[i] * p->dims[n] * p->R;
      fl += 2.0 * e;
      by += e * esize(p->bulk) + (double)p->dims[i] * p->R * 8;
    }
    by += (double)p->pp_slots[n] * count * 8;
    Prof pr(p, 1, c.s, fl, by);
    HIPCHK(launch_ttv(b, c.s));
    pr.end();
  }
  {
    Prof pr(p, 3, c.s, 0, (double)(p->pp_slots[n] + 3) * count * 8);
    HIPCHK(launch_combine(out, count, p->R, c.Mp(n), part, p->pp_slots[n], count,
                          p->second_order ? A[n] : nullptr,
                          p->second_order ? c.at<double>(p->off_W) : nullptr, c.s));
    pr.end();
  }
  return PPALS_OK;
}

ppals_status do_pp_sweep(ppals_plan* p, double* const* A, double* S, double normX2, void* ws,
                         ppals_sweep_record* rec, hipStream_t s) {
  Ctx c{p, (char*)ws, s};
  const int kind = p->sweeps_since_build == 0 ? PPALS_SWEEP_PP_INIT : PPALS_SWEEP_PP_APPROX;
  const bool dA_zero = p->dA_zero;
  p->dA_zero = false;
  int prev = -1;
  if (p->fast) {
    double* part = c.at<double>(p->off_ppart);
    int* tail_ctr = c.at<int>(p->off_gate) + 8;  // zero after every build and fused launch
    for (int n = 0; n < p->N; ++n) {
      TtvBatch b = p->ppb[n];
      b.gate = p->cur_gate;
      int64_t slot_off = 0;
      int nj = 0, nslots = 0;
      double fl = 0, by = 0;
      for (int k = 0; k < p->N - 1; ++k) {
        const int i = pp_job_mode(p->N, n, k);
        // Right after a build dA^(i) is exactly zero until mode i's solve in this sweep, so
        // the contraction with it adds exact zeros: the first sweep skips it (same bits).
        if (dA_zero && i > n) continue;
        b.job[nj] = p->ppb[n].job[k];
        TtvJob& J = b.job[nj++];
        const int lo = std::min(i, n), hi = std::max(i, n);
        J.T = c.buf(p->leaf_buf[lo][hi]);
        J.t_is_f32 = p->bulk == DT_F32;
        J.F = c.dA(i);
        J.out = part + slot_off;
        slot_off += (int64_t)J.xsplit * J.out_split_stride;
        nslots += J.xsplit;
        const double e = (double)p->dims[i] * p->dims[n] * p->R;
        fl += 2.0 * e;
        by += e * esize(p->bulk) + (double)p->dims[i] * p->R * 8;
      }
      b.njobs = nj;
      by += (double)nslots * p->dims[n] * p->R * 8;
      const HeadArgs h = head_args(c, S, n, 1);
      ppals_status st;
      const bool fusable = ttv_tail_fusable(b);
      // A sweep enqueued ahead starts with the threshold test on the record of the sweep
      // before.  With the fused launch for mode 0, its Gram role finishes that record (Grams
      // of the last mode, the fit), files it and takes the test; otherwise a gate kernel
      // does, and this sweep ends with its own last Grams and record.
      if (n == 0 && p->la_cur) {
        p->la_gate_fused = fusable;
        if (!fusable) {
          int* gate = (int*)p->cur_gate;
          HIPCHK(launch_pp_gate_ring(rec, p->N, p->la_eps_cur, gate, c.ws + p->off_ring, gate + 4, s));
        }
      }
      const bool fin_before = n == 0 && p->la_cur && fusable;
      if (fusable) {
        // contractions, the previous mode's Grams and this mode's head in one launch
        HeadArgs h2 = h;
        GramArgs g2;
        const GramArgs* gp = nullptr;
        if (prev >= 0 || fin_before) {
          const int gm = fin_before ? p->N - 1 : prev;
          g2 = gram_args(c, A, S, gm, 1, normX2, rec, fin_before ? 1 : 0,
                         fin_before ? PPALS_SWEEP_PP_APPROX : kind);
          if (fin_before) {
            int* gate = (int*)p->cur_gate;
            g2.ring = c.ws + p->off_ring;
            g2.ring_ctr = gate + 4;
            g2.gate_out = gate;
            g2.eps = p->la_eps_cur;
          }
          g2.N = h.N;
          g2.next = h.n;
          g2.wterm = h.pp && h.second_order;
          g2.S_all = h.S;
          g2.U_all = h.U;
          g2.gamma_out = h.gamma;
          g2.W_out = h.W;
          gram_split(c, g2);
          h2.gamma_ready = 1;
          gp = &g2;
        }
        {
          Prof pr(p, 1, s, fl, by);
          HIPCHK(launch_ttv_tail(b, gp, h2, tail_ctr, s));
          pr.end();
        }
        st = solve_fused(c, A, n, c.Mp(n), part, nslots, true, n == p->N - 1);
        if (st != PPALS_OK) return st;
        prev = n;
        continue;
      }
      if (prev >= 0) {
        const GramArgs g = gram_args(c, A, S, prev, 1, normX2, rec, 0, kind);
        st = tail_fork(c, &g, &h);
      } else {
        st = tail_fork(c, nullptr, &h);
      }
      if (st != PPALS_OK) return st;
      {
        Prof pr(p, 1, s, fl, by);
        HIPCHK(launch_ttv(b, s));
        pr.end();
      }
      st = tail_join(c);
      if (st == PPALS_OK)
        st = solve_fused(c, A, n, c.Mp(n), part, nslots, true, n == p->N - 1);
      if (st != PPALS_OK) return st;
      prev = n;
    }
    // a sweep enqueued ahead whose first launch took the test leaves its last Grams and
    // record to the next sweep's first launch (or to the kernel after the last one)
    ppals_status st = PPALS_OK;
    if (!(p->la_cur && p->la_gate_fused)) st = finish_sweep_fast(c, A, S, normX2, rec, prev, 1, kind);
    if (st == PPALS_OK) p->sweeps_since_build++;
    return st;
  }
  for (int n = 0; n < p->N; ++n) {
    ppals_status st;
    {
      Prof pr(p, 4, s);
      st = mode_begin(c, S, normX2, rec, n, prev, 1, 0, kind);
      pr.end();
    }
    if (st == PPALS_OK) st = pp_correct(c, A, n, c.M());
    if (st == PPALS_OK) {
      Prof pr(p, 4, s);
      st = solve_mode(c, A, S, n, true);
      pr.end();
    }
    if (st != PPALS_OK) return st;
    prev = n;
  }
  ppals_status st = mode_begin(c, S, normX2, rec, -1, prev, 1, 1, kind);
  if (st == PPALS_OK) p->sweeps_since_build++;
  return st;
}

}  // namespace

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
// A PP-approximated sweep of the rank <= 64 path is a fixed sequence of launches on the
// caller's and the auxiliary stream.  ppals_run captures it once (on a capture stream of
// its own, since the caller's may be the null stream) and replays the graph; the graph
// holds kernels and stream dependencies only.  It is rebuilt whenever the workspace,
// factor, Gram or record pointers or ||X||^2 change.  Every kernel of the captured sweep
// reads a device gate and does nothing when it is closed (the host opens it before this
// replay); la_sweep_graphed replays the same sweep behind the device-side test.
ppals_status pp_sweep_graphed(ppals_plan* p, double* const* A, double* S, double normX2, void* ws,
                              ppals_sweep_record* rec, hipStream_t s) {
  bool same = p->pp_exec && p->g_ws == ws && p->g_rec == rec && p->g_S == S &&
              p->g_normX2 == normX2;
  for (int n = 0; same && n < p->N; ++n) same = p->g_A[n] == A[n];
  if (!same) {
    if (p->pp_exec) (void)hipGraphExecDestroy(p->pp_exec);
    if (p->pp_graph) (void)hipGraphDestroy(p->pp_graph);
    p->pp_exec = nullptr;
    p->pp_graph = nullptr;
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    const int before = p->sweeps_since_build;
    p->cur_gate = (const int*)((char*)ws + p->off_gate);
    ppals_status st = do_pp_sweep(p, A, S, normX2, ws, rec, p->cap_stream);
    p->cur_gate = nullptr;
    p->sweeps_since_build = before;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != PPALS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(PPALS_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    p->pp_graph = g;
    HIPCHK(hipGraphInstantiate(&p->pp_exec, g, nullptr, nullptr, 0));
    p->g_ws = ws;
    p->g_rec = rec;
    p->g_S = S;
    p->g_normX2 = normX2;
    for (int n = 0; n < p->N; ++n) p->g_A[n] = A[n];
  }
  HIPCHK(launch_set_int((int*)((char*)ws + p->off_gate), 1, s));
  HIPCHK(hipGraphLaunch(p->pp_exec, s));
  p->sweeps_since_build++;
  return PPALS_OK;
}

// A host-decided ALS or PP-initialisation sweep replayed from a graph captured on the
// first call (the sequence of launches is fixed by the plan); rebuilt when a pointer or
// ||X||^2 changes.  body enqueues the sweep on the stream it is given; host-side plan state
// it changes is restored after the capture (the caller applies it after each replay).
template <typename Body>
ppals_status sweep_graphed(ppals_plan* p, ppals_plan::SweepGraph& G, const void* X, const void* Xb,
                           double* const* A, double* S, double normX2, void* ws,
                           ppals_sweep_record* rec, hipStream_t s, Body body) {
  bool same = G.e && G.ws == ws && G.rec == rec && G.S == S && G.X == X && G.Xb == Xb &&
              G.normX2 == normX2;
  for (int n = 0; same && n < p->N; ++n) same = G.A[n] == A[n];
  if (!same) {
    if (G.e) (void)hipGraphExecDestroy(G.e);
    if (G.g) (void)hipGraphDestroy(G.g);
    G.e = nullptr;
    G.g = nullptr;
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    const bool built = p->ops_built;
    const int since = p->sweeps_since_build;
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    ppals_status st = body(p->cap_stream);
    p->ops_built = built;
    p->sweeps_since_build = since;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != PPALS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(PPALS_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    G.g = g;
    HIPCHK(hipGraphInstantiate(&G.e, g, nullptr, nullptr, 0));
    G.ws = ws;
    G.rec = rec;
    G.S = S;
    G.X = X;
    G.Xb = Xb;
    G.normX2 = normX2;
    for (int n = 0; n < p->N; ++n) G.A[n] = A[n];
  }
  HIPCHK(hipGraphLaunch(G.e, s));
  return PPALS_OK;
}

// PP-approximated sweep enqueued ahead of the host's decision, replayed from a graph that
// starts with the threshold test of Algorithm 3 on the device (taken by mode 0's fused
// launch, or by k_pp_gate_ring before it), which also files the record before it in the
// ring; rebuilt when a pointer, ||X||^2 or eps changes.
ppals_status la_sweep_graphed(ppals_plan* p, double* const* A, double* S, double normX2, void* ws,
                              ppals_sweep_record* rec, double eps, hipStream_t s) {
  bool same = p->la_exec && p->la_ws == ws && p->la_recp == rec && p->la_S == S &&
              p->la_normX2 == normX2 && p->la_eps == eps;
  for (int n = 0; same && n < p->N; ++n) same = p->la_A[n] == A[n];
  if (!same) {
    if (p->la_exec) (void)hipGraphExecDestroy(p->la_exec);
    if (p->la_graph) (void)hipGraphDestroy(p->la_graph);
    p->la_exec = nullptr;
    p->la_graph = nullptr;
    if (!p->cap_stream) HIPCHK(hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking));
    HIPCHK(hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal));
    int* gate = (int*)((char*)ws + p->off_gate);
    const int before = p->sweeps_since_build;
    p->cur_gate = gate;
    p->la_cur = true;
    p->la_eps_cur = eps;
    const ppals_status st = do_pp_sweep(p, A, S, normX2, ws, rec, p->cap_stream);
    p->la_cur = false;
    p->cur_gate = nullptr;
    p->sweeps_since_build = before;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap_stream, &g);
    if (st != PPALS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return st;
    }
    if (e != hipSuccess) return fail(PPALS_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    p->la_graph = g;
    HIPCHK(hipGraphInstantiate(&p->la_exec, g, nullptr, nullptr, 0));
    p->la_ws = ws;
    p->la_recp = rec;
    p->la_S = S;
    p->la_normX2 = normX2;
    p->la_eps = eps;
    for (int n = 0; n < p->N; ++n) p->la_A[n] = A[n];
  }
  HIPCHK(hipGraphLaunch(p->la_exec, s));
  return PPALS_OK;
}

// Right-hand-side error of the PP update at the current factors (the learned
// controller's label): the exact MTTKRP of every mode through the ALS dimension tree
// without solves, the general PP update of every mode from the operators, and
// err = max_n ||M~^(n) - M^(n)||_F / ||M^(n)||_F.
ppals_status rhs_error(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                       const double* S, void* ws, double* err, hipStream_t s) {
  Ctx c{p, (char*)ws, s};
  double* Mx = c.at<double>(p->off_Mx);
  for (const Op& o : p->dt_ops) {
    ppals_status st = PPALS_OK;
    if (o.kind == OP_L1) {
      const L1Step& l = p->l1[o.idx];
      st = run_l1(c, l, X, Xb, A, c.buf(l.out_buf));
    } else if (o.kind == OP_TTV) {
      const TtvStep& t = p->ttv[o.idx];
      st = run_ttv(c, t, A, t.out_buf < 0 ? Mx + p->mode_off[t.out_mode] : nullptr);
    }
    if (st != PPALS_OK) return st;
  }
  p->dA_zero = false;  // dA is rewritten from the current factors
  for (int i = 0; i < p->N; ++i) {
    const int64_t cnt = p->dims[i] * (int64_t)p->R;
    HIPCHK(launch_sub(c.dA(i), A[i], c.Ap(i), cnt, s));
    HIPCHK(launch_gram(A[i], c.dA(i), p->dims[i], p->R, c.at<double>(p->off_L),
                       c.U() + (size_t)i * p->R * p->R, s));
  }
  double* Mt = c.at<double>(p->off_Mt);
  double* sums = c.at<double>(p->off_errsum);
  for (int n = 0; n < p->N; ++n) {
    ppals_status st = mode_begin(c, (double*)S, 1.0, nullptr, n, -1, 1, 0, PPALS_SWEEP_PP_APPROX);
    if (st == PPALS_OK) st = pp_correct(c, A, n, Mt);
    if (st != PPALS_OK) return st;
    HIPCHK(launch_rhs_err(Mt, Mx + p->mode_off[n], p->dims[n] * (int64_t)p->R, sums + 2 * n, s));
  }
  HIPCHK(launch_rhs_err_max(sums, p->N, err, s));
  return PPALS_OK;
}

namespace {

// The solve behind gram_solve and gram_solve_noalloc.  w is the scratch: L (R x R), the
// per-row partial sums (rows x 4) and the status word, at the offsets of
// ppals_gram_solve_workspace_bytes.  Every entry of it that a kernel reads is written
// earlier in the same call, so nothing in it has to start at zero.
ppals_status gram_solve_impl(int32_t R, int64_t rows, const double* Gamma, const void* M,
                             int32_t m_dtype, double* A_inout, double* grad_norm_out,
                             int32_t* chol_status_out, char* w, hipStream_t s) {
  double* L = (double*)w;
  double* rowpart = (double*)(w + align256((size_t)R * R * 8));
  int* status = (int*)(w + align256((size_t)R * R * 8) + align256((size_t)rows * 4 * 8));
  HIPCHK(launch_chol_standalone(Gamma, R, L, status, s));
  SolveArgs a;
  memset(&a, 0, sizeof(a));
  a.R = R;
  a.rows = rows;
  if (m_dtype == PPALS_FP64) a.M = (const double*)M;
  else a.M32 = (const float*)M;
  a.L = L;
  a.gamma = Gamma;
  a.A = A_inout;
  a.rowpart = rowpart;
  a.status = status;
  a.step = 1.0;
  HIPCHK(launch_solve_rows(a, s));
  HIPCHK(launch_finish_gram_solve(rowpart, rows, grad_norm_out, chol_status_out, status, s));
  return PPALS_OK;
}

ppals_status gram_solve_check(int32_t R, int64_t rows, const double* Gamma, const void* M,
                              int32_t m_dtype, double* A_inout, double* grad_norm_out,
                              int32_t* chol_status_out) {
  if (R < 1 || R > PPALS_MAX_RANK) return fail(PPALS_E_UNSUPPORTED, "rank must be in [1, 128]");
  if (rows < 1) return fail(PPALS_E_ARG, "rows must be >= 1");
  if (!Gamma || !M || !A_inout || !grad_norm_out || !chol_status_out)
    return fail(PPALS_E_ARG, "NULL argument");
  if (m_dtype != PPALS_FP64 && m_dtype != PPALS_FP32)
    return fail(PPALS_E_UNSUPPORTED, "m_dtype must be FP64 or FP32");
  return PPALS_OK;
}

// Scratch of gram_solve_noalloc: a fixed device array of the library, laid out like the
// workspace of gram_solve at the largest supported size.  Each GPU holds its own copy until
// the process ends; host code reaches it only through the address hipGetSymbolAddress
// returns on that GPU (the array's name is a host-side stand-in, not a device address).
constexpr int64_t kNoAllocMaxRows = PPALS_GRAM_SOLVE_NOALLOC_MAX_ROWS;
constexpr size_t kNoAllocBytes = (size_t)PPALS_MAX_RANK * PPALS_MAX_RANK * 8 +
                                 (size_t)kNoAllocMaxRows * 4 * 8 + 256;
static_assert((size_t)PPALS_MAX_RANK * PPALS_MAX_RANK * 8 % 256 == 0, "L block must stay aligned");
static_assert((size_t)kNoAllocMaxRows * 4 * 8 % 256 == 0, "row block must stay aligned");
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
ppals_status scratch_address(char** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PPALS_E_UNSUPPORTED, "device index above 63");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    HIPCHK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PPALS_E_HIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = (char*)g_scratch_ptr[dev];
  return PPALS_OK;
}

}  // namespace

extern "C" {

ppals_status ppals_plan_create(const ppals_desc* d, ppals_plan** out) {
  if (!d || !out) return fail(PPALS_E_ARG, "desc or out is NULL");
  *out = nullptr;
  if (d->order < 3 || d->order > PPALS_MAX_ORDER)
    return fail(PPALS_E_UNSUPPORTED, "order must be in [3, 8]");
  if (d->rank < 1 || d->rank > PPALS_MAX_RANK)
    return fail(PPALS_E_UNSUPPORTED, "rank must be in [1, 128]");
  for (int i = 0; i < d->order; ++i)
    if (d->dims[i] < 1) return fail(PPALS_E_ARG, "dims must be >= 1");
  const bool tier_ok = (d->tensor_dtype == PPALS_FP64 && d->level1_dtype == PPALS_FP64) ||
                       (d->tensor_dtype == PPALS_FP32 &&
                        (d->level1_dtype == PPALS_FP32 || d->level1_dtype == PPALS_BF16));
  if (!tier_ok) return fail(PPALS_E_UNSUPPORTED, "unsupported (tensor_dtype, level1_dtype) pair");
  const double step = d->step_size == 0.0 ? 1.0 : d->step_size;
  if (!(step > 0.0 && step <= 1.0)) return fail(PPALS_E_ARG, "step_size must be in (0, 1] (or 0 for 1)");
  int combine = 1;
  std::string model = "null";
  if (d->order > 3 && d->pp_build_levels != 0) {
    if (d->pp_build_levels < -1)
      return fail(PPALS_E_ARG, "pp_build_levels must be -1 (automatic), 0 or >= 1");
    std::vector<double> est;
    combine = choose_combine(d, d->pp_build_levels, &est);
    if (combine < 0) {
      return fail(PPALS_E_UNSUPPORTED,
                  combine == -1 ? "combined operator build needs the FP64 or FP32 first level"
                                : "combined operator build: contracted extent above 2^31 - 64");
    }
    if (!est.empty()) {
      model = "[";
      for (size_t l = 0; l < est.size(); ++l) {
        char t[64];
        snprintf(t, sizeof(t), "%s%.4g", l ? "," : "", est[l]);
        model += t;
      }
      model += "]";
    }
  }
  ppals_plan* p = new ppals_plan();
  p->combine = combine;
  p->combine_auto = d->order > 3 && d->pp_build_levels == -1;
  p->combine_model = model;
  p->step = step;
  p->N = d->order;
  p->R = d->rank;
  for (int i = 0; i < p->N; ++i) p->dims[i] = d->dims[i];
  p->tdt = d->tensor_dtype;
  p->l1dt = d->level1_dtype;
  p->bulk = d->tensor_dtype == PPALS_FP64 ? DT_F64 : DT_F32;
  p->second_order = d->use_second_order ? 1 : 0;
  p->fast = p->R <= 64;
  p->mode_off.resize(p->N);
  for (int i = 0; i < p->N; ++i) {
    p->mode_off[i] = (size_t)p->sum_s * p->R;
    p->sum_s += p->dims[i];
    p->max_s = std::max(p->max_s, p->dims[i]);
  }
  build_dt(p);
  prune_dt(p);
  build_pp(p);
  find_reuse(p);
  layout(p);
  make_describe(p);
  *out = p;
  return PPALS_OK;
}

void ppals_plan_destroy(ppals_plan* p) {
  if (!p) return;
  for (auto& e : p->pending) {
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  for (auto e : p->pool) (void)hipEventDestroy(e);
  if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
  if (p->ev_join) (void)hipEventDestroy(p->ev_join);
  if (p->aux) (void)hipStreamDestroy(p->aux);
  if (p->pinned_rec) (void)hipHostFree(p->pinned_rec);
  if (p->pp_exec) (void)hipGraphExecDestroy(p->pp_exec);
  if (p->pp_graph) (void)hipGraphDestroy(p->pp_graph);
  if (p->la_exec) (void)hipGraphExecDestroy(p->la_exec);
  if (p->la_graph) (void)hipGraphDestroy(p->la_graph);
  for (auto* G : {&p->als_g, &p->init_g, &p->init_rg}) {
    if (G->e) (void)hipGraphExecDestroy(G->e);
    if (G->g) (void)hipGraphDestroy(G->g);
  }
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  if (p->la_rec) (void)hipHostFree(p->la_rec);
  for (int k = 0; k < ppals_plan::kLookahead; ++k) {
    if (p->la_e0[k]) (void)hipEventDestroy(p->la_e0[k]);
    if (p->la_e1[k]) (void)hipEventDestroy(p->la_e1[k]);
  }
  delete p;
}

ppals_status ppals_mlp_forward(const float* params, int32_t d, int32_t hidden, const float* X,
                               int64_t B, float* y, float* hcache, hipStream_t s) {
  if (!params || !X || !y) return fail(PPALS_E_ARG, "NULL argument");
  if (d < 1 || d > MLP_MAX_IN) return fail(PPALS_E_UNSUPPORTED, "need 1 <= d <= 16");
  if (hidden < 1 || hidden > MLP_MAX_HIDDEN) return fail(PPALS_E_UNSUPPORTED, "need 1 <= hidden <= 1024");
  if (B < 0) return fail(PPALS_E_ARG, "B < 0");
  HIPCHK(launch_mlp_forward(params, d, hidden, X, B, y, hcache, s));
  return PPALS_OK;
}

ppals_status ppals_mlp_backward(const float* params, int32_t d, int32_t hidden, const float* X,
                                const float* hcache, const float* y, const float* t, int64_t B,
                                float* grad, float* loss, hipStream_t s) {
  if (!params || !X || !hcache || !y || !t || !grad) return fail(PPALS_E_ARG, "NULL argument");
  if (d < 1 || d > MLP_MAX_IN) return fail(PPALS_E_UNSUPPORTED, "need 1 <= d <= 16");
  if (hidden < 1 || hidden > MLP_MAX_HIDDEN) return fail(PPALS_E_UNSUPPORTED, "need 1 <= hidden <= 1024");
  if (B < 1) return fail(PPALS_E_ARG, "B < 1");
  HIPCHK(launch_mlp_backward(params, d, hidden, X, hcache, y, t, B, grad, loss, s));
  return PPALS_OK;
}

ppals_status ppals_mlp_adam(float* params, const float* grad, float* m, float* v, int64_t P,
                            int32_t step, float lr, float beta1, float beta2, float eps,
                            hipStream_t s) {
  if (!params || !grad || !m || !v) return fail(PPALS_E_ARG, "NULL argument");
  if (P < 0) return fail(PPALS_E_ARG, "P < 0");
  if (step < 1) return fail(PPALS_E_ARG, "step must be >= 1");
  if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f))
    return fail(PPALS_E_ARG, "betas must lie in [0, 1)");
  if (P == 0) return PPALS_OK;
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  HIPCHK(launch_mlp_adam(params, grad, m, v, P, lr, beta1, beta2, eps, c1, c2, s));
  return PPALS_OK;
}

ppals_status ppals_pp_rhs_error(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                                const double* S, void* ws, double* err, hipStream_t s) {
  ppals_status st = check_common(p, X, Xb, A, ws);
  if (st != PPALS_OK) return st;
  if (!S || !err) return fail(PPALS_E_ARG, "NULL argument");
  if (!p->ops_built) return fail(PPALS_E_STATE, "operators not built");
  return rhs_error(p, X, Xb, A, S, ws, err, s);
}

ppals_status ppals_set_controller(ppals_plan* p, const ppals_controller* ctl) {
  if (!p) return fail(PPALS_E_ARG, "plan is NULL");
  if (!ctl) {
    p->ctl_set = false;
    return PPALS_OK;
  }
  if (!ctl->params) return fail(PPALS_E_ARG, "controller params are NULL");
  if (ctl->hidden < 1 || ctl->hidden > MLP_MAX_HIDDEN)
    return fail(PPALS_E_UNSUPPORTED, "need 1 <= hidden <= 1024");
  if (p->N + 2 > MLP_MAX_IN) return fail(PPALS_E_UNSUPPORTED, "order + 2 exceeds 16 inputs");
  if (ctl->check_period < 0) return fail(PPALS_E_ARG, "check_period < 0");
  if (!(ctl->rho_cap > 0.0)) return fail(PPALS_E_ARG, "rho_cap must be > 0");
  if (!(ctl->fallback_factor > 0.0)) return fail(PPALS_E_ARG, "fallback_factor must be > 0");
  p->ctl = *ctl;
  p->ctl_set = true;
  return PPALS_OK;
}

ppals_status ppals_set_profiling(ppals_plan* p, int32_t enable) {
  if (!p) return fail(PPALS_E_ARG, "plan is NULL");
  p->prof = enable != 0;
  return PPALS_OK;
}

ppals_status ppals_get_profile(ppals_plan* p, ppals_kernel_stat* out, int32_t max_entries,
                               int32_t* n_out, int32_t reset) {
  if (!p || !out || !n_out) return fail(PPALS_E_ARG, "NULL argument");
  prof_resolve(p);
  const int n = std::min<int>(max_entries, PPALS_PROF_CLASSES);
  for (int i = 0; i < n; ++i) {
    out[i] = p->stats[i];
    snprintf(out[i].name, sizeof(out[i].name), "%s", kProfNames[i]);
  }
  *n_out = n;
  if (reset) memset(p->stats, 0, sizeof(p->stats));
  return PPALS_OK;
}

size_t ppals_workspace_bytes(const ppals_plan* p) { return p ? p->ws_bytes : 0; }

ppals_status ppals_plan_describe(const ppals_plan* p, char* buf, size_t len) {
  if (!p || !buf) return fail(PPALS_E_ARG, "plan or buf is NULL");
  if (len < p->describe.size() + 1) return fail(PPALS_E_ARG, "buffer too small");
  memcpy(buf, p->describe.c_str(), p->describe.size() + 1);
  return PPALS_OK;
}

ppals_status cp_als_sweep(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                          double* S, double normX2, void* ws, ppals_sweep_record* rec,
                          hipStream_t s) {
  ppals_status st = check_common(p, X, Xb, A, ws);
  if (st != PPALS_OK) return st;
  if (!S || !rec) return fail(PPALS_E_ARG, "S or rec is NULL");
  if (!(normX2 > 0.0)) return fail(PPALS_E_ARG, "normX2 must be > 0");
  return do_als_sweep(p, X, Xb, A, S, normX2, ws, rec, s);
}

ppals_status pp_build_operators(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                                void* ws, hipStream_t s) {
  ppals_status st = check_common(p, X, Xb, A, ws);
  if (st != PPALS_OK) return st;
  return do_pp_build(p, X, Xb, A, ws, s);
}

ppals_status pp_sweep(ppals_plan* p, double* const* A, double* S, double normX2, void* ws,
                      ppals_sweep_record* rec, hipStream_t s) {
  if (!p || !A || !S || !rec) return fail(PPALS_E_ARG, "NULL argument");
  if (!ws) return fail(PPALS_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(PPALS_E_WORKSPACE, "workspace is not 256-byte aligned");
  for (int n = 0; n < p->N; ++n)
    if (!A[n]) return fail(PPALS_E_ARG, "A[n] is NULL");
  if (!p->ops_built) return fail(PPALS_E_STATE, "pp_sweep before pp_build_operators");
  if (!(normX2 > 0.0)) return fail(PPALS_E_ARG, "normX2 must be > 0");
  return do_pp_sweep(p, A, S, normX2, ws, rec, s);
}

size_t ppals_gram_solve_workspace_bytes(int32_t R, int64_t rows) {
  if (R < 1 || rows < 1) return 0;
  return align256((size_t)R * R * 8) + align256((size_t)rows * 4 * 8) + 256;
}

ppals_status gram_solve(int32_t R, int64_t rows, const double* Gamma, const void* M,
                        int32_t m_dtype, double* A_inout, double* grad_norm_out,
                        int32_t* chol_status_out, void* ws, hipStream_t s) {
  ppals_status st = gram_solve_check(R, rows, Gamma, M, m_dtype, A_inout, grad_norm_out,
                                     chol_status_out);
  if (st != PPALS_OK) return st;
  if (!ws) return fail(PPALS_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(PPALS_E_WORKSPACE, "workspace is not 256-byte aligned");
  return gram_solve_impl(R, rows, Gamma, M, m_dtype, A_inout, grad_norm_out, chol_status_out,
                         (char*)ws, s);
}

ppals_status gram_solve_noalloc(int32_t R, int64_t rows, const double* Gamma, const void* M,
                                int32_t m_dtype, double* A_inout, double* grad_norm_out,
                                int32_t* chol_status_out, hipStream_t s) {
  ppals_status st = gram_solve_check(R, rows, Gamma, M, m_dtype, A_inout, grad_norm_out,
                                     chol_status_out);
  if (st != PPALS_OK) return st;
  if (rows > kNoAllocMaxRows)
    return fail(PPALS_E_UNSUPPORTED, "gram_solve_noalloc: rows = " + std::to_string(rows) +
                                         " exceeds the fixed scratch limit of " +
                                         std::to_string(kNoAllocMaxRows) + " rows");
  char* w = nullptr;
  st = scratch_address(&w);
  if (st != PPALS_OK) return st;
  return gram_solve_impl(R, rows, Gamma, M, m_dtype, A_inout, grad_norm_out, chol_status_out, w,
                         s);
}

size_t ppals_norm2_workspace_bytes(void) { return 1024 * sizeof(double); }

ppals_status ppals_tensor_norm2(const void* X, int32_t dtype, int64_t count, double* out,
                                void* ws, hipStream_t s) {
  if (!X || !out) return fail(PPALS_E_ARG, "NULL argument");
  if (!ws) return fail(PPALS_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(PPALS_E_WORKSPACE, "workspace is not 256-byte aligned");
  if (dtype != PPALS_FP64 && dtype != PPALS_FP32) return fail(PPALS_E_UNSUPPORTED, "dtype");
  if (count < 1) return fail(PPALS_E_ARG, "count must be >= 1");
  HIPCHK(launch_norm2(X, dtype == PPALS_FP64 ? DT_F64 : DT_F32, count, (double*)ws, 1024, out, s));
  return PPALS_OK;
}

ppals_status ppals_cast_bf16(const float* in, uint16_t* out, int64_t count, hipStream_t s) {
  if (!in || !out) return fail(PPALS_E_ARG, "NULL argument");
  if (count < 0) return fail(PPALS_E_ARG, "count must be >= 0");
  if (count == 0) return PPALS_OK;
  HIPCHK(launch_cast_bf16(in, out, count, s));
  return PPALS_OK;
}

ppals_status ppals_level1(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                          uint32_t mask, void* out, void* ws, hipStream_t s) {
  ppals_status st = check_common(p, X, Xb, A, ws);
  if (st != PPALS_OK) return st;
  if (!out) return fail(PPALS_E_ARG, "out is NULL");
  int lo = -1, hi = -1;
  for (int i = 0; i < p->N; ++i)
    if (mask & (1u << i)) {
      if (lo < 0) lo = i;
      hi = i + 1;
    }
  if (lo < 0 || (mask >> p->N) != 0) return fail(PPALS_E_ARG, "contract_mask empty or out of range");
  for (int i = lo; i < hi; ++i)
    if (!(mask & (1u << i))) return fail(PPALS_E_ARG, "contract_mask must be contiguous");
  if (hi - lo == p->N) return fail(PPALS_E_ARG, "cannot contract every mode");
  L1Step stp;
  stp.lo = lo;
  stp.hi = hi;
  stp.geom = l1_config(p, lo, hi);
  // the workspace was sized for the plan's own contractions
  Level1Geom& g = stp.geom;
  if ((size_t)g.nslices * g.Kpad * 16 * g.NB * esize(p->l1dt) > p->sz_B)
    return fail(PPALS_E_UNSUPPORTED, "contraction larger than the plan's operand buffer");
  if (g.ksplit > 1 && (size_t)g.ksplit * g.M * p->R * esize(p->bulk) > p->sz_l1part) {
    g.ksplit = 1;
    g.kchunk = g.Kpad;
  }
  Ctx c{p, (char*)ws, s};
  return run_l1(c, stp, X, Xb, A, out);
}

ppals_status ppals_mttkrp(ppals_plan* p, const void* X, const void* Xb, double* const* A,
                          int32_t mode, void* out, void* ws, hipStream_t s) {
  ppals_status st = check_common(p, X, Xb, A, ws);
  if (st != PPALS_OK) return st;
  if (!out) return fail(PPALS_E_ARG, "out is NULL");
  if (mode < 0 || mode >= p->N) return fail(PPALS_E_ARG, "mode out of range");
  // Run the ALS tree up to the first time M^(mode) is formed, without solving.
  Ctx c{p, (char*)ws, s};
  for (const Op& o : p->dt_ops) {
    if (o.kind == OP_L1) {
      const L1Step& l = p->l1[o.idx];
      st = run_l1(c, l, X, Xb, A, c.buf(l.out_buf));
    } else if (o.kind == OP_TTV) {
      const TtvStep& t = p->ttv[o.idx];
      if (t.out_buf < 0 && t.out_mode != mode) continue;
      st = run_ttv(c, t, A, t.out_buf < 0 ? (double*)out : nullptr);
      if (st == PPALS_OK && t.out_buf < 0 && t.out_mode == mode) return PPALS_OK;
    }
    if (st != PPALS_OK) return st;
  }
  return fail(PPALS_E_STATE, "mode not produced by the dimension tree");
}

ppals_status ppals_pp_rhs(ppals_plan* p, double* const* A, const double* S, int32_t mode,
                          double* out, void* ws, hipStream_t s) {
  if (!p || !A || !S || !out) return fail(PPALS_E_ARG, "NULL argument");
  if (!ws) return fail(PPALS_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(PPALS_E_WORKSPACE, "workspace is not 256-byte aligned");
  if (mode < 0 || mode >= p->N) return fail(PPALS_E_ARG, "mode out of range");
  if (!p->ops_built) return fail(PPALS_E_STATE, "operators not built");
  Ctx c{p, (char*)ws, s};
  // dA_i = A_i - A_p,i and U_i = A_i^T dA_i for every mode (the gram kernel's S
  // output goes to the L scratch, which mode_begin overwrites afterwards)
  p->dA_zero = false;  // dA is rewritten from the current factors
  for (int i = 0; i < p->N; ++i) {
    const int64_t cnt = p->dims[i] * (int64_t)p->R;
    HIPCHK(launch_sub(c.dA(i), A[i], c.Ap(i), cnt, s));
    HIPCHK(launch_gram(A[i], c.dA(i), p->dims[i], p->R, c.at<double>(p->off_L),
                       c.U() + (size_t)i * p->R * p->R, s));
  }
  ppals_status st = mode_begin(c, (double*)S, 1.0, nullptr, mode, -1, 1, 0, PPALS_SWEEP_PP_APPROX);
  if (st != PPALS_OK) return st;
  return pp_correct(c, A, mode, out);
}

ppals_status ppals_get_operator(ppals_plan* p, const void* ws, int32_t i, int32_t j, void* out,
                                hipStream_t s) {
  if (!p || !ws || !out) return fail(PPALS_E_ARG, "NULL argument");
  if (!(0 <= i && i < j && j < p->N)) return fail(PPALS_E_ARG, "need 0 <= i < j < N");
  if (!p->ops_built) return fail(PPALS_E_STATE, "operators not built");
  const BufDesc& b = p->bufs[p->leaf_buf[i][j]];
  const size_t bytes = (size_t)p->dims[i] * p->dims[j] * p->R * esize(p->bulk);
  HIPCHK(hipMemcpyAsync(out, (const char*)ws + b.off, bytes, hipMemcpyDeviceToDevice, s));
  return PPALS_OK;
}

ppals_status ppals_exact_residual2(ppals_plan* p, const void* X, double* const* A, double* out,
                                   void* ws, hipStream_t s) {
  if (!p || !X || !A || !out) return fail(PPALS_E_ARG, "NULL argument");
  if (!ws) return fail(PPALS_E_WORKSPACE, "workspace is NULL");
  if ((uintptr_t)ws % 256 != 0) return fail(PPALS_E_WORKSPACE, "workspace is not 256-byte aligned");
  Ctx c{p, (char*)ws, s};
  HIPCHK(launch_residual2(X, p->bulk, A, p->dims, p->N, p->R, c.at<double>(p->off_norm), 4096,
                          out, s));
  return PPALS_OK;
}

ppals_status ppals_run(ppals_plan* p, const void* X, const void* Xb, double* const* A, double* S,
                       double normX2, void* ws, ppals_sweep_record* rec_dev, double eps,
                       double delta, int32_t max_sweeps, const int32_t* replay,
                       ppals_sweep_record* host_records, float* sweep_ms, int32_t* n_done,
                       hipStream_t s) {
  ppals_status st = check_common(p, X, Xb, A, ws);
  if (st != PPALS_OK) return st;
  if (!S || !rec_dev || !host_records || !n_done) return fail(PPALS_E_ARG, "NULL argument");
  if (max_sweeps < 0) return fail(PPALS_E_ARG, "max_sweeps < 0");
  if (!(normX2 > 0.0)) return fail(PPALS_E_ARG, "normX2 must be > 0");
  *n_done = 0;
  for (int n = 0; n < p->N; ++n)
    HIPCHK(launch_gram(A[n], nullptr, p->dims[n], p->R, S + (size_t)n * p->R * p->R, nullptr, s));
  p->ops_built = false;
  std::vector<double> rel(p->N, 1.0);
  const double normX = std::sqrt(normX2);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (sweep_ms) {
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
  }
  int prev_kind = -1;
  // learned controller: decides whether to stay in the PP phase until a periodic
  // check of the true right-hand-side error falls back to the threshold rule
  bool ctl_on = p->ctl_set;
  bool leave_pp = false;
  int pp_count = 0;
  bool fell_back = false;
  const double tau = std::pow(10.0, p->ctl.log10_tau);
  for (int it = 0; it < max_sweeps; ++it) {
    int kind;
    const bool in_pp = prev_kind == PPALS_SWEEP_PP_INIT || prev_kind == PPALS_SWEEP_PP_APPROX;
    if (replay) {
      kind = replay[it];
    } else if (in_pp && ctl_on) {
      bool stay = !leave_pp;
      for (int n = 0; n < p->N; ++n) stay = stay && rel[n] < p->ctl.rho_cap;
      kind = stay ? PPALS_SWEEP_PP_APPROX : PPALS_SWEEP_ALS;
    } else {
      bool small = eps > 0.0;
      for (int n = 0; n < p->N; ++n) small = small && rel[n] < eps;
      kind = small ? (prev_kind == PPALS_SWEEP_ALS || prev_kind < 0 ? PPALS_SWEEP_PP_INIT
                                                                     : PPALS_SWEEP_PP_APPROX)
                   : PPALS_SWEEP_ALS;
    }
    // Inside a PP phase, with no controller, replay, gradient stop or profiling, up to
    // kLookahead PP-approximated sweeps are enqueued at once; a device gate before each
    // takes the threshold test of Algorithm 3 on the previous sweep's record, and the
    // sweeps after the first failed test do nothing.  One synchronisation serves them all.
    if (kind == PPALS_SWEEP_PP_APPROX && !replay && !ctl_on && !(delta > 0.0) && p->fast &&
        !p->prof && p->ops_built && p->sweeps_since_build > 0) {
      // how many sweeps to enqueue: the sweeps left before the largest relative change
      // reaches eps, extrapolated linearly from the last two sweeps of this PP phase
      int L = 2;
      if (it >= 1 && host_records[it - 1].sweep_kind != PPALS_SWEEP_ALS) {
        double r1 = 0.0, r0 = 0.0;
        for (int n = 0; n < p->N; ++n) {
          r1 = std::max(r1, rel[n]);
          if (it >= 2) r0 = std::max(r0, host_records[it - 2].rel_change[n]);
        }
        if (it >= 2 && host_records[it - 2].sweep_kind == PPALS_SWEEP_PP_APPROX && r1 > r0)
          L = 1 + (int)std::min<double>(ppals_plan::kLookahead,
                                        std::max(0.0, std::floor((eps - r1) / (r1 - r0))));
      }
      L = std::max(1, std::min(L, std::min(ppals_plan::kLookahead, max_sweeps - it)));
      if (!p->la_rec)
        HIPCHK(hipHostMalloc((void**)&p->la_rec, sizeof(ppals_sweep_record) * ppals_plan::kLookahead,
                             hipHostMallocDefault));
      for (int k = 0; k < L && sweep_ms; ++k) {
        if (!p->la_e0[k]) HIPCHK(hipEventCreate(&p->la_e0[k]));
        if (!p->la_e1[k]) HIPCHK(hipEventCreate(&p->la_e1[k]));
      }
      int* gate = (int*)((char*)ws + p->off_gate);
      ppals_sweep_record* ring = (ppals_sweep_record*)((char*)ws + p->off_ring);
      HIPCHK(launch_set_int2(gate, 1, gate + 4, 0, s));
      for (int k = 0; k < L; ++k) {
        if (sweep_ms) HIPCHK(hipEventRecord(p->la_e0[k], s));
        st = la_sweep_graphed(p, A, S, normX2, ws, rec_dev, eps, s);
        if (st != PPALS_OK) return st;
        if (sweep_ms) HIPCHK(hipEventRecord(p->la_e1[k], s));
      }
      if (p->la_gate_fused) {
        // the last enqueued sweep's Grams of its last mode, fit and record (if it ran)
        Ctx c{p, (char*)ws, s};
        GramArgs g = gram_args(c, A, S, p->N - 1, 1, normX2, rec_dev, 1, PPALS_SWEEP_PP_APPROX);
        gram_split(c, g);
        g.gate = gate;
        HIPCHK(launch_gram_tiles(g, s, true));
      }
      // ring[0] holds the record before the first enqueued sweep, ring[k + 1] that of sweep k
      HIPCHK(launch_rec_store(rec_dev, ring, gate + 4, s));
      HIPCHK(hipMemcpyAsync(p->la_rec, ring + 1, sizeof(ppals_sweep_record) * L,
                            hipMemcpyDeviceToHost, s));
      HIPCHK(sync_spin(s));
      int ran = 0;
      while (ran < L && p->la_rec[ran].sweep_kind == PPALS_SWEEP_PP_APPROX) ++ran;
      if (ran == 0) return fail(PPALS_E_STATE, "device gate closed a sweep the host opened");
      for (int k = 0; k < ran; ++k) {
        ppals_sweep_record& hr = host_records[it];
        hr = p->la_rec[k];
        if (sweep_ms) HIPCHK(hipEventElapsedTime(&sweep_ms[it], p->la_e0[k], p->la_e1[k]));
        hr.sweep_kind = PPALS_SWEEP_PP_APPROX;
        hr.ctrl_pred = std::nan("");
        hr.ctrl_leave = -1;
        hr.ctrl_true_err = -1.0;
        hr.ctrl_fallback = fell_back ? 1 : 0;
        for (int n = 0; n < p->N; ++n) rel[n] = hr.rel_change[n];
        p->sweeps_since_build++;
        prev_kind = PPALS_SWEEP_PP_APPROX;
        ++it;
        *n_done = it;
      }
      --it;  // the loop increments
      continue;
    }
    if (sweep_ms) HIPCHK(hipEventRecord(e0, s));
    const bool graph_ok = p->fast && !p->prof;
    if (kind == PPALS_SWEEP_PP_INIT) {
      // right after an ALS sweep of this run, its tree's buffer holds one build tensor
      const bool reuse = prev_kind == PPALS_SWEEP_ALS && p->reuse_l1 >= 0;
      if (graph_ok) {
        st = sweep_graphed(p, reuse ? p->init_rg : p->init_g, X, Xb, A, S, normX2, ws, rec_dev, s,
                           [&](hipStream_t cs) {
          ppals_status r = do_pp_build(p, X, Xb, A, ws, cs, reuse);
          if (r == PPALS_OK) r = do_pp_sweep(p, A, S, normX2, ws, rec_dev, cs);
          return r;
        });
        if (st == PPALS_OK) {
          p->ops_built = true;
          p->sweeps_since_build = 1;
        }
      } else {
        st = do_pp_build(p, X, Xb, A, ws, s, reuse);
        if (st == PPALS_OK) st = do_pp_sweep(p, A, S, normX2, ws, rec_dev, s);
      }
    } else if (kind == PPALS_SWEEP_PP_APPROX) {
      if (!p->ops_built) return fail(PPALS_E_STATE, "replay asks for pp_approx before a build");
      // graph replay unless per-kernel profiling is on (its events are host-side state)
      if (p->fast && !p->prof && p->sweeps_since_build > 0)
        st = pp_sweep_graphed(p, A, S, normX2, ws, rec_dev, s);
      else
        st = do_pp_sweep(p, A, S, normX2, ws, rec_dev, s);
    } else if (graph_ok) {
      st = sweep_graphed(p, p->als_g, X, Xb, A, S, normX2, ws, rec_dev, s, [&](hipStream_t cs) {
        return do_als_sweep(p, X, Xb, A, S, normX2, ws, rec_dev, cs);
      });
    } else {
      st = do_als_sweep(p, X, Xb, A, S, normX2, ws, rec_dev, s);
    }
    if (st != PPALS_OK) return st;
    const bool pp_kind = kind != PPALS_SWEEP_ALS;
    bool checked = false;
    if (ctl_on && pp_kind) {
      HIPCHK(launch_mlp_decide(p->ctl.params, p->ctl.hidden, p->N, rec_dev, it, p->ctl.log10_tau, s));
      ++pp_count;
      if (p->ctl.check_period > 0 && pp_count % p->ctl.check_period == 0) {
        st = rhs_error(p, X, Xb, A, S, ws, &rec_dev->ctrl_true_err, s);
        if (st != PPALS_OK) return st;
        checked = true;
      }
    }
    // the sweep's time includes the controller's inference and checks
    if (sweep_ms) HIPCHK(hipEventRecord(e1, s));
    if (!p->pinned_rec)
      HIPCHK(hipHostMalloc((void**)&p->pinned_rec, sizeof(ppals_sweep_record), hipHostMallocDefault));
    HIPCHK(hipMemcpyAsync(p->pinned_rec, rec_dev, sizeof(ppals_sweep_record), hipMemcpyDeviceToHost,
                          s));
    HIPCHK(sync_spin(s));
    host_records[it] = *p->pinned_rec;
    ppals_sweep_record& hr = host_records[it];
    if (sweep_ms) HIPCHK(hipEventElapsedTime(&sweep_ms[it], e0, e1));
    if (p->prof) prof_resolve(p);
    hr.sweep_kind = kind;
    if (!(ctl_on && pp_kind)) {
      hr.ctrl_pred = std::nan("");
      hr.ctrl_leave = -1;
    }
    if (!checked) hr.ctrl_true_err = -1.0;
    if (checked && hr.ctrl_true_err > p->ctl.fallback_factor * tau) {
      ctl_on = false;
      fell_back = true;
    }
    hr.ctrl_fallback = fell_back ? 1 : 0;
    leave_pp = ctl_on && pp_kind && hr.ctrl_leave == 1;
    for (int n = 0; n < p->N; ++n) rel[n] = hr.rel_change[n];
    prev_kind = kind;
    *n_done = it + 1;
    if (delta > 0.0) {
      double g = 0;
      for (int n = 0; n < p->N; ++n) g += hr.grad_norm[n];
      if (g <= delta * normX) break;
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  return PPALS_OK;
}

}  // extern "C"
