// Batched PP-CP-ALS engine: many independent order-3 decompositions advanced together
// by grouped kernels (k_batch.hip), with per-problem state machines on the device, a
// whole batched sweep captured once in a HIP graph and replayed, and first-level
// contraction tile shapes chosen per (rank, size) bucket by a measuring autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/ppals.h"
#include "batch.h"
#include "common.h"

namespace ppk {
ppals_status set_error(ppals_status st, const std::string& msg);
}

using namespace ppk;

#define BHIPCHK(expr)                                                                         \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return set_error(PPALS_E_HIP, std::string(#expr) + ": " + hipGetErrorString(e_));      \
  } while (0)

namespace {

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

constexpr int NBUCKET_R = 4, NBUCKET_S = 3;
int bucket_of(const ppals_batch_problem& p) {
  const int rb = std::min(NBUCKET_R - 1, (p.rank - 1) / 16);
  const int smax = std::max(p.dims[0], std::max(p.dims[1], p.dims[2]));
  const int sb = smax <= 64 ? 0 : (smax <= 128 ? 1 : 2);
  return rb * NBUCKET_S + sb;
}

}  // namespace

struct ppals_batch {
  int count = 0;
  int max_sweeps = 0;
  int maxR = 0, max_s = 0;
  std::vector<ppals_batch_problem> probs;
  std::vector<size_t> off_op[3], off_Mp[3], off_Ap[3], off_dA[3], off_Af[3], off_S, off_U, off_M,
      off_klog;
  size_t off_prob = 0, off_state = 0, off_conf = 0, off_tiles = 0, tiles_bytes = 0;
  size_t ws_bytes = 0;
  std::vector<int> variant;                 // GEMM tile variant per problem
  int bucket_variant[NBUCKET_R * NBUCKET_S];
  double bucket_ms[NBUCKET_R * NBUCKET_S][BATCH_GEMM_VARIANTS];
  bool tuned = false;
  // tile lists (host copies; device copies at off_tiles)
  std::vector<BTile> tiles;
  int g_off[3][BATCH_GEMM_VARIANTS], g_cnt[3][BATCH_GEMM_VARIANTS];
  int t_off[3], t_cnt[3];
  std::vector<BProb> hprob;
  BConf hconf{};
  char* bound_ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char* graph_ws = nullptr;
  hipStream_t graph_stream = nullptr;  // capture stream (default priority)
};

namespace {

void build_tiles(ppals_batch* b) {
  b->tiles.clear();
  for (int c = 0; c < 3; ++c)
    for (int v = 0; v < BATCH_GEMM_VARIANTS; ++v) {
      b->g_off[c][v] = (int)b->tiles.size();
      for (int p = 0; p < b->count; ++p) {
        if (b->variant[p] != v) continue;
        const auto& q = b->probs[p];
        int64_t M = 1;
        for (int i = 0; i < 3; ++i)
          if (i != c) M *= q.dims[i];
        for (int64_t m0 = 0; m0 < M; m0 += BATCH_RUN_ROWS) b->tiles.push_back(BTile{p, (int)m0});
      }
      b->g_cnt[c][v] = (int)b->tiles.size() - b->g_off[c][v];
    }
  for (int n = 0; n < 3; ++n) {
    b->t_off[n] = (int)b->tiles.size();
    for (int p = 0; p < b->count; ++p) {
      const int64_t cnt = (int64_t)b->probs[p].dims[n] * b->probs[p].rank;
      for (int64_t e0 = 0; e0 < cnt; e0 += 256) b->tiles.push_back(BTile{p, (int)e0});
    }
    b->t_cnt[n] = (int)b->tiles.size() - b->t_off[n];
  }
}

size_t max_tiles_bytes(const ppals_batch* b) {
  // one GEMM work item per BATCH_RUN_ROWS rows of each contraction, one TTV tile per
  // 256 output elements
  size_t n = 0;
  for (const auto& q : b->probs) {
    for (int c = 0; c < 3; ++c) {
      int64_t M = 1;
      for (int i = 0; i < 3; ++i)
        if (i != c) M *= q.dims[i];
      n += (size_t)((M + BATCH_RUN_ROWS - 1) / BATCH_RUN_ROWS);
    }
    for (int i = 0; i < 3; ++i) n += (size_t)(((int64_t)q.dims[i] * q.rank + 255) / 256);
  }
  return n * sizeof(BTile);
}

ppals_status upload_tiles(ppals_batch* b, hipStream_t s) {
  if (b->tiles.size() * sizeof(BTile) > b->tiles_bytes)
    return set_error(PPALS_E_WORKSPACE, "tile list exceeds its workspace region");
  BHIPCHK(hipMemcpyAsync(b->bound_ws + b->off_tiles, b->tiles.data(), b->tiles.size() * sizeof(BTile),
                         hipMemcpyHostToDevice, s));
  BHIPCHK(hipStreamSynchronize(s));
  return PPALS_OK;
}

ppals_status enqueue_sweep(ppals_batch* b, char* ws, hipStream_t s) {
  BProb* pr = (BProb*)(ws + b->off_prob);
  BState* st = (BState*)(ws + b->off_state);
  const BConf* cf = (const BConf*)(ws + b->off_conf);
  const BTile* tl = (const BTile*)(ws + b->off_tiles);
  const int C = b->count;
  auto gemm = [&](int c, int out, int mask) -> ppals_status {
    for (int v = 0; v < BATCH_GEMM_VARIANTS; ++v)
      BHIPCHK(launch_b_gemm(v, pr, st, tl + b->g_off[c][v], b->g_cnt[c][v], c, out, mask, s));
    return PPALS_OK;
  };
  ppals_status r;
  BHIPCHK(launch_b_begin(st, pr, cf, C, s));
  BHIPCHK(launch_b_prep(pr, st, C, s));
  if ((r = gemm(2, 0, BMASK_ALS | BMASK_INIT)) != PPALS_OK) return r;  // X x_2 A^(2)
  if ((r = gemm(1, 1, BMASK_INIT)) != PPALS_OK) return r;              // X x_1 A^(1)
  if ((r = gemm(0, 2, BMASK_INIT)) != PPALS_OK) return r;              // X x_0 A^(0)
  for (int n = 0; n < 3; ++n) BHIPCHK(launch_b_ttv(pr, st, tl + b->t_off[n], b->t_cnt[n], n, 1, s));
  for (int n = 0; n < 3; ++n) {
    BHIPCHK(launch_b_ttv(pr, st, tl + b->t_off[n], b->t_cnt[n], n, 0, s));
    BHIPCHK(launch_b_solve(pr, st, cf, C, n, b->maxR, s));
    if (n != 1) BHIPCHK(launch_b_f32(pr, st, C, n == 0 ? 1 : 6, s));  // FP32 factor copies
    if (n == 0 && (r = gemm(0, 2, BMASK_ALS)) != PPALS_OK) return r;  // X x_0 A^(0), updated
  }
  BHIPCHK(launch_b_end(st, cf, C, s));
  return PPALS_OK;
}

void drop_graph(ppals_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_ws = nullptr;
}

}  // namespace

extern "C" {

ppals_status ppals_batch_create(const ppals_batch_problem* probs, int32_t count,
                                int32_t max_sweeps, ppals_batch** out) {
  if (!probs || !out) return set_error(PPALS_E_ARG, "NULL argument");
  *out = nullptr;
  if (count < 1) return set_error(PPALS_E_ARG, "count must be >= 1");
  if (max_sweeps < 1) return set_error(PPALS_E_ARG, "max_sweeps must be >= 1");
  for (int p = 0; p < count; ++p) {
    const auto& q = probs[p];
    if (q.rank < 1 || q.rank > BATCH_MAX_R)
      return set_error(PPALS_E_UNSUPPORTED, "problem " + std::to_string(p) + ": need 1 <= rank <= 64");
    for (int i = 0; i < 3; ++i)
      if (q.dims[i] < 1 || q.dims[i] > BATCH_MAX_S)
        return set_error(PPALS_E_UNSUPPORTED,
                         "problem " + std::to_string(p) + ": need 1 <= dims <= 256");
  }
  ppals_batch* b = new ppals_batch();
  b->count = count;
  b->max_sweeps = max_sweeps;
  b->probs.assign(probs, probs + count);
  for (const auto& q : b->probs) {
    b->maxR = std::max(b->maxR, (int)q.rank);
    for (int i = 0; i < 3; ++i) b->max_s = std::max(b->max_s, (int)q.dims[i]);
  }
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += al256(std::max<size_t>(bytes, 1));
    return o;
  };
  b->off_prob = take(sizeof(BProb) * count);
  b->off_state = take(sizeof(BState) * count);
  b->off_conf = take(sizeof(BConf));
  b->tiles_bytes = max_tiles_bytes(b);
  b->off_tiles = take(b->tiles_bytes);
  for (int p = 0; p < count; ++p) {
    const auto& q = b->probs[p];
    const size_t R = q.rank;
    const size_t s0 = q.dims[0], s1 = q.dims[1], s2 = q.dims[2];
    b->off_op[0].push_back(take(s0 * s1 * R * 4));
    b->off_op[1].push_back(take(s0 * s2 * R * 4));
    b->off_op[2].push_back(take(s1 * s2 * R * 4));
    for (int n = 0; n < 3; ++n) {
      b->off_Mp[n].push_back(take((size_t)q.dims[n] * R * 8));
      b->off_Ap[n].push_back(take((size_t)q.dims[n] * R * 8));
      b->off_dA[n].push_back(take((size_t)q.dims[n] * R * 8));
      b->off_Af[n].push_back(take((size_t)((q.dims[n] + 31) / 32 * 32) * BATCH_MAX_R * 4));
    }
    b->off_S.push_back(take(3 * R * R * 8));
    b->off_U.push_back(take(3 * R * R * 8));
    b->off_M.push_back(take((size_t)std::max(s0, std::max(s1, s2)) * R * 8));
    b->off_klog.push_back(take((size_t)max_sweeps));
  }
  b->ws_bytes = off;
  b->variant.resize(count);
  for (int p = 0; p < count; ++p) {
    const auto& q = b->probs[p];
    const int64_t M = (int64_t)q.dims[0] * q.dims[1];
    b->variant[p] = M >= 128 * 64 ? 1 : 0;
  }
  for (int k = 0; k < NBUCKET_R * NBUCKET_S; ++k) {
    b->bucket_variant[k] = -1;
    for (int v = 0; v < BATCH_GEMM_VARIANTS; ++v) b->bucket_ms[k][v] = -1.0;
  }
  build_tiles(b);
  *out = b;
  return PPALS_OK;
}

void ppals_batch_destroy(ppals_batch* b) {
  if (!b) return;
  drop_graph(b);
  if (b->graph_stream) (void)hipStreamDestroy(b->graph_stream);
  delete b;
}

size_t ppals_batch_workspace_bytes(const ppals_batch* b) { return b ? b->ws_bytes : 0; }

ppals_status ppals_batch_bind(ppals_batch* b, const float* const* X, double* const* A, void* ws,
                              double eps, double tol, int32_t second_order, hipStream_t s) {
  if (!b || !X || !A || !ws) return set_error(PPALS_E_ARG, "NULL argument");
  for (int p = 0; p < b->count; ++p) {
    if (!X[p]) return set_error(PPALS_E_ARG, "X[" + std::to_string(p) + "] is NULL");
    for (int n = 0; n < 3; ++n)
      if (!A[3 * p + n]) return set_error(PPALS_E_ARG, "A[" + std::to_string(3 * p + n) + "] is NULL");
  }
  if (!(tol >= 0.0)) return set_error(PPALS_E_ARG, "tol must be >= 0");
  drop_graph(b);
  char* w = (char*)ws;
  b->bound_ws = w;
  b->hprob.assign(b->count, BProb{});
  for (int p = 0; p < b->count; ++p) {
    BProb& P = b->hprob[p];
    const auto& q = b->probs[p];
    for (int i = 0; i < 3; ++i) P.s[i] = q.dims[i];
    P.R = q.rank;
    P.X = X[p];
    for (int n = 0; n < 3; ++n) {
      P.A[n] = A[3 * p + n];
      P.op[n] = (float*)(w + b->off_op[n][p]);
      P.Mp[n] = (double*)(w + b->off_Mp[n][p]);
      P.Ap[n] = (double*)(w + b->off_Ap[n][p]);
      P.dA[n] = (double*)(w + b->off_dA[n][p]);
      P.Af[n] = (float*)(w + b->off_Af[n][p]);
    }
    P.S = (double*)(w + b->off_S[p]);
    P.U = (double*)(w + b->off_U[p]);
    P.M = (double*)(w + b->off_M[p]);
    P.klog = (uint8_t*)(w + b->off_klog[p]);
  }
  b->hconf.eps = eps;
  b->hconf.tol = tol;
  b->hconf.max_sweeps = b->max_sweeps;
  b->hconf.second_order = second_order ? 1 : 0;
  BHIPCHK(hipMemcpyAsync(w + b->off_prob, b->hprob.data(), sizeof(BProb) * b->count,
                         hipMemcpyHostToDevice, s));
  BHIPCHK(hipMemcpyAsync(w + b->off_conf, &b->hconf, sizeof(BConf), hipMemcpyHostToDevice, s));
  ppals_status r = upload_tiles(b, s);
  if (r != PPALS_OK) return r;
  BHIPCHK(launch_b_norm((BProb*)(w + b->off_prob), (BState*)(w + b->off_state),
                        (const BConf*)(w + b->off_conf), b->count, s));
  BHIPCHK(batch_prepare());
  return PPALS_OK;
}

ppals_status ppals_batch_autotune(ppals_batch* b, void* ws, int32_t reps, hipStream_t s) {
  if (!b || !ws) return set_error(PPALS_E_ARG, "NULL argument");
  if ((char*)ws != b->bound_ws) return set_error(PPALS_E_STATE, "workspace not bound");
  if (reps < 1) return set_error(PPALS_E_ARG, "reps must be >= 1");
  char* w = (char*)ws;
  const BProb* pr = (const BProb*)(w + b->off_prob);
  const BState* st = (const BState*)(w + b->off_state);
  hipEvent_t e0, e1;
  BHIPCHK(hipEventCreate(&e0));
  BHIPCHK(hipEventCreate(&e1));
  std::vector<BTile> saved = b->tiles;
  std::vector<int> saved_variant = b->variant;
  for (int k = 0; k < NBUCKET_R * NBUCKET_S; ++k) {
    std::vector<int> members;
    for (int p = 0; p < b->count; ++p)
      if (bucket_of(b->probs[p]) == k) members.push_back(p);
    if (members.empty()) continue;
    double best = 1e300;
    for (int v = 0; v < BATCH_GEMM_VARIANTS; ++v) {
      // the bucket's problems with variant v, the contraction of the contiguous mode and of
      // the leading mode (the two access patterns), into the operator scratch
      for (int p = 0; p < b->count; ++p) b->variant[p] = -1;
      for (int p : members) b->variant[p] = v;
      build_tiles(b);
      ppals_status r = upload_tiles(b, s);
      if (r != PPALS_OK) return r;
      float ms = 0.f;
      for (int it = 0; it <= reps; ++it) {  // first pass warms up
        if (it == 1) BHIPCHK(hipEventRecord(e0, s));
        for (int c : {2, 0}) {
          const int out = c == 2 ? 0 : 2;
          BHIPCHK(launch_b_gemm(v, pr, st, (const BTile*)(w + b->off_tiles) + b->g_off[c][v],
                                b->g_cnt[c][v], c, out, 0xF, s));
        }
      }
      BHIPCHK(hipEventRecord(e1, s));
      BHIPCHK(hipEventSynchronize(e1));
      BHIPCHK(hipEventElapsedTime(&ms, e0, e1));
      b->bucket_ms[k][v] = ms / reps;
      if (ms < best) {
        best = ms;
        b->bucket_variant[k] = v;
      }
    }
    for (int p : members) saved_variant[p] = b->bucket_variant[k];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  b->variant = saved_variant;
  build_tiles(b);
  b->tuned = true;
  drop_graph(b);
  return upload_tiles(b, s);
}

ppals_status ppals_batch_sweep(ppals_batch* b, void* ws, hipStream_t s) {
  if (!b || !ws) return set_error(PPALS_E_ARG, "NULL argument");
  if ((char*)ws != b->bound_ws) return set_error(PPALS_E_STATE, "workspace not bound");
  return enqueue_sweep(b, (char*)ws, s);
}

ppals_status ppals_batch_run(ppals_batch* b, void* ws, int32_t sweeps, int32_t use_graph,
                             hipStream_t s) {
  if (!b || !ws) return set_error(PPALS_E_ARG, "NULL argument");
  if ((char*)ws != b->bound_ws) return set_error(PPALS_E_STATE, "workspace not bound");
  if (sweeps < 0) return set_error(PPALS_E_ARG, "sweeps < 0");
  if (!use_graph) {
    for (int i = 0; i < sweeps; ++i) {
      ppals_status r = enqueue_sweep(b, (char*)ws, s);
      if (r != PPALS_OK) return r;
    }
    return PPALS_OK;
  }
  if (!b->exec || b->graph_ws != (char*)ws) {
    drop_graph(b);
    // captured on a stream of the library's own (the caller's may be the null stream,
    // which cannot be captured); the graph is then launched on the caller's stream
    if (!b->graph_stream)
      BHIPCHK(hipStreamCreateWithFlags(&b->graph_stream, hipStreamNonBlocking));
    BHIPCHK(hipStreamBeginCapture(b->graph_stream, hipStreamCaptureModeThreadLocal));
    ppals_status r = enqueue_sweep(b, (char*)ws, b->graph_stream);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(b->graph_stream, &g);
    if (r != PPALS_OK) {
      if (g) (void)hipGraphDestroy(g);
      return r;
    }
    if (e != hipSuccess) return set_error(PPALS_E_HIP, std::string("capture: ") + hipGetErrorString(e));
    b->graph = g;
    BHIPCHK(hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0));
    b->graph_ws = (char*)ws;
  }
  for (int i = 0; i < sweeps; ++i) BHIPCHK(hipGraphLaunch(b->exec, s));
  return PPALS_OK;
}

ppals_status ppals_batch_results(ppals_batch* b, const void* ws, ppals_batch_result* out,
                                 hipStream_t s) {
  if (!b || !ws || !out) return set_error(PPALS_E_ARG, "NULL argument");
  if ((const char*)ws != b->bound_ws) return set_error(PPALS_E_STATE, "workspace not bound");
  std::vector<BState> hs(b->count);
  BHIPCHK(hipMemcpyAsync(hs.data(), (const char*)ws + b->off_state, sizeof(BState) * b->count,
                         hipMemcpyDeviceToHost, s));
  BHIPCHK(hipStreamSynchronize(s));
  int dev = 0, khz = 0;
  BHIPCHK(hipGetDevice(&dev));
  BHIPCHK(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
  for (int p = 0; p < b->count; ++p) {
    const BState& S = hs[p];
    ppals_batch_result& r = out[p];
    memset(&r, 0, sizeof(r));
    r.sweeps = S.sweep;
    r.converged_sweep = S.conv_sweep;
    r.n_als = S.n_als;
    r.n_pp_init = S.n_init;
    r.n_pp_approx = S.n_approx;
    r.done = S.done;
    r.fit = S.fit;
    r.normX2 = S.normX2;
    for (int n = 0; n < 3; ++n) {
      r.rel_change[n] = S.rel[n];
      r.chol_status[n] = S.chol[n];
    }
    r.time_to_converge_ms =
        (S.conv_sweep > 0 && khz > 0) ? (double)(S.t_conv - S.t_start) / (double)khz : -1.0;
  }
  return PPALS_OK;
}

ppals_status ppals_batch_kind_log(ppals_batch* b, const void* ws, uint8_t* out, hipStream_t s) {
  if (!b || !ws || !out) return set_error(PPALS_E_ARG, "NULL argument");
  if ((const char*)ws != b->bound_ws) return set_error(PPALS_E_STATE, "workspace not bound");
  for (int p = 0; p < b->count; ++p)
    BHIPCHK(hipMemcpyAsync(out + (size_t)p * b->max_sweeps, (const char*)ws + b->off_klog[p],
                           b->max_sweeps, hipMemcpyDeviceToHost, s));
  BHIPCHK(hipStreamSynchronize(s));
  return PPALS_OK;
}

ppals_status ppals_batch_describe(const ppals_batch* b, char* buf, size_t len) {
  if (!b || !buf || len == 0) return set_error(PPALS_E_ARG, "NULL argument");
  std::string j = "{\"count\":" + std::to_string(b->count) + ",\"max_rank\":" +
                  std::to_string(b->maxR) + ",\"max_dim\":" + std::to_string(b->max_s) +
                  ",\"workspace_bytes\":" + std::to_string(b->ws_bytes) +
                  ",\"tuned\":" + (b->tuned ? "true" : "false") + ",\"buckets\":[";
  bool first = true;
  char tmp[256];
  for (int k = 0; k < NBUCKET_R * NBUCKET_S; ++k) {
    int members = 0;
    for (const auto& q : b->probs) members += bucket_of(q) == k;
    if (!members) continue;
    snprintf(tmp, sizeof(tmp),
             "%s{\"rank_max\":%d,\"dim_max\":%d,\"problems\":%d,\"tile_rows\":%d,"
             "\"ms_64\":%.6f,\"ms_128\":%.6f}",
             first ? "" : ",", 16 * (k / NBUCKET_S + 1), (k % NBUCKET_S == 0) ? 64 : (k % NBUCKET_S == 1 ? 128 : 256),
             members, b->bucket_variant[k] < 0 ? -1 : batch_gemm_rows(b->bucket_variant[k]),
             b->bucket_ms[k][0], b->bucket_ms[k][1]);
    j += tmp;
    first = false;
  }
  j += "]}";
  if (j.size() + 1 > len) return set_error(PPALS_E_ARG, "buffer too small");
  memcpy(buf, j.c_str(), j.size() + 1);
  return PPALS_OK;
}

}  // extern "C"
