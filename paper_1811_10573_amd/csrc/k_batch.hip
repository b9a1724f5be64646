// Batched PP-CP-ALS kernels for many independent order-3 problems of uneven size
// and rank (s_n <= 256, R <= 64), FP32 tensors, FP64 factors and small dense work.
//
// One batched sweep is a fixed sequence of grouped launches.  Each problem carries a
// device-side state machine (BState): at the start of a sweep it picks ALS,
// PP initialisation or PP-approximated for itself with the threshold rule of
// Algorithm 3, or nothing once it has converged, and every grouped kernel skips the
// problems whose current kind it does not serve.  No launch depends on a host
// decision, so a sweep can be captured once in a HIP graph and replayed.
//
// Per sweep, for every problem (N = 3, Section 2.5 dimension tree, Section 3.2.1 PP):
//   ALS:        I01 = X x_2 A^(2); M^(0) = I01 x_1 A^(1); M^(1) = I01 x_0 A^(0);
//               I12 = X x_0 A^(0); M^(2) = I12 x_1 A^(1)  (with the updated factors)
//   PP build:   M^(0,1) = X x_2 A, M^(0,2) = X x_1 A, M^(1,2) = X x_0 A and M_p^(n)
//   PP sweep:   M~^(n) = M_p^(n) + sum_{i != n} M^(i,n) x_i dA^(i) + A^(n) W^(n),
//               W^(n) = U^(i) * U^(j) for the two other modes i, j
// followed by the FP64 solve A^(n) = M Gamma^-1 (Cholesky), Grams and norms.
#include "batch.h"
#include "common.h"
#include "tail_dev.h"

namespace ppk {

// The per-problem pointers live in BProb records in device memory, so the compiler cannot
// tell their address space and would access them with flat instructions, whose completion
// is counted together with LDS operations (every wait for an LDS read would then also wait
// for all outstanding global loads).  They all point to global memory: gl() says so.
#define GLB __attribute__((address_space(1)))
template <typename T> __device__ __forceinline__ GLB T* gl(T* p) { return (GLB T*)p; }
template <typename T> __device__ __forceinline__ const GLB T* gl(const T* p) { return (const GLB T*)p; }
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));  // 4-byte aligned 16-byte vector

// ---------------------------------------------------------------------------
// State machine
// ---------------------------------------------------------------------------
__global__ void k_b_begin(BState* st, BProb* pr, const BConf* conf, int count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  BState& S = st[p];
  if (S.sweep == 0 && !S.done) S.t_start = wall_clock64();
  if (S.done) {
    S.kind = BK_NONE;
    return;
  }
  if (S.sweep >= conf->max_sweeps) {
    S.done = 1;
    S.kind = BK_NONE;
    return;
  }
  bool small = conf->eps > 0.0;
  for (int n = 0; n < 3; ++n) small = small && S.rel[n] < conf->eps;
  int kind = BK_ALS;
  if (small) kind = (S.prev_kind == BK_PP_INIT || S.prev_kind == BK_PP_APPROX) ? BK_PP_APPROX
                                                                              : BK_PP_INIT;
  S.kind = kind;
  gl(pr[p].klog)[S.sweep] = (uint8_t)kind;
}

// PP initialisation of the problems that start a PP phase: A_p := A, dA := 0, U := 0.
__global__ __launch_bounds__(256) void k_b_prep(const BProb* pr, const BState* st, int count) {
  const int p = blockIdx.x;
  if (p >= count || st[p].kind != BK_PP_INIT) return;
  const BProb& P = pr[p];
  const int R = P.R;
  for (int n = 0; n < 3; ++n) {
    const int64_t cnt = (int64_t)P.s[n] * R;
    for (int64_t e = threadIdx.x; e < cnt; e += blockDim.x) {
      gl(P.Ap[n])[e] = gl(P.A[n])[e];
      gl(P.dA[n])[e] = 0.0;
    }
  }
  for (int e = threadIdx.x; e < 3 * R * R; e += blockDim.x) gl(P.U)[e] = 0.0;
}

// ---------------------------------------------------------------------------
// Grouped first-level contraction: out[m][r] = sum_k X(m, k) A^(c)[k][r], FP32 on the
// matrix cores (f32 16x16x4: lane l supplies A[m0 + l%16][k_g] and B[k_g][c0 + l%16] for
// the k-index g = l/16 of the step; accumulator register v holds row 4 (l/16) + v, column
// l%16).  The order in which k enters the sum is free as long as both operands follow
// it: step s of a 16-deep k block gives group g the k-value 4 g + s, so each lane reads
// four consecutive k of its row (and of its factor column) with one 16-byte LDS read and
// feeds them to four steps.
// With P = prod s_{<c}, Q = prod s_{>c}: X(m, k) = X[p K Q + k Q + q], m = p Q + q.
// TM output rows per tile, 4 waves of TM/4 rows each, R padded to 16-column tiles.
// A work item is a run of consecutive tiles of one problem (BATCH_RUN_ROWS rows), walked
// as one sequence of (tile, k-chunk) steps: the next step's X and factor entries are
// loaded into registers while the current step is multiplied, also across tile
// boundaries, so the problem's descriptors and the first chunk's load latency are paid
// once per run.  Chunks of BKC k-values pass through double-buffered LDS, X as [m][k]
// and the factor as [c][k], from the factor's transposed FP32 copy (64 columns of
// BKC-padded length, zero-filled), which a chunk reads with two unconditional 16-byte
// loads per thread.
// ---------------------------------------------------------------------------
constexpr int BKC = 32;  // k per LDS chunk
template <int V> struct IC { static constexpr int value = V; };  // compile-time index

// LDS position (in floats) of the k-quad kq of row r in a chunk of 32-float rows.  Rows
// are not padded; the quad index is XOR-ed with (r / 2) mod 8, so the 16 rows of one
// 16-byte read (one per lane of a 16-lane group) and the rows of a 16-lane store land on
// distinct banks.
__device__ __forceinline__ int swz_q(int r, int kq) { return r * BKC + 4 * (kq ^ ((r >> 1) & 7)); }

template <int TM, bool KCM>
__global__ __launch_bounds__(256) void k_b_gemm(const BProb* pr, const BState* st,
                                                const BTile* tiles, int ntiles, int cmode,
                                                int out_op, int kind_mask) {
  static_assert(BATCH_RUN_ROWS % TM == 0, "a run holds whole tiles");
  static_assert(BKC == 32 && BATCH_MAX_R == 64, "layout assumes 32-deep chunks of 64 columns");
  constexpr int RS = TM / 64;                        // 16-row subtiles per wave
  constexpr int XQ = BKC * TM / 4 / 256;             // X k-quads staged per thread
  constexpr int AV4 = BKC * BATCH_MAX_R / 4 / 256;   // factor 16-byte vectors per thread
  __shared__ __attribute__((aligned(16))) float xs[2][TM * BKC];
  __shared__ __attribute__((aligned(16))) float as[2][BATCH_MAX_R * BKC];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, g = l >> 4;
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BTile tile = tiles[t];
    const int p = tile.prob;
    if (!(kind_mask & (1 << st[p].kind))) continue;
    const BProb& P = pr[p];
    const int R = P.R;
    int Pd = 1, Qi = 1;
    for (int i = 0; i < cmode; ++i) Pd *= P.s[i];
    for (int i = cmode + 1; i < 3; ++i) Qi *= P.s[i];
    // 32-bit element offsets (a problem holds at most 256^3 elements)
    const int Ki = P.s[cmode], Mi = Pd * Qi;
    const int Kpad = (Ki + BKC - 1) / BKC * BKC;
    const int mend = min(Mi, tile.m0 + BATCH_RUN_ROWS);
    const GLB float* X = gl(P.X);
    const GLB float* Af = gl(P.Af[cmode]);
    GLB float* out = gl(P.op[out_op]);
    const int NCT = (R + 15) >> 4;
    // X staging.
    //   Q == 1 (rows k-contiguous): quad u of this thread is row m0 + tid/8 + 32 u,
    //   k-quad tid%8; 8 lanes read one row's 32 consecutive k with 16-byte loads (4-byte
    //   aligned addresses suffice).  A quad that crosses the row's end is read element by
    //   element.
    //   otherwise (rows contiguous for a fixed k): this thread reads row m0 + tid%TM at
    //   the k of quads tid/TM + (256/TM) u, consecutive lanes reading consecutive rows.
    constexpr bool kcm = KCM;  // Q == 1 exactly when the last mode is contracted
    constexpr int QSTEP = 256 / TM;
    f4 xr[2][XQ], ar[2][AV4];  // two register sets: steps i + 1 and i + 2
    auto xm = [&](int u) { return kcm ? tid / 8 + 32 * u : tid % TM; };
    auto xq = [&](int u) { return kcm ? tid % 8 : tid / TM + QSTEP * u; };
    int xbase = 0;
    bool rowv = true;
    auto set_rows = [&](int m0) {
      if (!kcm) {
        const int m = m0 + tid % TM;
        rowv = m < Mi;
        const int pp = rowv ? m / Qi : 0, q = rowv ? m - pp * Qi : 0;
        xbase = pp * Ki * Qi + q;
      }
    };
    auto load_chunk = [&](auto set, int m0, int k0) {
      constexpr int S = decltype(set)::value;
#pragma unroll
      for (int u = 0; u < XQ; ++u) {
        const int kb = k0 + 4 * xq(u);
        f4 v = f4{0.f, 0.f, 0.f, 0.f};
        if (kcm) {
          const int m = m0 + xm(u);
          if (m < Mi) {
            const GLB float* src = X + m * Ki + kb;
            if (kb + 3 < Ki) {
              const f4u w4 = *reinterpret_cast<const GLB f4u*>(src);
              v = f4{w4.x, w4.y, w4.z, w4.w};
            } else {
              if (kb < Ki) v.x = src[0];
              if (kb + 1 < Ki) v.y = src[1];
              if (kb + 2 < Ki) v.z = src[2];
            }
          }
        } else if (rowv) {
          const GLB float* src = X + xbase + kb * Qi;
          if (kb < Ki) v.x = src[0];
          if (kb + 1 < Ki) v.y = src[Qi];
          if (kb + 2 < Ki) v.z = src[2 * Qi];
          if (kb + 3 < Ki) v.w = src[3 * Qi];
        }
        xr[S][u] = v;
      }
#pragma unroll
      for (int j = 0; j < AV4; ++j) {
        const int vi = tid + 256 * j, c = vi / 8, q = vi % 8;
        ar[S][j] = *reinterpret_cast<const GLB f4*>(Af + c * Kpad + k0 + 4 * q);
      }
    };
    auto store_chunk = [&](auto set, int buf) {
      constexpr int S = decltype(set)::value;
#pragma unroll
      for (int u = 0; u < XQ; ++u) *reinterpret_cast<f4*>(&xs[buf][swz_q(xm(u), xq(u))]) = xr[S][u];
#pragma unroll
      for (int j = 0; j < AV4; ++j) {
        const int vi = tid + 256 * j, c = vi / 8, q = vi % 8;
        *reinterpret_cast<f4*>(&as[buf][swz_q(c, q)]) = ar[S][j];
      }
    };
    f4 acc[RS][4];
#pragma unroll
    for (int i = 0; i < RS; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    // Step being multiplied (cm0, ck0, in LDS buffer buf), the next step (nm0, nk0, in a
    // register set while nv) and the step being loaded (lm0, lk0).
    int cm0 = tile.m0, ck0 = 0, nm0 = 0, nk0 = 0, lm0 = tile.m0, lk0 = 0;
    bool nv = false;
    auto advance = [&]() {
      lk0 += BKC;
      if (lk0 >= Ki) {
        lk0 = 0;
        lm0 += TM;
        set_rows(lm0);
      }
    };
    __syncthreads();  // the previous run's last chunk is no longer read
    set_rows(lm0);
    load_chunk(IC<0>{}, lm0, lk0);
    advance();
    if (lm0 < mend) {
      nv = true;
      nm0 = lm0;
      nk0 = lk0;
      load_chunk(IC<1>{}, lm0, lk0);
      advance();
    }
    store_chunk(IC<0>{}, 0);
    __syncthreads();
    int buf = 0;
    // One step with the next step's data in register set N; loads the step after it into
    // the other set.  Returns false after the run's last step.
    auto step = [&](auto nset) -> bool {
      constexpr int N = decltype(nset)::value;
      const bool ld = nv && lm0 < mend;
      if (ld) load_chunk(IC<1 - N>{}, lm0, lk0);
#pragma unroll
      for (int kb = 0; kb < BKC / 16; ++kb) {  // 16-deep k blocks: quad 4 kb + g per lane
        f4 a[RS], b[4];
#pragma unroll
        for (int i = 0; i < RS; ++i)
          a[i] = *reinterpret_cast<const f4*>(&xs[buf][swz_q(w * (TM / 4) + i * 16 + (l & 15), 4 * kb + g)]);
#pragma unroll
        for (int j = 0; j < 4; ++j)
          if (j < NCT) b[j] = *reinterpret_cast<const f4*>(&as[buf][swz_q(j * 16 + (l & 15), 4 * kb + g)]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (j < NCT) {
#pragma unroll
              for (int i = 0; i < RS; ++i)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i][s], b[j][s], acc[i][j], 0, 0, 0);
            }
      }
      if (ck0 + BKC >= Ki) {  // last chunk of the tile at cm0: write it out, restart
#pragma unroll
        for (int i = 0; i < RS; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (j >= NCT) continue;
            const int c = j * 16 + (l & 15);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int m = cm0 + w * (TM / 4) + i * 16 + 4 * g + v;
              if (m < Mi && c < R) out[(int64_t)m * R + c] = acc[i][j][v];
            }
            acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
          }
      }
      if (nv) store_chunk(IC<N>{}, buf ^ 1);
      __syncthreads();
      if (!nv) return false;
      buf ^= 1;
      cm0 = nm0;
      ck0 = nk0;
      if (ld) {
        nm0 = lm0;
        nk0 = lk0;
        advance();
      } else {
        nv = false;
      }
      return true;
    };
    while (step(IC<1>{}) && step(IC<0>{})) {
    }
  }
}

// ---------------------------------------------------------------------------
// Grouped multi-TTV: out[y][r] = base[y][r] + sum_jobs sum_x T[p][x][q][r] F[x][r],
// y = p Q + q, FP64 accumulation, one output element per thread.  A workgroup's 256
// elements belong to one problem and share F: it passes through LDS BTTV_XC rows at a
// time (double-buffered, one barrier per chunk), so each F entry is read from global
// memory once per workgroup instead of once per output row.  The chunk's T values are
// requested before the chunk's F rows are stored, so both loads overlap.
// ---------------------------------------------------------------------------
constexpr int BTTV_XC = 32;  // x per chunk

struct BJob {
  const float* T;
  const double* F;
  int P, X, Q;
};

__global__ __launch_bounds__(256) void k_b_ttv(const BProb* pr, const BState* st, const BTile* tiles,
                                               int ntiles, int n, int build_mp) {
  __shared__ double fsh[2 * BTTV_XC * BATCH_MAX_R];
  for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const BTile tile = tiles[t];
    const int p = tile.prob;
    const int kind = st[p].kind;
    if (build_mp ? kind != BK_PP_INIT : kind == BK_NONE) continue;
    const BProb& P = pr[p];
    const int R = P.R;
    const int s0 = P.s[0], s1 = P.s[1], s2 = P.s[2];
    const int ne = P.s[n] * R;
    const int e = tile.m0 + threadIdx.x;
    const bool act = e < ne;
    const int ec = act ? e : ne - 1;
    const int y = ec / R, r = ec - y * R;
    BJob J[2];
    int nj = 0;
    const double* base = nullptr;
    double* out = P.M;
    if (build_mp || kind == BK_ALS) {
      const double* const* F = P.A;
      if (build_mp) out = P.Mp[n];
      if (n == 0) J[nj++] = BJob{P.op[0], F[1], s0, s1, 1};
      else if (n == 1) J[nj++] = BJob{P.op[0], F[0], 1, s0, s1};
      else if (build_mp) J[nj++] = BJob{P.op[1], F[0], 1, s0, s2};
      else J[nj++] = BJob{P.op[2], F[1], 1, s1, s2};
    } else {
      base = P.Mp[n];
      if (n == 0) {
        J[nj++] = BJob{P.op[0], P.dA[1], s0, s1, 1};
        J[nj++] = BJob{P.op[1], P.dA[2], s0, s2, 1};
      } else if (n == 1) {
        J[nj++] = BJob{P.op[0], P.dA[0], 1, s0, s1};
        J[nj++] = BJob{P.op[2], P.dA[2], s1, s2, 1};
      } else {
        J[nj++] = BJob{P.op[1], P.dA[0], 1, s0, s2};
        J[nj++] = BJob{P.op[2], P.dA[1], 1, s1, s2};
      }
    }
    double acc0 = 0.0, acc1 = 0.0;
    int buf = 0;
    __syncthreads();  // the previous tile's last chunk is no longer read
    for (int j = 0; j < nj; ++j) {
      const int X = J[j].X, QR = J[j].Q * R;
      const int pp = y / J[j].Q, q = y - pp * J[j].Q;
      const GLB float* T = gl(J[j].T) + ((int64_t)pp * X * QR + (int64_t)q * R + r);
      const GLB double* F = gl(J[j].F);
      for (int x0 = 0; x0 < X; x0 += BTTV_XC) {
        const int xn = min(BTTV_XC, X - x0), cnt = xn * R;
        double* fl = fsh + buf * (BTTV_XC * BATCH_MAX_R);
        double fr[BTTV_XC * BATCH_MAX_R / 256];
#pragma unroll
        for (int i = 0; i < BTTV_XC * BATCH_MAX_R / 256; ++i) {
          const int idx = (int)threadIdx.x + 256 * i;
          fr[i] = F[(int64_t)x0 * R + min(idx, cnt - 1)];
        }
        float tv[BTTV_XC];
#pragma unroll
        for (int xx = 0; xx < BTTV_XC; ++xx) tv[xx] = T[(int64_t)(x0 + min(xx, xn - 1)) * QR];
#pragma unroll
        for (int i = 0; i < BTTV_XC * BATCH_MAX_R / 256; ++i) {
          const int idx = (int)threadIdx.x + 256 * i;
          if (idx < cnt) fl[idx] = fr[i];
        }
        __syncthreads();
#pragma unroll
        for (int xx = 0; xx < BTTV_XC; xx += 2) {
          const double f0 = fl[min(xx, xn - 1) * R + r], f1 = fl[min(xx + 1, xn - 1) * R + r];
          acc0 = fma(xx < xn ? (double)tv[xx] : 0.0, f0, acc0);
          acc1 = fma(xx + 1 < xn ? (double)tv[xx + 1] : 0.0, f1, acc1);
        }
        buf ^= 1;
      }
    }
    if (act) gl(out)[e] = (base ? gl(base)[e] : 0.0) + (acc0 + acc1);
  }
}

// ---------------------------------------------------------------------------
// Per-problem solve of mode n (one workgroup of BSOLVE_WAVES waves per problem):
// Gamma = S^(i) * S^(j), W = U^(i) * U^(j) (PP), the one-wave Cholesky of the rank <= 64
// tail (matrix-core panel updates) with one diagonal-shift retry, the unit-triangular
// factors L D^-1 and D^-1 L, the rows of A^(n) = M Gamma^-1 (plus A^(n) W in the PP
// right-hand side; BSOLVE_RPW rows per wave at a time, their substitution chains
// interleaved), dA, norms, and the Grams S^(n) = A^T A and U^(n) = A^T dA on the matrix
// cores, BSOLVE_CH rows at a time.
// ---------------------------------------------------------------------------
constexpr int BSOLVE_WAVES = 8;
constexpr int BSOLVE_CH = 32;
constexpr int BSOLVE_RPW = BSOLVE_CH / BSOLVE_WAVES;  // rows per wave per chunk
constexpr int BSOLVE_TPW = 4;                         // Gram tiles per wave (<= 32 tiles)

__global__ __launch_bounds__(BSOLVE_WAVES * 64) void k_b_solve(const BProb* pr, BState* st,
                                                               const BConf* conf, int n) {
  constexpr int UB = 8;  // steps whose LDS operands are read together
  extern __shared__ double sm[];
  __shared__ double red[BSOLVE_WAVES][4];
  __shared__ double cb[128];
  __shared__ int status;
  const int p = blockIdx.x;
  const int kind = st[p].kind;
  if (kind == BK_NONE) return;
  const BProb& P = pr[p];
  const int R = P.R, RR = R * R;
  const int rows = P.s[n];
  const bool pp = kind != BK_ALS;
  const bool wterm = pp && conf->second_order;
  const int i1 = n == 0 ? 1 : 0, i2 = n == 2 ? 1 : 2;  // the two other modes
  double* Lm = sm;                          // 64 x 65: Gamma, then L, then D^-1 L
  double* LF = Lm + 64 * CH64_LS;           // R x R: LF[j][k] = L[k][j] / L[j][j] (k > j)
  double* Ws = LF + RR;                     // R x R
  double* invd = Ws + RR;                   // 64
  double* ca = invd + 64;                   // BSOLVE_CH x R: new rows
  double* cd = ca + BSOLVE_CH * R;          // BSOLVE_CH x R: dA rows
  double* bv = cd + BSOLVE_CH * R;          // BSOLVE_WAVES x BSOLVE_RPW x 64 broadcast rows
  const int tid = threadIdx.x, nthr = blockDim.x, w = tid >> 6, l = tid & 63;
  const bool lv = l < R;
  const int lc = lv ? l : 0;
  const GLB double* S = gl(P.S);
  const GLB double* U = gl(P.U);
  // Gamma = S^(i1) * S^(i2) into the zero-padded 64 x 65 array and W = U^(i1) * U^(i2): all
  // loads unconditional (clamped) and issued before the first wait
  constexpr int NT = BSOLVE_WAVES * 64;
  constexpr int GE = (64 * CH64_LS + NT - 1) / NT, WE = (64 * 64 + NT - 1) / NT;
  double g1[GE], g2[GE], u1[WE], u2[WE];
#pragma unroll
  for (int j = 0; j < GE; ++j) {
    const int e = tid + j * NT, r = e / CH64_LS, c = e - r * CH64_LS;
    const int idx = (e < 64 * CH64_LS && r < R && c < R) ? r * R + c : 0;
    g1[j] = S[i1 * RR + idx];
    g2[j] = S[i2 * RR + idx];
  }
#pragma unroll
  for (int j = 0; j < WE; ++j) {
    const int e = tid + j * NT, idx = e < RR ? e : 0;
    u1[j] = U[i1 * RR + idx];
    u2[j] = U[i2 * RR + idx];
  }
  double dmax = 0.0;
#pragma unroll
  for (int j = 0; j < GE; ++j) {
    const int e = tid + j * NT, r = e / CH64_LS, c = e - r * CH64_LS;
    if (e < 64 * CH64_LS) {
      const double g = (r < R && c < R) ? g1[j] * g2[j] : 0.0;
      if (r == c && r < R) dmax = fmax(dmax, g);
      Lm[e] = g;
    }
  }
#pragma unroll
  for (int j = 0; j < WE; ++j) {
    const int e = tid + j * NT;
    if (e < RR) Ws[e] = wterm ? u1[j] * u2[j] : 0.0;
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if (l == 0) red[w][0] = dmax;
  __syncthreads();
  if (w == 0) {
    int stv = 0;
    for (int attempt = 0;; ++attempt) {
      if (chol_wave64(Lm, cb, R) < 0) break;
      if (attempt == 1) {
        stv = 2;
        break;
      }
      double mx = 0.0;
      for (int q = 0; q < BSOLVE_WAVES; ++q) mx = fmax(mx, red[q][0]);
      const double delta = (double)R * 0x1p-52 * mx;
      for (int e = l; e < 64 * CH64_LS; e += 64) {
        const int r = e / CH64_LS, c = e - r * CH64_LS;
        Lm[e] = (r < R && c < R) ? S[i1 * RR + r * R + c] * S[i2 * RR + r * R + c] + (r == c ? delta : 0.0)
                                 : 0.0;
      }
      stv = 1;
    }
    if (l == 0) status = stv;
    if (l < R) invd[l] = 1.0 / Lm[l * CH64_LS + l];
  }
  __syncthreads();
  const int stv = status;
  // unit factors: LF from L, then D^-1 L in place (strictly lower, zero elsewhere)
  for (int e = tid; e < RR; e += nthr) {
    const int i = e / R, k = e - i * R;
    LF[k * R + i] = i > k ? Lm[i * CH64_LS + k] * invd[k] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < RR; e += nthr) {
    const int i = e / R, k = e - i * R;
    Lm[i * CH64_LS + k] = k < i ? Lm[i * CH64_LS + k] * invd[i] : 0.0;
  }
  __syncthreads();
  // Gram tiles owned by this wave: tt = w + BSOLVE_WAVES * t over NBR^2 S tiles then
  // NBR^2 U tiles
  const int NBR = (R + 15) >> 4;
  const int ntile = NBR * NBR * (pp ? 2 : 1);
  d4 gacc[BSOLVE_TPW];
#pragma unroll
  for (int t = 0; t < BSOLVE_TPW; ++t) gacc[t] = d4{0.0, 0.0, 0.0, 0.0};
  double nd = 0.0, na = 0.0, nm = 0.0;
  GLB double* An = gl(P.A[n]);
  const GLB double* M = gl(P.M);
  const GLB double* Apn = gl(P.Ap[n]);
  GLB double* dAn = gl(P.dA[n]);
  double* bw = bv + w * BSOLVE_RPW * 64;
  const double dl = lv ? invd[lc] : 0.0;
  for (int c0 = 0; c0 < rows; c0 += BSOLVE_CH) {
    double m[BSOLVE_RPW], ao[BSOLVE_RPW], x[BSOLVE_RPW], ap[BSOLVE_RPW];
    bool rv[BSOLVE_RPW];
    // the chunk's row operands in one round trip (unconditional, clamped, masked): M~,
    // A_old and, in PP sweeps, A_p
    const GLB double* Aref = pp ? Apn : An;
#pragma unroll
    for (int q = 0; q < BSOLVE_RPW; ++q) {
      const int y = c0 + w * BSOLVE_RPW + q;
      rv[q] = y < rows;
      const int64_t off = (int64_t)(rv[q] ? y : rows - 1) * R + lc;
      const bool ok = rv[q] && lv;
      const double mv = M[off], av = An[off], pv = Aref[off];
      m[q] = ok ? mv : 0.0;
      ao[q] = ok ? av : 0.0;
      ap[q] = pv;
    }
    if (wterm) {  // M~ += A_old W, A_old rows read back as broadcasts
#pragma unroll
      for (int q = 0; q < BSOLVE_RPW; ++q) bw[q * 64 + l] = ao[q];
      __builtin_amdgcn_wave_barrier();
      for (int j0 = 0; j0 < R; j0 += UB) {
        double wv[UB], av[BSOLVE_RPW][UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          const int j = min(j0 + u, R - 1);
          wv[u] = Ws[j * R + lc];
#pragma unroll
          for (int q = 0; q < BSOLVE_RPW; ++q) av[q][u] = j0 + u < R ? bw[q * 64 + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < UB; ++u)
#pragma unroll
          for (int q = 0; q < BSOLVE_RPW; ++q) m[q] = fma(av[q][u], wv[u], m[q]);
      }
      __builtin_amdgcn_wave_barrier();
    }
    double mo[BSOLVE_RPW];
#pragma unroll
    for (int q = 0; q < BSOLVE_RPW; ++q) mo[q] = m[q];
    if (stv != 2) {
      for (int j0 = 0; j0 < R; j0 += UB) {            // (L D^-1) y = M~
        double lf[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) lf[u] = LF[min(j0 + u, R - 1) * R + lc];
#pragma unroll
        for (int u = 0; u < UB; ++u)
          if (j0 + u < R) {
#pragma unroll
            for (int q = 0; q < BSOLVE_RPW; ++q) m[q] = fma(-lf[u], bcast(m[q], j0 + u), m[q]);
          }
      }
#pragma unroll
      for (int q = 0; q < BSOLVE_RPW; ++q) m[q] *= dl;
      for (int j1 = R - 1; j1 >= 0; j1 -= UB) {       // (D^-1 L)^T v = D^-1 y, descending
        double lb[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) lb[u] = Lm[max(j1 - u, 0) * CH64_LS + lc];
#pragma unroll
        for (int u = 0; u < UB; ++u)
          if (j1 - u >= 0) {
#pragma unroll
            for (int q = 0; q < BSOLVE_RPW; ++q) m[q] = fma(-lb[u], bcast(m[q], j1 - u), m[q]);
          }
      }
#pragma unroll
      for (int q = 0; q < BSOLVE_RPW; ++q) x[q] = lv ? m[q] * dl : 0.0;
    } else {
#pragma unroll
      for (int q = 0; q < BSOLVE_RPW; ++q) x[q] = ao[q];
    }
#pragma unroll
    for (int q = 0; q < BSOLVE_RPW; ++q) {
      const int y = c0 + w * BSOLVE_RPW + q;
      const int yl = y - c0;
      double d = 0.0;
      if (rv[q] && lv) {
        d = x[q] - ap[q];  // A_p in PP sweeps, A_old otherwise
        An[(int64_t)y * R + l] = x[q];
        if (pp) dAn[(int64_t)y * R + l] = d;
        nd = fma(d, d, nd);
        na = fma(x[q], x[q], na);
        nm = fma(mo[q], x[q], nm);
      }
      if (lv) {
        ca[yl * R + l] = (rv[q] ? x[q] : 0.0);
        cd[yl * R + l] = (rv[q] ? d : 0.0);
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < BSOLVE_TPW; ++t) {
      const int tt = w + BSOLVE_WAVES * t;
      if (tt < ntile) {
        const bool isU = tt >= NBR * NBR;
        const int tl = isU ? tt - NBR * NBR : tt;
        const int r0 = (tl / NBR) * 16, cc0 = (tl % NBR) * 16;
        const double* Bm = isU ? cd : ca;
        const int ra = r0 + (l & 15), cbx = cc0 + (l & 15);
        for (int kk = 0; kk < BSOLVE_CH; kk += 4) {
          const int k = kk + (l >> 4);
          const double a = ra < R ? ca[k * R + ra] : 0.0;
          const double b = cbx < R ? Bm[k * R + cbx] : 0.0;
          gacc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, gacc[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // both output pointers read together, outside the branches (a record field read under
  // a branch costs a round trip each)
  GLB double* const Sout = gl(P.S) + (size_t)n * RR;
  GLB double* const Uout = gl(P.U) + (size_t)n * RR;
#pragma unroll
  for (int t = 0; t < BSOLVE_TPW; ++t) {
    const int tt = w + BSOLVE_WAVES * t;
    if (tt < ntile) {
      const bool isU = tt >= NBR * NBR;
      const int tl = isU ? tt - NBR * NBR : tt;
      const int r0 = (tl / NBR) * 16, cc0 = (tl % NBR) * 16;
      GLB double* out = isU ? Uout : Sout;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + 4 * v + (l >> 4), c = cc0 + (l & 15);
        if (r < R && c < R) out[r * R + c] = gacc[t][v];
      }
    }
  }
  nd = wsum(nd);
  na = wsum(na);
  nm = wsum(nm);
  if (l == 0) {
    red[w][1] = nd;
    red[w][2] = na;
    red[w][3] = nm;
  }
  __syncthreads();
  if (tid == 0) {
    BState& B = st[p];
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int q = 0; q < BSOLVE_WAVES; ++q) {
      s1 += red[q][1];
      s2 += red[q][2];
      s3 += red[q][3];
    }
    B.sums[n][0] = s1;
    B.sums[n][1] = s2;
    B.sums[n][2] = s3;
    B.chol[n] = stv;
  }
  if (n == 2) {
    // sum of Gamma^(2) * S^(2) with the new Gram (written above by this workgroup)
    __syncthreads();
    double g = 0.0;
    for (int e = tid; e < RR; e += nthr) g = fma(S[e] * S[RR + e], S[2 * RR + e], g);
    g = wsum(g);
    if (l == 0) red[w][0] = g;
    __syncthreads();
    if (tid == 0) {
      double gs = 0.0;
      for (int q = 0; q < BSOLVE_WAVES; ++q) gs += red[q][0];
      st[p].gs = gs;
    }
  }
}

// End of a sweep: relative changes, fit, convergence.
__global__ void k_b_end(BState* st, const BConf* conf, int count) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  BState& S = st[p];
  if (S.kind == BK_NONE) return;
  for (int n = 0; n < 3; ++n) {
    const double d2 = S.sums[n][0], a2 = S.sums[n][1];
    S.rel[n] = a2 > 0.0 ? sqrt(d2) / sqrt(a2) : (d2 > 0.0 ? INFINITY : 0.0);
  }
  const double r2 = S.normX2 - 2.0 * S.sums[2][2] + S.gs;
  S.fit = 1.0 - sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(S.normX2);
  if (S.kind == BK_ALS) S.n_als++;
  else if (S.kind == BK_PP_INIT) S.n_init++;
  else S.n_approx++;
  const bool conv = S.sweep >= 1 && fabs(S.fit - S.fit_prev) < conf->tol;
  S.fit_prev = S.fit;
  S.prev_kind = S.kind;
  S.sweep++;
  if (conv) {
    S.done = 1;
    S.conv_sweep = S.sweep;
    S.t_conv = wall_clock64();
  }
}

// FP32 copies of the factors of the modes in mode_mask, for the problems that swept.
__global__ __launch_bounds__(256) void k_b_f32(const BProb* pr, const BState* st, int count,
                                               int mode_mask) {
  const int p = blockIdx.x;
  if (p >= count || st[p].kind == BK_NONE) return;
  const BProb& P = pr[p];
  const int R = P.R;
  for (int n = 0; n < 3; ++n) {
    if (!(mode_mask & (1 << n))) continue;
    const int sn = P.s[n], Kpad = (sn + BKC - 1) / BKC * BKC;
    for (int e = threadIdx.x; e < R * sn; e += 256) {  // columns >= R and rows >= s_n stay 0
      const int c = e / sn, y = e - c * sn;
      gl(P.Af[n])[c * Kpad + y] = (float)gl(P.A[n])[y * R + c];
    }
  }
}

// Initialisation: ||X||^2, the Grams of the initial factors, their FP32 copies, a fresh
// state and an empty sweep-kind log.
__global__ __launch_bounds__(256) void k_b_norm(const BProb* pr, BState* st, const BConf* conf,
                                                int count) {
  __shared__ double red[4];
  const int p = blockIdx.x;
  if (p >= count) return;
  const BProb& P = pr[p];
  for (int k = threadIdx.x; k < conf->max_sweeps; k += 256) gl(P.klog)[k] = 0;
  const int64_t total = (int64_t)P.s[0] * P.s[1] * P.s[2];
  double a = 0.0;
  for (int64_t e = threadIdx.x; e < total; e += 256) {
    const double v = gl(P.X)[e];
    a = fma(v, v, a);
  }
  a = wsum(a);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) red[w] = a;
  const int R = P.R;
  for (int n = 0; n < 3; ++n)
    for (int e = threadIdx.x; e < R * R; e += 256) {
      const int r = e / R, c = e - r * R;
      double g = 0.0;
      const GLB double* An = gl(P.A[n]);
      for (int y = 0; y < P.s[n]; ++y) g = fma(An[y * R + r], An[y * R + c], g);
      gl(P.S)[n * R * R + e] = g;
    }
  for (int n = 0; n < 3; ++n) {
    const int Kpad = (P.s[n] + BKC - 1) / BKC * BKC;
    for (int e = threadIdx.x; e < Kpad * BATCH_MAX_R; e += 256) {
      const int c = e / Kpad, y = e - c * Kpad;
      gl(P.Af[n])[e] = (y < P.s[n] && c < R) ? (float)gl(P.A[n])[y * R + c] : 0.f;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    BState& S = st[p];
    S.normX2 = ((red[0] + red[1]) + red[2]) + red[3];
    S.kind = BK_NONE;
    S.prev_kind = BK_NONE;
    S.sweep = 0;
    S.done = 0;
    S.conv_sweep = -1;
    S.n_als = S.n_init = S.n_approx = 0;
    S.fit = S.fit_prev = 0.0;
    for (int n = 0; n < 3; ++n) {
      S.rel[n] = 1.0;
      S.chol[n] = 0;
    }
    S.gs = 0.0;
    S.t_start = 0;
    S.t_conv = 0;
  }
}

// ---------------------------------------------------------------------------
int batch_gemm_rows(int variant) { return variant == 0 ? 64 : 128; }

static int grid_for(int ntiles) { return ntiles < 2048 ? (ntiles > 0 ? ntiles : 1) : 2048; }

hipError_t launch_b_begin(BState* st, BProb* pr, const BConf* conf, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_b_begin, dim3((count + 255) / 256), dim3(256), 0, s, st, pr, conf, count);
  return hipGetLastError();
}
hipError_t launch_b_f32(const BProb* pr, const BState* st, int count, int mode_mask, hipStream_t s) {
  hipLaunchKernelGGL(k_b_f32, dim3(count), dim3(256), 0, s, pr, st, count, mode_mask);
  return hipGetLastError();
}
hipError_t launch_b_prep(const BProb* pr, const BState* st, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_b_prep, dim3(count), dim3(256), 0, s, pr, st, count);
  return hipGetLastError();
}
hipError_t launch_b_gemm(int variant, const BProb* pr, const BState* st, const BTile* tiles,
                         int ntiles, int cmode, int out_op, int kind_mask, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  const dim3 grid(grid_for(ntiles)), block(256);
  const bool kcm = cmode == 2;
  if (variant == 0) {
    if (kcm) hipLaunchKernelGGL((k_b_gemm<64, true>), grid, block, 0, s, pr, st, tiles, ntiles, cmode, out_op, kind_mask);
    else hipLaunchKernelGGL((k_b_gemm<64, false>), grid, block, 0, s, pr, st, tiles, ntiles, cmode, out_op, kind_mask);
  } else {
    if (kcm) hipLaunchKernelGGL((k_b_gemm<128, true>), grid, block, 0, s, pr, st, tiles, ntiles, cmode, out_op, kind_mask);
    else hipLaunchKernelGGL((k_b_gemm<128, false>), grid, block, 0, s, pr, st, tiles, ntiles, cmode, out_op, kind_mask);
  }
  return hipGetLastError();
}
hipError_t launch_b_ttv(const BProb* pr, const BState* st, const BTile* tiles, int ntiles, int mode,
                        int build_mp, hipStream_t s) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_b_ttv, dim3(ntiles < 16384 ? ntiles : 16384), dim3(256), 0, s, pr, st, tiles,
                     ntiles, mode, build_mp);
  return hipGetLastError();
}
static size_t b_solve_lds(int maxR) {
  return ((size_t)64 * CH64_LS + 2 * (size_t)maxR * maxR + 64 + 2 * (size_t)BSOLVE_CH * maxR +
          (size_t)BSOLVE_WAVES * BSOLVE_RPW * 64) *
         sizeof(double);
}
// The solve's LDS request above 64 KB is enabled once, outside any graph capture.
hipError_t batch_prepare() {
  return hipFuncSetAttribute((const void*)k_b_solve, hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)b_solve_lds(BATCH_MAX_R));
}
hipError_t launch_b_solve(const BProb* pr, BState* st, const BConf* conf, int count, int mode,
                          int maxR, hipStream_t s) {
  hipLaunchKernelGGL(k_b_solve, dim3(count), dim3(BSOLVE_WAVES * 64), b_solve_lds(maxR), s, pr, st,
                     conf, mode);
  return hipGetLastError();
}
hipError_t launch_b_end(BState* st, const BConf* conf, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_b_end, dim3((count + 255) / 256), dim3(256), 0, s, st, conf, count);
  return hipGetLastError();
}
hipError_t launch_b_norm(const BProb* pr, BState* st, const BConf* conf, int count, hipStream_t s) {
  hipLaunchKernelGGL(k_b_norm, dim3(count), dim3(256), 0, s, pr, st, conf, count);
  return hipGetLastError();
}

}  // namespace ppk
