// Latency-optimised FP64 mode tail for rank <= 64 (one 64-lane wave spans a row of
// any R x R quantity).  Per mode:
//
//  1. a one-workgroup "head" kernel, launched on an auxiliary stream so that it runs
//     concurrently with the mode's contractions (TTV or first-level GEMM) on the main
//     stream: it forms Gamma^(n) = Hadamard_{i != n} S^(i) and, in PP sweeps,
//     W^(n) = sum over unordered pairs {i,j} (i,j != n) of U^(i)*U^(j)*Hadamard_{k != i,j,n} S^(k),
//     and factorises Gamma^(n) = L L^T (one wave, LDS resident, panels of 16 columns
//     updated on the matrix cores, no workgroup barriers), retrying once with
//     Gamma + delta I, delta = R 2^-52 max(diag Gamma), if a pivot is not positive;
//  2. a fused solve with small blocks spread over the chip: M~ = base + sum of the
//     contraction's partial slots + A^(n) W^(n) (PP), the two triangular solves (as
//     unit-triangular substitutions and diagonal scalings), G = (A_old - A_new) Gamma,
//     dA and per-block norm partials;
//  3. the Grams S^(n) = A^T A and U^(n) = A^T dA on the matrix cores (one block per
//     16 x 16 tile), whose first block also writes the sweep record and the fit.
//     On the auxiliary stream it precedes the next mode's head; after the last mode it
//     runs on the main stream.
#include "common.h"
#include "tail_dev.h"
#include <algorithm>
#include "../../include/ppals.h"

namespace ppk {

// Gamma^(n)[e] = prod_{i != n} S^(i)[e]
__device__ __forceinline__ double gamma_entry(const double* S, int N, int n, int64_t RR, int e) {
  double sv[PP_MAXN];
#pragma unroll
  for (int i = 0; i < PP_MAXN; ++i) sv[i] = (i < N && i != n) ? S[i * RR + e] : 1.0;
  double v = 1.0;
#pragma unroll
  for (int i = 0; i < PP_MAXN; ++i) v *= sv[i];
  return v;
}

constexpr int HEAD_THREADS = 256;

// Head of mode n (one workgroup of four waves): Gamma^(n), W^(n) (PP), the Cholesky
// factor (wave 0, one diagonal-shift retry) and the solve operands.  Small enough to be
// co-resident with the contraction kernels that run meanwhile on the other stream.  NM
// is the tensor order; thread t takes row t / 4 and columns t % 4 + 4 j, a batch of CB
// columns at a time with the loads of every other mode's S (and U) issued together.
template <int NM>
__global__ __launch_bounds__(HEAD_THREADS) void k_head(HeadArgs h) {
  constexpr int NO = NM - 1;                 // modes other than n
  constexpr int CB = 16 / NO > 1 ? 16 / NO : 2;
  __shared__ double Lm[64 * CH64_LS];        // Gamma, zero-padded to 64 x 64
  __shared__ double cb[128];
  __shared__ double red[HEAD_THREADS / 64];
  if (h.gate && *h.gate == 0) return;
  __builtin_amdgcn_s_setprio(3);  // latency-bound: first in line for issue beside streaming kernels
  const int tid = threadIdx.x;
  const int R = h.R, RR = R * R;
  const int n = h.n;
  const bool wterm = h.pp && h.second_order;
  for (int e = tid; e < 64 * CH64_LS; e += HEAD_THREADS) {
    const int r = e / CH64_LS, c = e - r * CH64_LS;
    if (r >= R || c >= R) Lm[e] = 0.0;
  }
  const int row = tid >> 2, c0 = tid & 3;
  double dmax = 0.0;
  if (h.gamma_ready) {
    if (row < R) {
      double gv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = c0 + 4 * j;
        gv[j] = h.gamma[row * R + (c < R ? c : 0)];
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = c0 + 4 * j;
        if (c < R) {
          Lm[row * CH64_LS + c] = gv[j];
          if (row == c) dmax = fmax(dmax, gv[j]);
        }
      }
    }
  } else if (row < R) {
    for (int j0 = 0; c0 + 4 * j0 < R; j0 += CB) {
      double sv[CB][NO], uv[CB][NO];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int c = c0 + 4 * (j0 + j);
        const int e = row * R + (c < R ? c : 0);
#pragma unroll
        for (int k = 0; k < NO; ++k) {
          const int mk = k + (k >= n ? 1 : 0);
          sv[j][k] = h.S[(int64_t)mk * RR + e];
          uv[j][k] = wterm ? h.U[(int64_t)mk * RR + e] : 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int c = c0 + 4 * (j0 + j);
        if (c < R) {
          // Running sums over the modes k != n: P0 = prod s_k (= Gamma), P1 = sum_i u_i
          // prod_{k != i} s_k, P2 = sum_{i<j} u_i u_j prod_{k != i,j} s_k (= W).
          double P0 = 1.0, P1 = 0.0, P2 = 0.0;
#pragma unroll
          for (int k = 0; k < NO; ++k) {
            P2 = fma(P2, sv[j][k], P1 * uv[j][k]);
            P1 = fma(P1, sv[j][k], P0 * uv[j][k]);
            P0 *= sv[j][k];
          }
          const int e = row * R + c;
          h.gamma[e] = P0;
          Lm[row * CH64_LS + c] = P0;
          if (row == c) dmax = fmax(dmax, P0);
          if (wterm) h.W[e] = P2;
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  if (tid < 64) {  // the factorisation is wave 0's alone; the other waves wait below
    int st = 0;
    for (int attempt = 0;; ++attempt) {
      if (chol_wave64(Lm, cb, R)) break;
      if (attempt == 1) {
        st = 2;
        break;
      }
      double mx = 0.0;
      for (int i = 0; i < HEAD_THREADS / 64; ++i) mx = fmax(mx, red[i]);
      const double delta = (double)R * 0x1p-52 * mx;
      for (int e = tid; e < 64 * CH64_LS; e += 64) {
        const int r = e / CH64_LS, c = e - r * CH64_LS;
        Lm[e] = (r < R && c < R) ? gamma_entry(h.S, h.N, n, RR, r * R + c) + (r == c ? delta : 0.0) : 0.0;
      }
      st = 1;
    }
    if (tid < R) cb[tid] = 1.0 / Lm[tid * CH64_LS + tid];
    if (tid == 0) h.status[n] = st;
  }
  __syncthreads();
  // the solve operands: LF[k][i] = L[i][k] / L[k][k] (i > k), LB[i][k] = L[i][k] / L[i][i]
  // (k < i), zero elsewhere, then 1 / L[i][i]
  double* LF = h.pack;
  double* LB = LF + RR;
  if (row < R) {
    const double di = cb[row];
    for (int c = c0; c < R; c += 4) {
      const double v = c <= row ? Lm[row * CH64_LS + c] : 0.0;
      LF[c * R + row] = row > c ? v * cb[c] : 0.0;
      LB[row * R + c] = c < row ? v * di : 0.0;
    }
    if (c0 == 0) LB[RR + row] = di;
  }
}

// ---------------------------------------------------------------------------
// Fused right-hand-side assembly + solve + per-block norm partials.
// Block: SOLVE_WAVES waves, one row each.
// ---------------------------------------------------------------------------
constexpr int SOLVE_WAVES = 4;
constexpr int SOLVE_BR = SOLVE_WAVES;               // rows per block
constexpr int NPART = 5;                            // per-block norm partials

// Fused right-hand-side assembly + solve.  Per row: M~ = base + sum of the contraction's
// partial slots + A_old W (PP second-order term); then Gamma x = M~ through L L^T with
// the factor split as L = (L D^-1) D (D = diag L): a unit lower substitution, a scaling
// by D^-1, a unit upper substitution with D^-1 L and a last scaling by D^-1 (the head
// forms the unit factors).  Each substitution step is one lane broadcast and one FMA.
// Products with a full R x R matrix (A_old W, the gradient and the fit term) read the
// row vector back from LDS as broadcasts, eight entries per batch.  Then
// g = (A_old - A_new) Gamma and dA = A_new - ref.  Per block it writes NPART partial
// sums: ||g||^2, ||dA||^2, ||A_new||^2, <M~, A_new> and, for the fit, sum of
// A_new Gamma A_new^T (the squared norm of the CP model, row by row).
__global__ __launch_bounds__(SOLVE_WAVES * 64) void k_solve_fused(FusedSolveArgs a) {
  constexpr int UB = 8;  // steps whose LDS operands are read together
  extern __shared__ double sm[];
  if (a.gate && *a.gate == 0) return;
  __builtin_amdgcn_s_setprio(3);
  const int R = a.R, RR = R * R;
  const int npk = 2 * RR + R;
  double* LF = sm;               // LF[j][k] = L[k][j] / L[j][j] for k > j, else 0
  double* LB = LF + RR;          // LB[j][k] = L[j][k] / L[j][j] for k < j, else 0
  double* invd = LB + RR;        // 1 / L[j][j]
  double* Gs = LF + npk;         // Gamma
  double* Ws = Gs + RR;          // second-order term
  double* vb = Ws + RR;          // per-wave broadcast vectors, SOLVE_WAVES x 3 x 64
  __shared__ double red[SOLVE_WAVES][NPART];

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid >> 6, l = tid & 63;
  const bool lv = l < R;
  const int lc = lv ? l : 0;
  const int64_t row = (int64_t)blockIdx.x * SOLVE_BR + w;
  const bool rv = row < a.rows;
  const bool ok = rv && lv;
  const int64_t off = row * R + l;
  // loads are unconditional (clamped row and column), masked afterwards
  const int64_t offc = (rv ? row : a.rows - 1) * R + lc;
  double m = a.base ? a.base[offc] : 0.0;
  double ao = a.A[offc];
  double rf = a.Aref ? a.Aref[offc] : 0.0;
  {
    // slot loads issued SLOTB at a time (clamped to the last slot, masked), summed in order
    constexpr int SLOTB = 32;
    for (int sl = 0; sl < a.nslots; sl += SLOTB) {
      double ps[SLOTB];
#pragma unroll
      for (int u = 0; u < SLOTB; ++u)
        ps[u] = a.part[(int64_t)min(sl + u, a.nslots - 1) * a.slot_stride + offc];
#pragma unroll
      for (int u = 0; u < SLOTB; ++u)
        if (sl + u < a.nslots) m += ps[u];
    }
  }
  m = ok ? m : 0.0;
  ao = ok ? ao : 0.0;
  rf = ok ? rf : 0.0;
  // stage the head's unit factors and 1 / diag L, Gamma and W
  {
    constexpr int ST = 8;
    auto copy = [&](double* dst, const double* src, int cnt) {
      for (int e0 = tid; e0 < cnt; e0 += ST * nthr) {
        double v[ST];
#pragma unroll
        for (int u = 0; u < ST; ++u) v[u] = src[min(e0 + u * nthr, cnt - 1)];
#pragma unroll
        for (int u = 0; u < ST; ++u)
          if (e0 + u * nthr < cnt) dst[e0 + u * nthr] = v[u];
      }
    };
    copy(LF, a.pack, npk);
    copy(Gs, a.gamma, RR);
    if (a.W) copy(Ws, a.W, RR);
  }
  __syncthreads();

  double* bv = vb + w * 3 * 64;
  const int st = *a.status;
  if (a.W) {  // M~ += A_old W
    bv[l] = ao;
    __builtin_amdgcn_wave_barrier();
    for (int j0 = 0; j0 < R; j0 += UB) {
      double wv[UB], av[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        const int j = min(j0 + u, R - 1);
        wv[u] = Ws[j * R + lc];
        av[u] = j0 + u < R ? bv[j] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) m = fma(av[u], wv[u], m);
    }
  }
  const double mo = m;
  double x;
  if (st != 2) {
    const double dl = lv ? invd[lc] : 0.0;
    for (int j0 = 0; j0 < R; j0 += UB) {            // (L D^-1) y = M~
      double lf[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) lf[u] = LF[min(j0 + u, R - 1) * R + lc];
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (j0 + u < R) m = fma(-lf[u], bcast(m, j0 + u), m);
    }
    m *= dl;
    for (int j1 = R - 1; j1 >= 0; j1 -= UB) {       // (D^-1 L)^T v = D^-1 y, descending
      double lb[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) lb[u] = LB[max(j1 - u, 0) * R + lc];
#pragma unroll
      for (int u = 0; u < UB; ++u)
        if (j1 - u >= 0) m = fma(-lb[u], bcast(m, j1 - u), m);
    }
    x = m * dl;
  } else {
    x = ao;
  }
  // g = (a_old - a_new) Gamma; h = a_new Gamma (fit)
  double g = 0.0, hq = 0.0;
  bv[64 + l] = lv ? ao - x : 0.0;
  bv[128 + l] = lv ? x : 0.0;
  __builtin_amdgcn_wave_barrier();
  for (int j0 = 0; j0 < R; j0 += UB) {
    double gv[UB], dv[UB], xv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      const int j = min(j0 + u, R - 1);
      const bool in = j0 + u < R;
      gv[u] = Gs[j * R + lc];
      dv[u] = in ? bv[64 + j] : 0.0;
      xv[u] = in ? bv[128 + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      g = fma(dv[u], gv[u], g);
      hq = fma(xv[u], gv[u], hq);
    }
  }
  double v[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (ok) {
    const double ref = a.Aref ? rf : ao;
    const double d = x - ref;
    a.A[off] = x;
    if (a.dA) a.dA[off] = d;
    v[0] = g * g;
    v[1] = d * d;
    v[2] = x * x;
    v[3] = mo * x;
    v[4] = a.write_fit ? x * hq : 0.0;
  }
#pragma unroll
  for (int c = 0; c < NPART; ++c) v[c] = wsum(v[c]);
  if (l == 0) {
#pragma unroll
    for (int c = 0; c < NPART; ++c) red[w][c] = v[c];
  }
  __syncthreads();
  if (tid < NPART) {
    double s = 0.0;
    for (int q = 0; q < SOLVE_WAVES; ++q) s += red[q][tid];
    a.blockpart[(int64_t)blockIdx.x * NPART + tid] = s;
  }
}

// Grams of the updated factor on the matrix cores: S = A^T A and, in PP sweeps,
// U = A^T dA.  One workgroup of GRAM_WAVES waves per 16 x 16 output tile, computing the
// tile of S and of U from one read of A's tile columns; each wave takes GRAM_U groups of
// 4 rows at a time and loads the next groups before the current matrix-core steps
// (f64 16x16x4: lane l supplies A[y0 + l/16][r0 + l%16] and B[y0 + l/16][c0 + l%16];
// accumulator register v holds tile row 4v + l/16, column l%16).  When asked, each
// workgroup also forms its tile of Gamma^(next) and W^(next) for the following mode's
// head, with the other modes' S and U tiles loaded at the start.  Block 0 also reduces the
// solve's per-block partials into the sweep record (and the fit).
constexpr int GRAM_WAVES = 16;
constexpr int GRAM_U = 4;

__global__ __launch_bounds__(GRAM_WAVES * 64) void k_gram_tiles(GramArgs a) {
  __shared__ double racc[(GRAM_WAVES / 2) * 2 * 4 * 64];
  __shared__ double tileS[256], tileU[256];
  extern __shared__ double tileO[];  // the other modes' S and U tiles, (N - 2) x 2 x 256
  if (a.gate && *a.gate == 0) return;
  __builtin_amdgcn_s_setprio(3);
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int R = a.R, RR = R * R;
  const int NBR = (R + 15) / 16;
  const int r0 = (blockIdx.x / NBR) * 16, c0 = (blockIdx.x % NBR) * 16;
  const bool has_u = a.dA != nullptr;
  // this thread's tile entry for Gamma^(next): the other modes' S and U, loaded up front
  const bool want_g = a.gamma_out != nullptr;
  const int te_r = r0 + ((tid & 255) >> 4), te_c = c0 + (tid & 15);
  const bool te_ok = want_g && te_r < R && te_c < R;
  const int ky = l >> 4, cc = l & 15;
  const bool oka = r0 + cc < R, okb = c0 + cc < R;
  const int64_t rows = a.rows;
  d4 accS = {0.0, 0.0, 0.0, 0.0}, accU = {0.0, 0.0, 0.0, 0.0};
  double xa[GRAM_U], xb[GRAM_U], xd[GRAM_U];
  auto load = [&](int64_t y0, double (&va)[GRAM_U], double (&vb)[GRAM_U], double (&vd)[GRAM_U]) {
#pragma unroll
    for (int u = 0; u < GRAM_U; ++u) {
      const int64_t y = y0 + 4 * u + ky;
      const bool in = y < rows;
      va[u] = (in && oka) ? a.A[y * R + r0 + cc] : 0.0;
      vb[u] = (in && okb) ? a.A[y * R + c0 + cc] : 0.0;
      vd[u] = (in && okb && has_u) ? a.dA[y * R + c0 + cc] : 0.0;
    }
  };
  const int64_t step = (int64_t)4 * GRAM_U * GRAM_WAVES;
  int64_t y0 = (int64_t)w * 4 * GRAM_U;
  load(y0, xa, xb, xd);
  if (want_g) {
    // the other modes' tiles, in the same round trip as the first operands: thread t takes
    // entry t % 256 of mode k = t / 256 + 4 j (S and U)
    // (other mode o = the o-th mode that is neither this one nor the next)
    const int e = te_ok ? te_r * R + te_c : 0;
#pragma unroll
    for (int j = 0; j < (PP_MAXN - 2 + 3) / 4; ++j) {
      const int o = (tid >> 8) + 4 * j;
      int k = -1;
      for (int q = 0, cnt = 0; q < a.N; ++q)
        if (q != a.mode && q != a.next && cnt++ == o) k = q;
      if (k >= 0) {
        const double sv = a.S_all[(int64_t)k * RR + e];
        const double uv = a.wterm ? a.U_all[(int64_t)k * RR + e] : 0.0;
        tileO[(o * 2 + 0) * 256 + (tid & 255)] = sv;
        tileO[(o * 2 + 1) * 256 + (tid & 255)] = uv;
      }
    }
  }
  for (; y0 < rows; y0 += step) {
    double na[GRAM_U], nb[GRAM_U], nd[GRAM_U];
    const bool more = y0 + step < rows;
    if (more) load(y0 + step, na, nb, nd);
#pragma unroll
    for (int u = 0; u < GRAM_U; ++u) {
      accS = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xb[u], accS, 0, 0, 0);
      if (has_u) accU = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xd[u], accU, 0, 0, 0);
    }
    if (more) {
#pragma unroll
      for (int u = 0; u < GRAM_U; ++u) {
        xa[u] = na[u];
        xb[u] = nb[u];
        xd[u] = nd[u];
      }
    }
  }
  // two-stage reduction over the waves: the upper half adds into the lower half
  constexpr int HW = GRAM_WAVES / 2;
  if (w >= HW) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      racc[(((w - HW) * 2 + 0) * 4 + v) * 64 + l] = accS[v];
      racc[(((w - HW) * 2 + 1) * 4 + v) * 64 + l] = accU[v];
    }
  }
  __syncthreads();
  if (w < HW) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      racc[((w * 2 + 0) * 4 + v) * 64 + l] += accS[v];
      racc[((w * 2 + 1) * 4 + v) * 64 + l] += accU[v];
    }
  }
  __syncthreads();
  if (w < 2 && (w == 0 || has_u)) {
    double* out = w ? a.U_out : a.S_out;
    double* tile = w ? tileU : tileS;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double sum = 0.0;
      for (int q = 0; q < HW; ++q) sum += racc[((q * 2 + w) * 4 + v) * 64 + l];
      const int tr = 4 * v + (l >> 4), tc = l & 15;
      const int r = r0 + tr, c = c0 + tc;
      if (r < R && c < R) out[r * R + c] = sum;
      tile[tr * 16 + tc] = sum;
    }
  }
  if (want_g) {
    __syncthreads();
    if (te_ok && tid < 256) {
      // Running sums over the modes k != next (order of k as in the head): P0 = Gamma,
      // P2 = W (second-order term)
      double P0 = 1.0, P1 = 0.0, P2 = 0.0;
      int o = 0;
      for (int k = 0; k < a.N; ++k) {
        if (k == a.next) continue;
        double sk, uk;
        if (k == a.mode) {
          sk = tileS[tid];
          uk = has_u ? tileU[tid] : 0.0;
        } else {
          sk = tileO[(o * 2 + 0) * 256 + tid];
          uk = tileO[(o * 2 + 1) * 256 + tid];
          ++o;
        }
        P2 = fma(P2, sk, P1 * uk);
        P1 = fma(P1, sk, P0 * uk);
        P0 *= sk;
      }
      const int e = te_r * R + te_c;
      a.gamma_out[e] = P0;
      if (a.wterm) a.W_out[e] = P2;
    }
  }
  if (blockIdx.x != 0) return;
  // record for this mode from the solve's per-block partials
  __shared__ double sums[NPART];
  if (w == 0) {
    double v[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int b = l; b < a.nblk; b += 64)
#pragma unroll
      for (int c = 0; c < NPART; ++c) v[c] += a.blockpart[(int64_t)b * NPART + c];
#pragma unroll
    for (int c = 0; c < NPART; ++c) v[c] = wsum(v[c]);
    if (l == 0) {
#pragma unroll
      for (int c = 0; c < NPART; ++c) sums[c] = v[c];
      ppals_sweep_record* rec = (ppals_sweep_record*)a.rec;
      const double g2 = sums[0], d2 = sums[1], a2 = sums[2];
      rec->grad_norm[a.mode] = sqrt(g2);
      rec->rel_change[a.mode] = a2 > 0.0 ? sqrt(d2) / sqrt(a2) : (d2 > 0.0 ? INFINITY : 0.0);
      rec->chol_status[a.mode] = *a.status;
      if (a.write_fit) {
        const double r2 = a.normX2 - 2.0 * sums[3] + sums[4];
        rec->fit_est = 1.0 - sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(a.normX2);
        rec->sweep_kind = a.sweep_kind;
      }
    }
  }
}

// ---------------------------------------------------------------------------
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_head(const HeadArgs& h, hipStream_t s) {
  if (h.R > 64 || h.N < 2 || h.N > PP_MAXN) return hipErrorInvalidValue;
  switch (h.N) {
    case 2: hipLaunchKernelGGL(k_head<2>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
    case 3: hipLaunchKernelGGL(k_head<3>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
    case 4: hipLaunchKernelGGL(k_head<4>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
    case 5: hipLaunchKernelGGL(k_head<5>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
    case 6: hipLaunchKernelGGL(k_head<6>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
    case 7: hipLaunchKernelGGL(k_head<7>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
    default: hipLaunchKernelGGL(k_head<8>, dim3(1), dim3(HEAD_THREADS), 0, s, h); break;
  }
  return hipGetLastError();
}

int solve_fused_blocks(int64_t rows) { return (int)((rows + SOLVE_BR - 1) / SOLVE_BR); }

__global__ void k_set_int(int* p, int v) {
  if (threadIdx.x == 0) *p = v;
}

// Gate of a PP-approximated sweep enqueued ahead of the host's decision (Algorithm 3's
// test on the device), the first node of the graph such sweeps replay: the gate stays open
// while every relative change of the sweep before is below eps, closes otherwise and stays
// closed; the sweep kind of the record tells the host which of the enqueued sweeps ran
// (-1: skipped).  It first files the record of the sweep before (or of the host's last
// sweep, for the first replay) in ring[*ctr] and advances *ctr, so that the host reads all
// the records of the enqueued sweeps with one copy.
__global__ void k_pp_gate_ring(ppals_sweep_record* rec, int N, double eps, int* gate,
                               ppals_sweep_record* ring, int* ctr) {
  constexpr int W = (int)(sizeof(ppals_sweep_record) / sizeof(int));
  const int k = *ctr;
  const int* src = (const int*)rec;
  int* dst = (int*)(ring + k);
  for (int i = threadIdx.x; i < W; i += blockDim.x) dst[i] = src[i];
  __syncthreads();
  if (threadIdx.x != 0) return;
  bool open = *gate != 0;
  for (int n = 0; n < N; ++n) open = open && rec->rel_change[n] < eps;
  *gate = open ? 1 : 0;
  rec->sweep_kind = open ? PPALS_SWEEP_PP_APPROX : -1;
  *ctr = k + 1;
}

// Files the record of the last enqueued sweep in ring[*ctr].
__global__ void k_rec_store(const ppals_sweep_record* rec, ppals_sweep_record* ring, const int* ctr) {
  constexpr int W = (int)(sizeof(ppals_sweep_record) / sizeof(int));
  const int k = *ctr;
  const int* src = (const int*)rec;
  int* dst = (int*)(ring + k);
  for (int i = threadIdx.x; i < W; i += blockDim.x) dst[i] = src[i];
}

hipError_t launch_pp_gate_ring(void* rec, int N, double eps, int* gate, void* ring, int* ctr,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_pp_gate_ring, dim3(1), dim3(64), 0, s, (ppals_sweep_record*)rec, N, eps, gate,
                     (ppals_sweep_record*)ring, ctr);
  return hipGetLastError();
}
hipError_t launch_rec_store(const void* rec, void* ring, const int* ctr, hipStream_t s) {
  hipLaunchKernelGGL(k_rec_store, dim3(1), dim3(64), 0, s, (const ppals_sweep_record*)rec,
                     (ppals_sweep_record*)ring, ctr);
  return hipGetLastError();
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}

hipError_t launch_gram_tiles(const GramArgs& a, hipStream_t s) {
  const int NBR = (a.R + 15) / 16;
  const size_t lds = a.gamma_out ? (size_t)std::max(1, a.N - 2) * 2 * 256 * sizeof(double) : 0;
  hipLaunchKernelGGL(k_gram_tiles, dim3(NBR * NBR), dim3(GRAM_WAVES * 64), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_solve_fused(const FusedSolveArgs& a, hipStream_t s) {
  const int R = a.R;
  const size_t lds = (4 * (size_t)R * R + R + (size_t)SOLVE_WAVES * 3 * 64) * sizeof(double);
  hipError_t e = allow_lds(k_solve_fused, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_fused, dim3(solve_fused_blocks(a.rows)), dim3(SOLVE_WAVES * 64), lds,
                     s, a);
  return hipGetLastError();
}

}  // namespace ppk
