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

// Head of mode n (one workgroup of four waves): Gamma^(n), W^(n) (PP) and, in wave 0,
// the Cholesky factor with one diagonal-shift retry.  Small enough to be co-resident
// with the contraction kernels that run meanwhile on the other stream.  NM is the
// tensor order: each thread takes EB entries at a time and issues the loads of every
// mode's S (and U) for them together.
template <int NM>
__global__ __launch_bounds__(HEAD_THREADS) void k_head(HeadArgs h) {
  __shared__ double Lm[64 * CH64_LS];  // Gamma, zero-padded to 64 x 64
  __shared__ double red[HEAD_THREADS / 64];
  if (h.gate && *h.gate == 0) return;
  const int tid = threadIdx.x;
  const int R = h.R, RR = R * R;
  const int n = h.n;
  const bool wterm = h.pp && h.second_order;
  for (int e = tid; e < 64 * CH64_LS; e += HEAD_THREADS) {
    const int r = e / CH64_LS, c = e - r * CH64_LS;
    if (r >= R || c >= R) Lm[e] = 0.0;
  }
  constexpr int EB = 16 / NM > 0 ? 16 / NM : 1;
  double dmax = 0.0;
  for (int e0 = tid; e0 < RR; e0 += EB * HEAD_THREADS) {
    double sv[EB][NM], uv[EB][NM];
#pragma unroll
    for (int b = 0; b < EB; ++b) {
      const int e = e0 + b * HEAD_THREADS;
      const int ec = e < RR ? e : 0;
#pragma unroll
      for (int k = 0; k < NM; ++k) sv[b][k] = h.S[(int64_t)k * RR + ec];
      if (wterm) {
#pragma unroll
        for (int k = 0; k < NM; ++k) uv[b][k] = h.U[(int64_t)k * RR + ec];
      } else {
#pragma unroll
        for (int k = 0; k < NM; ++k) uv[b][k] = 0.0;
      }
    }
#pragma unroll
    for (int b = 0; b < EB; ++b) {
      const int e = e0 + b * HEAD_THREADS;
      if (e < RR) {
        // Running sums over the modes k != n: P0 = prod s_k (= Gamma), P1 = sum_i u_i
        // prod_{k != i} s_k, P2 = sum_{i<j} u_i u_j prod_{k != i,j} s_k (= W).
        double P0 = 1.0, P1 = 0.0, P2 = 0.0;
#pragma unroll
        for (int k = 0; k < NM; ++k) {
          const double sk = k == n ? 1.0 : sv[b][k];
          const double uk = k == n ? 0.0 : uv[b][k];
          P2 = fma(P2, sk, P1 * uk);
          P1 = fma(P1, sk, P0 * uk);
          P0 *= sk;
        }
        h.gamma[e] = P0;
        const int r = e / R, c = e - r * R;
        Lm[r * CH64_LS + c] = P0;
        if (r == c) dmax = fmax(dmax, P0);
        if (wterm) h.W[e] = P2;
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  if (tid >= 64) return;  // the factorisation is wave 0's alone (no barriers follow)
  int st = 0;
  for (int attempt = 0;; ++attempt) {
    if (chol_wave64(Lm, R)) break;
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
  for (int e = tid; e < RR; e += 64) {
    const int r = e / R, c = e - r * R;
    h.L[e] = (c <= r) ? Lm[r * CH64_LS + c] : 0.0;
  }
  if (tid == 0) h.status[n] = st;
}

// ---------------------------------------------------------------------------
// Fused right-hand-side assembly + solve + per-block partial Grams and norms.
// Block: SOLVE_WAVES waves x SOLVE_ROWS rows.
// ---------------------------------------------------------------------------
constexpr int SOLVE_ROWS = 2;
constexpr int SOLVE_WAVES = 4;
constexpr int SOLVE_BR = SOLVE_ROWS * SOLVE_WAVES;  // rows per block
constexpr int SOLVE_STAGE = 16;                     // staged L/Gamma/W entries per thread
constexpr int NPART = 5;                            // per-block norm partials

// Fused right-hand-side assembly + solve.  Per row: M~ = base + sum of the contraction's
// partial slots + A_old W (PP second-order term); then Gamma x = M~ through L L^T with
// the factor split as L = (L D^-1) D (D = diag L): a unit lower substitution, a scaling
// by D^-1, a unit upper substitution with D^-1 L and a last scaling by D^-1.  The unit
// factors are formed once per block in LDS, row j holding the entries that step j of
// each substitution subtracts, so a step is one lane broadcast and one FMA and the
// LDS reads of eight steps are issued together.  Then g = (A_old - A_new) Gamma and
// dA = A_new - ref.  Per block it writes NPART partial sums: ||g||^2, ||dA||^2,
// ||A_new||^2, <M~, A_new> and, for the fit, sum of A_new Gamma A_new^T (the squared
// norm of the CP model, row by row).
__global__ __launch_bounds__(SOLVE_WAVES * 64) void k_solve_fused(FusedSolveArgs a) {
  constexpr int ROWS = SOLVE_ROWS;
  constexpr int BR = SOLVE_BR;
  constexpr int UB = 8;  // substitution steps whose LDS operands are read together
  extern __shared__ double sm[];
  if (a.gate && *a.gate == 0) return;
  const int R = a.R, RR = R * R;
  double* LF = sm;              // LF[j][k] = L[k][j] / L[j][j] for k > j, else 0
  double* LB = LF + RR;         // LB[j][k] = L[j][k] / L[j][j] for k < j, else 0
  double* Gs = LB + RR;         // Gamma
  double* Ws = Gs + RR;         // second-order term
  double* invd = Ws + RR;       // 1 / L[j][j]
  __shared__ double red[SOLVE_WAVES][NPART];

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid >> 6, l = tid & 63;
  const bool lv = l < R;
  const int lc = lv ? l : 0;
  const int64_t row0 = (int64_t)blockIdx.x * BR + (int64_t)w * ROWS;
  double m[ROWS], ao[ROWS], rf[ROWS], x[ROWS];
  bool rv[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    rv[q] = (row0 + q) < a.rows;
    const int64_t off = (row0 + q) * R + l;
    const bool ok = rv[q] && lv;
    m[q] = (ok && a.base) ? a.base[off] : 0.0;
    ao[q] = ok ? a.A[off] : 0.0;
    rf[q] = (ok && a.Aref) ? a.Aref[off] : 0.0;
  }
  if (tid < R) invd[tid] = 1.0 / a.L[tid * R + tid];
  // stage L (raw, into LB), Gamma and W
  for (int e0 = 0; e0 < RR; e0 += SOLVE_STAGE * nthr) {
    double stL[SOLVE_STAGE], stG[SOLVE_STAGE], stW[SOLVE_STAGE];
#pragma unroll
    for (int t = 0; t < SOLVE_STAGE; ++t) {
      const int e = e0 + tid + t * nthr;
      const bool ok = e < RR;
      stL[t] = ok ? a.L[e] : 0.0;
      stG[t] = ok ? a.gamma[e] : 0.0;
      stW[t] = (ok && a.W) ? a.W[e] : 0.0;
    }
#pragma unroll
    for (int t = 0; t < SOLVE_STAGE; ++t) {
      const int e = e0 + tid + t * nthr;
      if (e < RR) {
        LB[e] = stL[t];
        Gs[e] = stG[t];
        Ws[e] = stW[t];
      }
    }
  }
#pragma unroll 8
  for (int sl = 0; sl < a.nslots; ++sl) {
    const double* ps = a.part + (int64_t)sl * a.slot_stride;
#pragma unroll
    for (int q = 0; q < ROWS; ++q)
      if (rv[q] && lv) m[q] += ps[(row0 + q) * R + l];
  }
  __syncthreads();
  // unit factors: each thread rescales the entries it staged (no other thread reads them yet)
  for (int e = tid; e < RR; e += nthr) {
    const int i = e / R, k = e - i * R;
    const double v = LB[e];
    LF[k * R + i] = i > k ? v * invd[k] : 0.0;
    LB[e] = k < i ? v * invd[i] : 0.0;
  }
  __syncthreads();

  const int st = *a.status;
  if (a.W) {
    for (int j0 = 0; j0 < R; j0 += UB) {
      double wv[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) wv[u] = (j0 + u < R && lv) ? Ws[(j0 + u) * R + lc] : 0.0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (j0 + u < R) {
#pragma unroll
          for (int q = 0; q < ROWS; ++q) m[q] = fma(bcast(ao[q], j0 + u), wv[u], m[q]);
        }
      }
    }
  }
  double mo[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) mo[q] = m[q];
  if (st != 2) {
    const double dl = lv ? invd[lc] : 0.0;
    for (int j0 = 0; j0 < R; j0 += UB) {            // (L D^-1) y = M~
      double lf[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) lf[u] = (j0 + u < R && lv) ? LF[(j0 + u) * R + lc] : 0.0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (j0 + u < R) {
#pragma unroll
          for (int q = 0; q < ROWS; ++q) m[q] = fma(-lf[u], bcast(m[q], j0 + u), m[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < ROWS; ++q) m[q] *= dl;
    for (int j1 = R - 1; j1 >= 0; j1 -= UB) {       // (D^-1 L)^T v = D^-1 y, descending
      double lb[UB];
#pragma unroll
      for (int u = 0; u < UB; ++u) lb[u] = (j1 - u >= 0 && lv) ? LB[(j1 - u) * R + lc] : 0.0;
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (j1 - u >= 0) {
#pragma unroll
          for (int q = 0; q < ROWS; ++q) m[q] = fma(-lb[u], bcast(m[q], j1 - u), m[q]);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < ROWS; ++q) x[q] = m[q] * dl;
  } else {
#pragma unroll
    for (int q = 0; q < ROWS; ++q) x[q] = ao[q];
  }
  double g[ROWS], hq[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) g[q] = hq[q] = 0.0;
  double dx[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) dx[q] = ao[q] - x[q];
  for (int j0 = 0; j0 < R; j0 += UB) {   // g = (a_old - a_new) Gamma; h = a_new Gamma (fit)
    double gv[UB];
#pragma unroll
    for (int u = 0; u < UB; ++u) gv[u] = (j0 + u < R && lv) ? Gs[(j0 + u) * R + lc] : 0.0;
#pragma unroll
    for (int u = 0; u < UB; ++u) {
      if (j0 + u < R) {
#pragma unroll
        for (int q = 0; q < ROWS; ++q) {
          g[q] = fma(bcast(dx[q], j0 + u), gv[u], g[q]);
          if (a.write_fit) hq[q] = fma(bcast(x[q], j0 + u), gv[u], hq[q]);
        }
      }
    }
  }
  double v[NPART] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int64_t off = (row0 + q) * R + l;
    if (rv[q] && lv) {
      const double ref = a.Aref ? rf[q] : ao[q];
      const double d = x[q] - ref;
      a.A[off] = x[q];
      if (a.dA) a.dA[off] = d;
      v[0] = fma(g[q], g[q], v[0]);
      v[1] = fma(d, d, v[1]);
      v[2] = fma(x[q], x[q], v[2]);
      v[3] = fma(mo[q], x[q], v[3]);
      v[4] = fma(x[q], hq[q], v[4]);
    }
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
// U = A^T dA.  One workgroup of GRAM_WAVES waves per 16 x 16 output tile (grid.y selects
// S or U); each wave takes GRAM_UNROLL groups of 4 rows at a time, its MFMA operands
// loaded straight from memory (f64 16x16x4: lane l supplies A[y0 + l/16][r0 + l%16] and
// B[y0 + l/16][c0 + l%16]; accumulator register v holds tile row 4v + l/16, column
// l%16).  Block (0, 0) also reduces the solve's per-block partials into the sweep
// record (and the fit).
constexpr int GRAM_WAVES = 4;
constexpr int GRAM_UNROLL = 8;

__global__ __launch_bounds__(GRAM_WAVES * 64) void k_gram_tiles(GramArgs a) {
  __shared__ double racc[GRAM_WAVES * 4 * 64];
  if (a.gate && *a.gate == 0) return;
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int R = a.R;
  const int NBR = (R + 15) / 16;
  const int r0 = (blockIdx.x / NBR) * 16, c0 = (blockIdx.x % NBR) * 16;
  const double* B = blockIdx.y ? a.dA : a.A;
  double* out = blockIdx.y ? a.U_out : a.S_out;
  const int ky = l >> 4, cc = l & 15;
  const bool oka = r0 + cc < R, okb = c0 + cc < R;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t y0 = (int64_t)w * 4 * GRAM_UNROLL; y0 < a.rows;
       y0 += (int64_t)4 * GRAM_UNROLL * GRAM_WAVES) {
    double xa[GRAM_UNROLL], xb[GRAM_UNROLL];
#pragma unroll
    for (int u = 0; u < GRAM_UNROLL; ++u) {
      const int64_t y = y0 + 4 * u + ky;
      xa[u] = (y < a.rows && oka) ? a.A[y * R + r0 + cc] : 0.0;
      xb[u] = (y < a.rows && okb) ? B[y * R + c0 + cc] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < GRAM_UNROLL; ++u)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xb[u], acc, 0, 0, 0);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) racc[(w * 4 + v) * 64 + l] = acc[v];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double s = 0.0;
      for (int q = 0; q < GRAM_WAVES; ++q) s += racc[(q * 4 + v) * 64 + l];
      const int r = r0 + 4 * v + (l >> 4), c = c0 + (l & 15);
      if (r < R && c < R) out[r * R + c] = s;
    }
  }
  if (blockIdx.x != 0 || blockIdx.y != 0) return;
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
// test on the device): it stays open while every relative change of the sweep before
// is below eps, closes otherwise and stays closed.  The sweep kind of the record tells
// the host which of the enqueued sweeps ran (-1: skipped).
__global__ void k_pp_gate(ppals_sweep_record* rec, int N, double eps, int* gate) {
  if (threadIdx.x != 0) return;
  bool open = *gate != 0;
  for (int n = 0; n < N; ++n) open = open && rec->rel_change[n] < eps;
  *gate = open ? 1 : 0;
  rec->sweep_kind = open ? PPALS_SWEEP_PP_APPROX : -1;
}

hipError_t launch_set_int(int* p, int v, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, p, v);
  return hipGetLastError();
}
hipError_t launch_pp_gate(void* rec, int N, double eps, int* gate, hipStream_t s) {
  hipLaunchKernelGGL(k_pp_gate, dim3(1), dim3(64), 0, s, (ppals_sweep_record*)rec, N, eps, gate);
  return hipGetLastError();
}

hipError_t launch_gram_tiles(const GramArgs& a, hipStream_t s) {
  const int NBR = (a.R + 15) / 16;
  hipLaunchKernelGGL(k_gram_tiles, dim3(NBR * NBR, a.dA ? 2 : 1), dim3(GRAM_WAVES * 64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_solve_fused(const FusedSolveArgs& a, hipStream_t s) {
  const int R = a.R;
  const size_t lds = (4 * (size_t)R * R + R) * sizeof(double);
  hipError_t e = allow_lds(k_solve_fused, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_fused, dim3(solve_fused_blocks(a.rows)), dim3(SOLVE_WAVES * 64), lds,
                     s, a);
  return hipGetLastError();
}

}  // namespace ppk
