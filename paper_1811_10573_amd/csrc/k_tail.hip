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
#include "tail_bodies.h"
#include <algorithm>
#include "../../include/ppals.h"

namespace ppk {

template <int NM>
__global__ __launch_bounds__(HEAD_THREADS) void k_head(HeadArgs h) {
  __shared__ double lds[HEAD_LDS];
  if (h.gate && *h.gate == 0) return;
  head_body<NM>(h, lds, lds + 64 * CH64_LS, lds + 64 * CH64_LS + 128);
}

// ---------------------------------------------------------------------------
// Fused right-hand-side assembly + solve + per-block norm partials.
// Block: SOLVE_WAVES waves, one row each.
// ---------------------------------------------------------------------------
constexpr int SOLVE_WAVES = 4;
constexpr int SOLVE_BR = SOLVE_WAVES;               // rows per block

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
  // All of the block's global loads are unconditional (clamped row, column and index;
  // absent operands read A instead and are masked) and issued before the first wait: the
  // row's M_p, A and A_ref, the first SLOTB partial slots and the first SB staged
  // operand entries per thread.  Guarded loads and stores would become branches, each
  // closed by a wait, and the prologue would take one memory round trip per batch.
  const int64_t offc = (rv ? row : a.rows - 1) * R + lc;
  constexpr int SLOTB = 32, SB = 48;
  const double* basep = a.base ? a.base : a.A;
  const double* refp = a.Aref ? a.Aref : a.A;
  double m = basep[offc];
  double ao = a.A[offc];
  double rf = refp[offc];
  double ps[SLOTB];
#pragma unroll
  for (int u = 0; u < SLOTB; ++u)
    ps[u] = a.nslots > 0 ? a.part[(int64_t)min(u, a.nslots - 1) * a.slot_stride + offc] : 0.0;
  // staged operands, one flat range in LDS: the head's unit factors and 1 / diag L
  // (npk), Gamma (RR) and W (RR)
  const int tot = npk + RR + (a.W ? RR : 0);
  const double* Wsrc = a.W ? a.W : a.gamma;
  auto stage_src = [&](int e) {
    return e < npk ? a.pack + e : (e < npk + RR ? a.gamma + (e - npk) : Wsrc + (e - npk - RR));
  };
  double sv[SB];
#pragma unroll
  for (int u = 0; u < SB; ++u) sv[u] = *stage_src(min(tid + u * nthr, tot - 1));
  m = a.base ? m : 0.0;
#pragma unroll
  for (int u = 0; u < SLOTB; ++u) m += u < a.nslots ? ps[u] : 0.0;
  for (int sl = SLOTB; sl < a.nslots; sl += SLOTB) {  // more than SLOTB slots
#pragma unroll
    for (int u = 0; u < SLOTB; ++u)
      ps[u] = a.part[(int64_t)min(sl + u, a.nslots - 1) * a.slot_stride + offc];
#pragma unroll
    for (int u = 0; u < SLOTB; ++u) m += sl + u < a.nslots ? ps[u] : 0.0;
  }
  // out-of-range entries rewrite the last one with its own value
#pragma unroll
  for (int u = 0; u < SB; ++u) LF[min(tid + u * nthr, tot - 1)] = sv[u];
  for (int e0 = SB * nthr; e0 < tot; e0 += SB * nthr) {  // larger ranks
#pragma unroll
    for (int u = 0; u < SB; ++u) sv[u] = *stage_src(min(e0 + tid + u * nthr, tot - 1));
#pragma unroll
    for (int u = 0; u < SB; ++u) LF[min(e0 + tid + u * nthr, tot - 1)] = sv[u];
  }
  m = ok ? m : 0.0;
  ao = ok ? ao : 0.0;
  rf = ok ? rf : 0.0;
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
  if ((st & 3) != 2) {
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
  // Step-size variant (Section 5.1): A_new = A_old + step (A_sol - A_old).  The gradient
  // stays the one at A_old, (A_old - A_sol) Gamma.
  const double xs = x;
  if (a.step != 1.0) x = fma(a.step, xs - ao, ao);
  // g = (a_old - a_sol) Gamma; h = a_new Gamma (fit)
  double g = 0.0, hq = 0.0;
  bv[64 + l] = lv ? ao - xs : 0.0;
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

constexpr int GRAM_WAVES = 16;

template <int GW>
__global__ __launch_bounds__(GW * 64) void k_gram_tiles(GramArgs a) {
  __shared__ double racc[GRAM_RACC(GW)];
  __shared__ double tiles[512];
  extern __shared__ double tileO[];  // the other modes' S and U tiles, (N - 2) x 2 x 256
  if (a.gate && *a.gate == 0) return;
  gram_body<GW>(a, blockIdx.x, 0, racc, tiles, tiles + 256, tileO);
}

// The Gram tiles in row ranges, one workgroup per (tile, range), with the fused
// PP-correction launch's Gram role itself (same bits).
template <int GW>
__global__ __launch_bounds__(GW * 64) void k_gram_split(GramArgs a) {
  __shared__ double racc[GRAM_RACC(GW)];
  __shared__ double tiles[512];
  extern __shared__ double tileO[];
  if (a.gate && *a.gate == 0) return;
  gram_body<GW, true>(a, blockIdx.x / a.nsplit, blockIdx.x % a.nsplit, racc, tiles, tiles + 256,
                      tileO);
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
__global__ void k_set_int2(int* p, int v, int* q, int w) {
  if (threadIdx.x == 0) {
    *p = v;
    *q = w;
  }
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
hipError_t launch_set_int2(int* p, int v, int* q, int w, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int2, dim3(1), dim3(64), 0, s, p, v, q, w);
  return hipGetLastError();
}

hipError_t launch_gram_tiles(const GramArgs& a, hipStream_t s, bool tail_order) {
  const int NBR = (a.R + 15) / 16;
  const size_t lds = a.gamma_out ? (size_t)std::max(1, a.N - 2) * 2 * 256 * sizeof(double) : 0;
  constexpr int TW = TTV_VTHREADS / 64;  // the Gram role of the fused PP-correction launch
  if (tail_order && a.nsplit > 1) {
    if (!a.gpart || !a.gctr) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_gram_split<TW>, dim3(NBR * NBR * a.nsplit), dim3(TW * 64), lds, s, a);
  } else if (tail_order)
    hipLaunchKernelGGL(k_gram_tiles<TW>, dim3(NBR * NBR), dim3(TW * 64), lds, s, a);
  else
    hipLaunchKernelGGL(k_gram_tiles<GRAM_WAVES>, dim3(NBR * NBR), dim3(GRAM_WAVES * 64), lds, s, a);
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
