// Latency-optimised FP64 mode tail for rank <= 64 (one 64-lane wave spans a row of
// any R x R quantity).  Per mode:
//
//  1. a one-workgroup "head" kernel, launched on an auxiliary stream so that it runs
//     concurrently with the mode's contractions (TTV or first-level GEMM) on the main
//     stream: it forms Gamma^(n) = Hadamard_{i != n} S^(i) and, in PP sweeps,
//     W^(n) = sum over unordered pairs {i,j} (i,j != n) of U^(i)*U^(j)*Hadamard_{k != i,j,n} S^(k),
//     and factorises Gamma^(n) = L L^T (left-looking, one wave, LDS resident), retrying
//     once with Gamma + delta I, delta = R 2^-52 max(diag Gamma), if a pivot is not
//     positive;
//  2. a fused solve with small blocks spread over the chip: M~ = base + sum of the
//     contraction's partial slots + A^(n) W^(n) (PP), the forward and backward
//     triangular solves, G = (A_old - A_new) Gamma, dA and per-block norm partials;
//  3. the Grams S^(n) = A^T A and U^(n) = A^T dA on the matrix cores (one block per
//     16 x 16 tile), whose first block also writes the sweep record and the fit.
//     On the auxiliary stream it precedes the next mode's head; after the last mode it
//     runs on the main stream.
#include "common.h"
#include "../../include/ppals.h"

namespace ppk {

__device__ __forceinline__ double bcast(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wsum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ double bsum(double v, double* red) {
  v = wsum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
  return s;
}

// Left-looking Cholesky of the R x R matrix held in LDS (row stride LS) by wave 0 of
// the block; every thread of the block must call it (one barrier per column).
// Column j: lanes i >= j form s_i = a_ij - sum_{k<j} l_ik l_jk, then l_jj = sqrt(s_j)
// and l_ij = s_i / l_jj.  Returns 1 on success.
__device__ int chol_lds_wave(double* Lm, int R, int LS, int* fail) {
  const int tid = threadIdx.x;
  if (tid == 0) *fail = 0;
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    if (tid < 64) {
      const int i = tid;
      double s = 0.0;
      if (i >= j && i < R) {
        const double* li = Lm + i * LS;
        const double* lj = Lm + j * LS;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        int k = 0;
        for (; k + 3 < j; k += 4) {
          s0 = fma(li[k], lj[k], s0);
          s1 = fma(li[k + 1], lj[k + 1], s1);
          s2 = fma(li[k + 2], lj[k + 2], s2);
          s3 = fma(li[k + 3], lj[k + 3], s3);
        }
        for (; k < j; ++k) s0 = fma(li[k], lj[k], s0);
        s = li[j] - ((s0 + s1) + (s2 + s3));
      }
      const double sj = bcast(s, j);
      if (!(sj > 0.0) || !isfinite(sj)) {
        if (tid == 0) *fail = 1;
      } else {
        const double d = sqrt(sj);
        if (i == j) Lm[j * LS + j] = d;
        else if (i > j && i < R) Lm[i * LS + j] = s / d;
      }
    }
    __syncthreads();
    if (*fail) return 0;
  }
  return 1;
}

// Head of mode n (one workgroup): Gamma^(n), W^(n) (PP) and the Cholesky factor with one
// diagonal-shift retry.
__global__ __launch_bounds__(1024) void k_head(HeadArgs h) {
  extern __shared__ double Lm[];  // R x (R+1)
  __shared__ double red[32];
  __shared__ int fail;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int R = h.R, RR = R * R, N = h.N, LS = R + 1;
  const int n = h.n;
  double dmax = 0.0;
  for (int e = tid; e < RR; e += nthr) {
    double sv[PP_MAXN], uv[PP_MAXN];
#pragma unroll
    for (int i = 0; i < PP_MAXN; ++i) {
      sv[i] = (i < N) ? h.S[(int64_t)i * RR + e] : 1.0;
      uv[i] = (h.pp && h.second_order && i < N) ? h.U[(int64_t)i * RR + e] : 0.0;
    }
    double v = 1.0;
#pragma unroll
    for (int i = 0; i < PP_MAXN; ++i)
      if (i < N && i != n) v *= sv[i];
    h.gamma[e] = v;
    const int r = e / R, c = e - r * R;
    Lm[r * LS + c] = v;
    if (r == c) dmax = fmax(dmax, v);
    if (h.pp && h.second_order) {
      double w = 0.0;
      for (int i = 0; i < N; ++i) {
        if (i == n) continue;
        for (int j = i + 1; j < N; ++j) {
          if (j == n) continue;
          double t = uv[i] * uv[j];
          for (int k = 0; k < N; ++k)
            if (k != i && k != j && k != n) t *= sv[k];
          w += t;
        }
      }
      h.W[e] = w;
    }
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if ((tid & 63) == 0) red[16 + (tid >> 6)] = dmax;
  __syncthreads();
  int st = 0;
  if (!chol_lds_wave(Lm, R, LS, &fail)) {
    double mx = 0.0;
    for (int i = 0; i < nthr / 64; ++i) mx = fmax(mx, red[16 + i]);
    const double delta = (double)R * 0x1p-52 * mx;
    for (int e = tid; e < RR; e += nthr) {
      const int r = e / R, c = e - r * R;
      Lm[r * LS + c] = h.gamma[e] + (r == c ? delta : 0.0);
    }
    __syncthreads();
    st = chol_lds_wave(Lm, R, LS, &fail) ? 1 : 2;
  }
  for (int e = tid; e < RR; e += nthr) {
    const int r = e / R, c = e - r * R;
    h.L[e] = (c <= r) ? Lm[r * LS + c] : 0.0;
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
// partial slots + A_old W (PP second-order term); forward and backward substitution with
// L (lane k owns column k); g = (A_old - A_new) Gamma; dA = A_new - ref.  Per block it
// writes NPART partial sums: ||g||^2, ||dA||^2, ||A_new||^2, <M~, A_new> and, for the
// fit, sum of A_new Gamma A_new^T (the squared norm of the CP model, row by row).
__global__ __launch_bounds__(SOLVE_WAVES * 64) void k_solve_fused(FusedSolveArgs a) {
  constexpr int ROWS = SOLVE_ROWS;
  constexpr int BR = SOLVE_BR;
  extern __shared__ double sm[];
  const int R = a.R, LS = R + 1, RR = R * R;
  double* Ls = sm;                          // R x (R+1)
  double* Gs = Ls + (size_t)R * LS;         // R x R
  double* Ws = Gs + (size_t)R * R;          // R x R (second-order term)
  double* invd = Ws + (size_t)R * R;        // R
  __shared__ double red[SOLVE_WAVES][NPART];

  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid >> 6, l = tid & 63;
  const bool lv = l < R;
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
  // stage L, Gamma, W through registers (loads issued together)
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
        const int i = e / R, k = e - i * R;
        Ls[i * LS + k] = stL[t];
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
  for (int e = tid; e < R; e += nthr) invd[e] = 1.0 / Ls[e * LS + e];
  __syncthreads();

  const int st = *a.status;
  if (a.W) {
    for (int j = 0; j < R; ++j) {
      const double wj = lv ? Ws[j * R + l] : 0.0;
#pragma unroll
      for (int q = 0; q < ROWS; ++q) m[q] = fma(bcast(ao[q], j), wj, m[q]);
    }
  }
  double mo[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) mo[q] = m[q];
  if (st != 2) {
    for (int j = 0; j < R; ++j) {       // forward: L z = m
      const double lkj = (lv && l > j) ? Ls[l * LS + j] : 0.0;
      const double ij = invd[j];
#pragma unroll
      for (int q = 0; q < ROWS; ++q) {
        const double zj = bcast(m[q], j) * ij;
        m[q] = (l == j) ? zj : m[q] - lkj * zj;
      }
    }
    for (int j = R - 1; j >= 0; --j) {  // backward: L^T x = z
      const double ljk = (lv && l < j) ? Ls[j * LS + l] : 0.0;
      const double ij = invd[j];
#pragma unroll
      for (int q = 0; q < ROWS; ++q) {
        const double xj = bcast(m[q], j) * ij;
        m[q] = (l == j) ? xj : m[q] - ljk * xj;
      }
    }
#pragma unroll
    for (int q = 0; q < ROWS; ++q) x[q] = lv ? m[q] : 0.0;
  } else {
#pragma unroll
    for (int q = 0; q < ROWS; ++q) x[q] = ao[q];
  }
  double g[ROWS], hq[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) g[q] = hq[q] = 0.0;
  for (int j = 0; j < R; ++j) {          // g = (a_old - a_new) Gamma; h = a_new Gamma (fit)
    const double gjk = lv ? Gs[j * R + l] : 0.0;
#pragma unroll
    for (int q = 0; q < ROWS; ++q) {
      g[q] = fma(bcast(ao[q] - x[q], j), gjk, g[q]);
      if (a.write_fit) hq[q] = fma(bcast(x[q], j), gjk, hq[q]);
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
// U = A^T dA.  One block per 16 x 16 output tile (grid.y selects S or U); the rows are
// staged through LDS in chunks of GCH and split over the block's waves (f64 16x16x4;
// lane l: A operand A[k][r0 + l%16], B operand B[k][c0 + l%16] with k = 4s + l/16;
// accumulator register v holds tile row 4v + l/16, column l%16).  Block (0, 0) also
// reduces the solve's per-block partials into the sweep record (and the fit).
constexpr int GCH = 192;
constexpr int GWAVES = 16;

__global__ __launch_bounds__(GWAVES * 64) void k_gram_tiles(GramArgs a) {
  __shared__ double sh[2 * GCH * 16];  // two row panels; reused for the wave reduction
  double(*ta)[16] = (double(*)[16])sh;
  double(*tb)[16] = (double(*)[16])(sh + GCH * 16);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int w = tid >> 6, l = tid & 63;
  const int R = a.R;
  const int NBR = (R + 15) / 16;
  const int r0 = (blockIdx.x / NBR) * 16, c0 = (blockIdx.x % NBR) * 16;
  const double* B = blockIdx.y ? a.dA : a.A;
  double* out = blockIdx.y ? a.U_out : a.S_out;
  d4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int64_t y0 = 0; y0 < a.rows; y0 += GCH) {
    constexpr int PER = GCH * 16 / (GWAVES * 64);
    double va[PER], vb[PER];
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * nthr;
      const int rr = e >> 4, cc = e & 15;
      const int64_t y = y0 + rr;
      va[t] = (y < a.rows && r0 + cc < R) ? a.A[y * R + r0 + cc] : 0.0;
      vb[t] = (y < a.rows && c0 + cc < R) ? B[y * R + c0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int e = tid + t * nthr;
      ta[e >> 4][e & 15] = va[t];
      tb[e >> 4][e & 15] = vb[t];
    }
    __syncthreads();
#pragma unroll
    for (int k0 = 4 * w; k0 < GCH; k0 += 4 * GWAVES) {
      const int k = k0 + (l >> 4);
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[k][l & 15], tb[k][l & 15], acc, 0, 0, 0);
    }
  }
  __syncthreads();
  double* racc = sh;  // GWAVES x 4 x 64
#pragma unroll
  for (int v = 0; v < 4; ++v) racc[(w * 4 + v) * 64 + l] = acc[v];
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      double s = 0.0;
      for (int q = 0; q < GWAVES; ++q) s += racc[(q * 4 + v) * 64 + l];
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
  const size_t lds = (size_t)h.R * (h.R + 1) * sizeof(double);
  hipLaunchKernelGGL(k_head, dim3(1), dim3(1024), lds, s, h);
  return hipGetLastError();
}

int solve_fused_blocks(int64_t rows) { return (int)((rows + SOLVE_BR - 1) / SOLVE_BR); }

hipError_t launch_gram_tiles(const GramArgs& a, hipStream_t s) {
  const int NBR = (a.R + 15) / 16;
  hipLaunchKernelGGL(k_gram_tiles, dim3(NBR * NBR, a.dA ? 2 : 1), dim3(GWAVES * 64), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_solve_fused(const FusedSolveArgs& a, hipStream_t s) {
  const int R = a.R;
  const size_t lds = ((size_t)R * (R + 1) + 2 * (size_t)R * R + R) * sizeof(double);
  hipError_t e = allow_lds(k_solve_fused, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_fused, dim3(solve_fused_blocks(a.rows)), dim3(SOLVE_WAVES * 64), lds,
                     s, a);
  return hipGetLastError();
}

}  // namespace ppk
