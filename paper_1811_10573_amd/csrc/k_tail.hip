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
//  2. a fused solve: M~ = base + sum of the contraction's partial slots + A^(n) W^(n)
//     (PP), the forward and backward triangular solves, G = (A_old - A_new) Gamma, dA,
//     per-block partial Grams S = A^T A, U = A^T dA and norms.  Each wave carries ROWS
//     rows at once so their dependency chains interleave.  The last block to finish
//     (completion counter) reduces the partials into S^(n), U^(n), the sweep record and,
//     after the last mode, the fit.
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

// Head of mode n (one workgroup): Gamma^(n), W^(n) (PP), Cholesky with one diagonal-shift
// retry; zeroes the completion counter of the solve that follows.
__global__ __launch_bounds__(256) void k_head(HeadArgs h) {
  extern __shared__ double Lm[];  // R x (R+1)
  __shared__ double red[4];
  __shared__ int fail;
  const int tid = threadIdx.x;
  const int R = h.R, RR = R * R, N = h.N, LS = R + 1;
  const int n = h.n;
  if (tid == 0) h.counter[n] = 0;
  double dmax = 0.0;
  for (int e = tid; e < RR; e += blockDim.x) {
    double v = 1.0;
    for (int i = 0; i < N; ++i)
      if (i != n) v *= h.S[(int64_t)i * RR + e];
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
          double t = h.U[(int64_t)i * RR + e] * h.U[(int64_t)j * RR + e];
          for (int k = 0; k < N; ++k)
            if (k != i && k != j && k != n) t *= h.S[(int64_t)k * RR + e];
          w += t;
        }
      }
      h.W[e] = w;
    }
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  int st = 0;
  if (!chol_lds_wave(Lm, R, LS, &fail)) {
    double mx = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) mx = fmax(mx, red[i]);
    const double delta = (double)R * 0x1p-52 * mx;
    for (int e = tid; e < RR; e += blockDim.x) {
      const int r = e / R, c = e - r * R;
      Lm[r * LS + c] = h.gamma[e] + (r == c ? delta : 0.0);
    }
    __syncthreads();
    st = chol_lds_wave(Lm, R, LS, &fail) ? 1 : 2;
  }
  for (int e = tid; e < RR; e += blockDim.x) {
    const int r = e / R, c = e - r * R;
    h.L[e] = (c <= r) ? Lm[r * LS + c] : 0.0;
  }
  if (tid == 0) h.status[n] = st;
}

// ---------------------------------------------------------------------------
// Fused right-hand-side assembly + solve + Grams.  Block: 16 waves x ROWS rows; the last
// block to finish reduces the per-block partials into S^(n), U^(n) and the record.
// ---------------------------------------------------------------------------
constexpr int SOLVE_ROWS = 4;
constexpr int SOLVE_WAVES = 16;
constexpr int SOLVE_BR = SOLVE_ROWS * SOLVE_WAVES;

__global__ __launch_bounds__(1024) void k_solve_fused(FusedSolveArgs a) {
  constexpr int ROWS = SOLVE_ROWS;
  constexpr int BR = SOLVE_BR;
  extern __shared__ double sm[];
  const int R = a.R, LS = R + 1, RR = R * R;
  double* Ls = sm;                          // R x (R+1)
  double* Ws = Ls + (size_t)R * LS;         // R x R (second-order term)
  double* invd = Ws + (size_t)R * R;        // R
  double* An = invd + R;                    // BR x R new rows
  double* Dn = An + (size_t)BR * R;         // BR x R dA rows
  __shared__ double red[SOLVE_WAVES][4];
  __shared__ int is_last;

  const int tid = threadIdx.x;
  for (int e = tid; e < RR; e += blockDim.x) {
    const int i = e / R, k = e - i * R;
    Ls[i * LS + k] = a.L[e];
    if (a.W) Ws[e] = a.W[e];
  }
  __syncthreads();
  for (int e = tid; e < R; e += blockDim.x) invd[e] = 1.0 / Ls[e * LS + e];
  __syncthreads();

  const int st = *a.status;
  const int w = tid >> 6, l = tid & 63;
  const bool lv = l < R;
  const int64_t row0 = (int64_t)blockIdx.x * BR + (int64_t)w * ROWS;
  double m[ROWS], ao[ROWS], x[ROWS];
  bool rv[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    rv[q] = (row0 + q) < a.rows;
    const int64_t off = (row0 + q) * R + l;
    m[q] = (rv[q] && lv && a.base) ? a.base[off] : 0.0;
    ao[q] = (rv[q] && lv) ? a.A[off] : 0.0;
  }
  // partial slots of the contraction (independent loads, several in flight)
#pragma unroll 4
  for (int sl = 0; sl < a.nslots; ++sl) {
    const double* ps = a.part + (int64_t)sl * a.slot_stride;
#pragma unroll
    for (int q = 0; q < ROWS; ++q)
      if (rv[q] && lv) m[q] += ps[(row0 + q) * R + l];
  }
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
  double g[ROWS];
#pragma unroll
  for (int q = 0; q < ROWS; ++q) g[q] = 0.0;
  for (int j = 0; j < R; ++j) {          // g = (a_old - a_new) Gamma
    const double gjk = lv ? a.gamma[j * R + l] : 0.0;
#pragma unroll
    for (int q = 0; q < ROWS; ++q) g[q] = fma(bcast(ao[q] - x[q], j), gjk, g[q]);
  }
  double sg = 0, sd = 0, sa = 0, smm = 0;
#pragma unroll
  for (int q = 0; q < ROWS; ++q) {
    const int64_t off = (row0 + q) * R + l;
    const int lr = w * ROWS + q;
    double d = 0.0;
    if (rv[q] && lv) {
      const double ref = a.Aref ? a.Aref[off] : ao[q];
      d = x[q] - ref;
      a.A[off] = x[q];
      if (a.dA) a.dA[off] = d;
      sg = fma(g[q], g[q], sg);
      sd = fma(d, d, sd);
      sa = fma(x[q], x[q], sa);
      smm = fma(mo[q], x[q], smm);
    }
    if (lv) {
      An[lr * R + l] = rv[q] ? x[q] : 0.0;
      Dn[lr * R + l] = rv[q] ? d : 0.0;
    }
  }
  sg = wsum(sg);
  sd = wsum(sd);
  sa = wsum(sa);
  smm = wsum(smm);
  if (l == 0) {
    red[w][0] = sg;
    red[w][1] = sd;
    red[w][2] = sa;
    red[w][3] = smm;
  }
  __syncthreads();
  const int64_t blk = blockIdx.x;
  if (tid < 4) {
    double s = 0.0;
    for (int q = 0; q < SOLVE_WAVES; ++q) s += red[q][tid];
    a.blockpart[blk * 4 + tid] = s;
  }
  const int nrows = (int)min((int64_t)BR, a.rows - blk * BR);
  for (int e = tid; e < RR; e += blockDim.x) {
    const int r = e / R, c = e - (e / R) * R;
    double s = 0.0, u = 0.0;
    for (int t = 0; t < nrows; ++t) {
      const double ar = An[t * R + r];
      s = fma(ar, An[t * R + c], s);
      if (a.Upart) u = fma(ar, Dn[t * R + c], u);
    }
    a.Spart[blk * RR + e] = s;
    if (a.Upart) a.Upart[blk * RR + e] = u;
  }
  // completion count: the last block reduces every block's partials
  __threadfence();
  __syncthreads();
  if (tid == 0) is_last = (atomicAdd(a.counter, 1) == (int)gridDim.x - 1);
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  const int nb = gridDim.x;
  for (int e = tid; e < RR; e += blockDim.x) {
    double s0 = 0.0, s1 = 0.0, u0 = 0.0, u1 = 0.0;
    int b = 0;
    for (; b + 1 < nb; b += 2) {
      s0 += a.Spart[(int64_t)b * RR + e];
      s1 += a.Spart[(int64_t)(b + 1) * RR + e];
      if (a.Upart) {
        u0 += a.Upart[(int64_t)b * RR + e];
        u1 += a.Upart[(int64_t)(b + 1) * RR + e];
      }
    }
    if (b < nb) {
      s0 += a.Spart[(int64_t)b * RR + e];
      if (a.Upart) u0 += a.Upart[(int64_t)b * RR + e];
    }
    a.S_out[e] = s0 + s1;
    if (a.Upart) a.U_out[e] = u0 + u1;
  }
  if (w == 0) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int b = l; b < nb; b += 64)
#pragma unroll
      for (int c = 0; c < 4; ++c) v[c] += a.blockpart[(int64_t)b * 4 + c];
#pragma unroll
    for (int c = 0; c < 4; ++c) v[c] = wsum(v[c]);
    if (l == 0) {
      red[0][0] = v[0];
      red[0][1] = v[1];
      red[0][2] = v[2];
      red[0][3] = v[3];
    }
  }
  __threadfence_block();
  __syncthreads();
  ppals_sweep_record* rec = (ppals_sweep_record*)a.rec;
  if (a.write_fit) {
    double s = 0.0;
    for (int e = tid; e < RR; e += blockDim.x) s += a.gamma[e] * a.S_out[e];
    s = wsum(s);
    __shared__ double fr[SOLVE_WAVES];
    if (l == 0) fr[w] = s;
    __syncthreads();
    if (tid == 0) {
      double f = 0.0;
      for (int q = 0; q < SOLVE_WAVES; ++q) f += fr[q];
      const double r2 = a.normX2 - 2.0 * red[0][3] + f;
      rec->fit_est = 1.0 - sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(a.normX2);
      rec->sweep_kind = a.sweep_kind;
    }
  }
  if (tid == 0) {
    const double g2 = red[0][0], d2 = red[0][1], a2 = red[0][2];
    rec->grad_norm[a.mode] = sqrt(g2);
    rec->rel_change[a.mode] = a2 > 0.0 ? sqrt(d2) / sqrt(a2) : (d2 > 0.0 ? INFINITY : 0.0);
    rec->chol_status[a.mode] = st;
    *a.counter = 0;
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
  hipLaunchKernelGGL(k_head, dim3(1), dim3(256), lds, s, h);
  return hipGetLastError();
}

int solve_fused_blocks(int64_t rows) { return (int)((rows + SOLVE_BR - 1) / SOLVE_BR); }

hipError_t launch_solve_fused(const FusedSolveArgs& a, hipStream_t s) {
  const int R = a.R;
  const size_t lds = ((size_t)R * (R + 1) + (size_t)R * R + R + 2 * (size_t)SOLVE_BR * R) *
                     sizeof(double);
  hipError_t e = allow_lds(k_solve_fused, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_fused, dim3(solve_fused_blocks(a.rows)), dim3(1024), lds, s, a);
  return hipGetLastError();
}

}  // namespace ppk
