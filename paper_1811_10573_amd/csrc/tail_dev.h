// Wave-level FP64 helpers shared by the per-mode tail kernels: lane broadcast,
// wave sum and the one-wave blocked Cholesky factorisation of an LDS-resident
// symmetric positive definite matrix.
#pragma once
#include <hip/hip_runtime.h>

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

// Cholesky factorisation of the R x R matrix held in LDS (row stride LS), run by one
// wave with no workgroup barriers (the wave's LDS accesses complete in order); lane i
// owns row i.  Columns are taken in blocks of CHB (left-looking between blocks):
//  A. for the block's columns c = j0..j0+CHB-1, lanes i >= j0 form
//     t_ic = a_ic - sum_{k<j0} l_ik l_ck from the finished columns in LDS (the l_ck
//     are LDS broadcasts, the products independent, so this part is throughput-bound);
//  B. inside the block, column by column in registers: s_i = t_ic - sum_{j0<=k<c} l_ik l_ck
//     (l_ck read from lane c), l_cc = sqrt(s_c), l_ic = s_i * (1 / l_cc);
//  then the block's columns are written back to LDS.  Returns false at the first pivot
//  that is not positive (or not finite).
constexpr int CHB = 8;

__device__ inline bool chol_wave(double* Lm, int R, int LS) {
  const int l = threadIdx.x & 63;
  const bool own = l < R;
  for (int j0 = 0; j0 < R; j0 += CHB) {
    __builtin_amdgcn_wave_barrier();
    double t[CHB];
#pragma unroll
    for (int c = 0; c < CHB; ++c) t[c] = (own && l >= j0 && j0 + c < R) ? Lm[l * LS + j0 + c] : 0.0;
    if (own && l >= j0) {
      const double* li = Lm + l * LS;
      double u[CHB];
#pragma unroll
      for (int c = 0; c < CHB; ++c) u[c] = 0.0;
      for (int k = 0; k < j0; ++k) {
        const double lik = li[k];
#pragma unroll
        for (int c = 0; c < CHB; ++c) {
          const int rc = min(j0 + c, R - 1);  // rows past R are never used
          u[c] = fma(lik, Lm[rc * LS + k], u[c]);
        }
      }
#pragma unroll
      for (int c = 0; c < CHB; ++c) t[c] -= u[c];
    }
    double lb[CHB];
#pragma unroll
    for (int c = 0; c < CHB; ++c) {
      lb[c] = 0.0;
      const int col = j0 + c;
      if (col < R) {
        double s = t[c];
#pragma unroll
        for (int q = 0; q < c; ++q) s = fma(-lb[q], bcast(lb[q], col), s);
        const double sj = bcast(s, col);
        if (!(sj > 0.0) || !isfinite(sj)) return false;
        const double d = sqrt(sj);
        const double inv = 1.0 / d;
        lb[c] = (l == col) ? d : s * inv;
      }
    }
    if (own && l >= j0) {
#pragma unroll
      for (int c = 0; c < CHB; ++c)
        if (j0 + c < R && j0 + c <= l) Lm[l * LS + j0 + c] = lb[c];
    }
  }
  __builtin_amdgcn_wave_barrier();
  return true;
}

}  // namespace ppk
