// Wave-level FP64 helpers shared by the per-mode tail kernels: lane broadcast,
// wave sum and the one-wave Cholesky factorisation of an LDS-resident symmetric positive
// definite matrix of order <= 64.
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

// Cholesky factorisation by one wave, for R <= 64, of the matrix held in LDS as a
// zero-padded 64 x 65 array (row stride CH64_LS; rows and columns >= R are zero).
// Columns are taken in panels of 16:
//  A. left-looking update of the panel, T[i][c] -= sum_{k<j0} L[i][k] L[j0+c][k] for
//     the row tiles at or below the panel, on the f64 16x16x4 matrix cores (operands
//     read straight from LDS: lane l supplies row l%16 and k = l/16 of a tile; the
//     accumulator register v holds row 4v + l/16, column l%16);
//  B. the panel in registers, right-looking, lane i holding row i: pivot s = t_cc
//     (broadcast from lane c), r = 1/sqrt(s) from the hardware estimate refined by two
//     Newton steps, l_cc = s r, l_ic = t_ic r, then the panel's later columns are
//     updated with the new column (the next one through a lane broadcast, the others
//     through the LDS buffer cb of 2 x 64 entries, alternating between its halves).
// Returns false at the first pivot that is not positive (or not finite).
constexpr int CH64_LS = 65;

__device__ __forceinline__ double rsqrt_refined(double s) {
  double y = __builtin_amdgcn_rsq(s);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double h = s * y;
    const double e = fma(-h, y, 1.0);  // 1 - s y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// Cholesky of the R x R leading block of Lm (one wave).  Returns -1 on success, else the
// 0-based index of the first pivot that is not positive and finite.
__device__ __forceinline__ int chol_wave64(double* Lm, double* cb, int R) {
  constexpr int LS = CH64_LS;
  const int l = threadIdx.x & 63;
  const int i16 = l & 15, k4 = l >> 4;
  for (int j0 = 0; j0 < R; j0 += 16) {
    __builtin_amdgcn_wave_barrier();
    if (j0 > 0) {
      for (int i0 = j0; i0 < R; i0 += 16) {
        d4 acc = {0.0, 0.0, 0.0, 0.0};
        const double* ar = Lm + (i0 + i16) * LS + k4;
        const double* br = Lm + (j0 + i16) * LS + k4;
        for (int k0 = 0; k0 < j0; k0 += 16) {
          double av[4], bv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            av[u] = ar[k0 + 4 * u];
            bv[u] = br[k0 + 4 * u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u], bv[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          double* dst = Lm + (i0 + 4 * v + k4) * LS + j0 + i16;
          *dst -= acc[v];
        }
      }
      __builtin_amdgcn_wave_barrier();
    }
    double t[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) t[c] = Lm[l * LS + j0 + c];
    // One basic block per panel (no branches), so the scheduler can overlap a column's
    // LDS round trip with the next columns' pivot chains: the next two entries of the
    // new column reach the rows that need them through lane broadcasts, the others
    // through LDS.  The pivot test is off the chain; a column past R (only in the last
    // panel) meets zero padding and leaves rows below R unchanged.
    int bad = -1;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
      const int col = j0 + c;
      const double s = bcast(t[c], col);
      bad = (bad < 0 && col < R && !(s > 0.0 && s < INFINITY)) ? col : bad;
      const double r = rsqrt_refined(s);
      const double lc = (l == col) ? s * r : t[c] * r;
      t[c] = lc;
      if (c + 1 < 16) t[c + 1] = fma(-lc, bcast(lc, col + 1), t[c + 1]);
      if (c + 2 < 16) t[c + 2] = fma(-lc, bcast(lc, col + 2), t[c + 2]);
      if (c + 3 < 16) {
        double* cbc = cb + 64 * (c & 1);
        cbc[l] = lc;
#pragma unroll
        for (int c2 = c + 3; c2 < 16; ++c2) t[c2] = fma(-lc, cbc[j0 + c2], t[c2]);
      }
    }
    if (bad >= 0) return bad;
#pragma unroll
    for (int c = 0; c < 16; ++c)
      if (j0 + c <= l) Lm[l * LS + j0 + c] = t[c];
  }
  __builtin_amdgcn_wave_barrier();
  return -1;
}

// Cholesky status word: bits 0-1 the outcome (0 clean, 1 factorised after the diagonal
// shift, 2 failed after it), bits 8-30 one plus the first failed pivot of the unshifted
// factorisation (0: none).
__device__ __forceinline__ int chol_status_word(int code, int pivot) {
  return code | ((pivot + 1) << 8);
}

}  // namespace ppk
