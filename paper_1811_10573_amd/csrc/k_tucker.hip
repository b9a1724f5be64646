// Kernels of the Tucker-ALS and PP-Tucker-ALS path (Algorithms 2 and 4), FP64:
//
//  * a strided FP64 GEMM for the Gram matrix of an unfolding, W = Y_(n) Y_(n)^T, the
//    products of the subspace iteration and the core G = A^(N)T Y^(N)_(N);
//  * the Rayleigh-Ritz step of the subspace iteration that gives the leading
//    eigenvectors of W (one workgroup: Cholesky of V^T V, the projected matrix, cyclic
//    Jacobi rotations, decreasing order, column signs);
//  * the Ritz residuals, the sign rule of a start without a previous factor, the
//    first-order PP combination Y~ = Y_p + T_a + T_b^T and the core statistics.
// The TTMs themselves run on the first-level GEMM kernel (k_level1.hip).
#include "common.h"
#include "tucker.h"
#include <algorithm>

namespace ppk {

// ---------------------------------------------------------------------------
// C[m][n] = alpha * sum_k A(m, k) B(k, n) (+ beta C[m][n]) with
// A(m, k) = A[m * sam + k * sak] and B(k, n) = B[k * sbk + n * sbn]; C row-major (ldc).
// With kin > 0 the contracted index is two-level, k = k_out * kin + k_in, and
// A(m, k) = A[m * sam + k_out * sak + k_in * sak2] (same for B): the unfolding of a
// middle mode of a three-way tensor.
// 64 x 64 tiles, 256 threads with 4 x 4 outputs each, K in chunks of 16 through LDS;
// workgroup z takes the z-th of ks consecutive K ranges.  A tile is read with the
// operand's unit-stride index fastest across threads.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g, int64_t kchunk) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * GT, n0 = (int64_t)blockIdx.x * GT;
  const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
  const int64_t kend = kbeg + kchunk < g.K ? kbeg + kchunk : g.K;
  const int tm = (tid / 16) * 4, tn = (tid % 16) * 4;
  const bool a_kfast = g.kin ? g.sak2 == 1 : g.sak == 1;
  const bool b_kfast = g.kin ? g.sbk2 == 1 : g.sbk == 1;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int64_t k0 = kbeg; k0 < kend; k0 += GK) {
    for (int e = tid; e < GK * GT; e += 256) {
      const int kk = a_kfast ? e % GK : e / GT;
      const int mm = a_kfast ? e / GK : e % GT;
      const int64_t m = m0 + mm, k = k0 + kk;
      const int64_t ka = g.kin ? (k / g.kin) * g.sak + (k % g.kin) * g.sak2 : k * g.sak;
      As[kk][mm] = (m < g.M && k < kend) ? g.A[m * g.sam + ka] : 0.0;
    }
    for (int e = tid; e < GK * GT; e += 256) {
      const int kk = b_kfast ? e % GK : e / GT;
      const int nn = b_kfast ? e / GK : e % GT;
      const int64_t n = n0 + nn, k = k0 + kk;
      const int64_t kb = g.kin ? (k / g.kin) * g.sbk + (k % g.kin) * g.sbk2 : k * g.sbk;
      Bs[kk][nn] = (n < g.N && k < kend) ? g.B[kb + n * g.sbn] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][tm + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tn + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
  double* C = g.ks > 1 ? g.part + (int64_t)blockIdx.z * g.M * g.N : g.C;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t m = m0 + tm + i;
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t n = n0 + tn + j;
      if (n >= g.N) continue;
      double* c = C + m * g.ldc + n;
      *c = g.beta == 0.0 ? g.alpha * acc[i][j] : fma(g.alpha, acc[i][j], g.beta * *c);
    }
  }
}

hipError_t launch_gemm_f64(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  if (g.ks > 1 && (g.alpha != 1.0 || g.beta != 0.0 || g.ldc != g.N || !g.part))
    return hipErrorInvalidValue;
  const int ks = g.ks > 1 ? g.ks : 1;
  int64_t kchunk = (g.K + ks - 1) / ks;
  kchunk = (kchunk + GK - 1) / GK * GK;
  // splits that hold k-values (at most ks after the rounding of kchunk)
  const int nz = g.K > 0 ? (int)((g.K + kchunk - 1) / kchunk) : 1;
  const dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT), (unsigned)nz);
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, s, g, g.K > 0 ? kchunk : (int64_t)0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  return launch_reduce_splits_to(g.C, 0, g.part, 0, nz, g.M * g.N, s);
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz step (one workgroup, R <= 64).  With V the current basis (s x R),
// B = V^T V and H = V^T W V: L = chol(B), H' = L^-1 H L^-T, H' = Q diag(lam) Q^T by
// cyclic Jacobi rotations (parallel round-robin pairing), decreasing lam, and
// T = L^-T Q, so that V T are orthonormal Ritz vectors.  With P = V^T A_prev, column j
// of T is negated when (V T)_j . A_prev_j = (T^T P)_jj < 0.
// ---------------------------------------------------------------------------
constexpr int RRS = 65;  // LDS row stride

__global__ __launch_bounds__(256) void k_rayleigh_ritz(RRArgs a) {
  __shared__ double L[64 * RRS];
  __shared__ double H[64 * RRS];
  __shared__ double Q[64 * RRS];
  __shared__ double lam[64];
  __shared__ double cs[32], sn[32];
  __shared__ int pr[32], qr[32];
  __shared__ int bad;
  __shared__ double offn, diagn;
  const int tid = threadIdx.x;
  const int R = a.R;
  const int RP = R + (R & 1);  // even, for the round-robin pairing
  for (int e = tid; e < 64 * RRS; e += 256) {
    L[e] = 0.0;
    H[e] = 0.0;
    Q[e] = 0.0;
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, k = e - i * R;
    L[i * RRS + k] = a.B[e];
    H[i * RRS + k] = a.H[e];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  // Cholesky of B (lower, in place)
  for (int j = 0; j < R; ++j) {
    if (tid == 0) {
      const double d = L[j * RRS + j];
      if (!(d > 0.0) || !isfinite(d)) bad = 1;
      L[j * RRS + j] = sqrt(d > 0.0 ? d : 1.0);
    }
    __syncthreads();
    const double inv = 1.0 / L[j * RRS + j];
    for (int i = j + 1 + tid; i < R; i += 256) L[i * RRS + j] *= inv;
    __syncthreads();
    const int m = R - j - 1;
    for (int e = tid; e < m * m; e += 256) {
      const int ii = e / m, kk = e - ii * m;
      if (kk <= ii) {
        const int i = j + 1 + ii, k = j + 1 + kk;
        L[i * RRS + k] -= L[i * RRS + j] * L[k * RRS + j];
      }
    }
    __syncthreads();
  }
  // Z = L^-1 H (column j by thread j), then H' = L^-1 Z^T (symmetric)
  if (tid < R) {
    const int j = tid;
    for (int i = 0; i < R; ++i) {
      double z = H[i * RRS + j];
      for (int k = 0; k < i; ++k) z -= L[i * RRS + k] * Q[k * RRS + j];
      Q[i * RRS + j] = z / L[i * RRS + i];
    }
  }
  __syncthreads();
  if (tid < R) {
    const int j = tid;  // column j of H' = L^-1 (row j of Z)^T
    for (int i = 0; i < R; ++i) {
      double z = Q[j * RRS + i];
      for (int k = 0; k < i; ++k) z -= L[i * RRS + k] * H[k * RRS + j];
      H[i * RRS + j] = z / L[i * RRS + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < R * R; e += 256) {  // symmetrise, eigenvectors start at I
    const int i = e / R, k = e - i * R;
    if (k < i) {
      const double v = 0.5 * (H[i * RRS + k] + H[k * RRS + i]);
      H[i * RRS + k] = v;
      H[k * RRS + i] = v;
    }
  }
  for (int e = tid; e < 64 * RRS; e += 256) Q[e] = 0.0;
  __syncthreads();
  for (int i = tid; i < R; i += 256) Q[i * RRS + i] = 1.0;
  __syncthreads();
  // cyclic Jacobi, round-robin pairs (index RP-1 fixed, the others rotate)
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) {
      double o = 0.0, d = 0.0;
      for (int i = 0; i < R; ++i)
        for (int k = 0; k < R; ++k) {
          const double v = H[i * RRS + k];
          if (i == k) d += v * v;
          else o += v * v;
        }
      offn = o;
      diagn = d;
    }
    __syncthreads();
    if (!(offn > 1e-30 * diagn)) break;
    for (int round = 0; round < RP - 1; ++round) {
      if (tid < RP / 2) {
        int p, q;
        if (tid == 0) {
          p = RP - 1;
          q = round;
        } else {
          p = (round + tid) % (RP - 1);
          q = (round - tid + RP - 1) % (RP - 1);
        }
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, s = 0.0;
        if (q < R) {
          const double apq = H[p * RRS + q];
          if (apq != 0.0) {
            const double theta = (H[q * RRS + q] - H[p * RRS + p]) / (2.0 * apq);
            // tan of the rotation angle, the smaller root; 1 / (2 theta) once theta^2
            // would overflow
            const double t = fabs(theta) > 1e150
                                 ? 0.5 / theta
                                 : (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            s = t * c;
          }
        }
        pr[tid] = p;
        qr[tid] = q;
        cs[tid] = c;
        sn[tid] = s;
      }
      __syncthreads();
      // rows: H <- J^T H
      for (int e = tid; e < (RP / 2) * R; e += 256) {
        const int w = e / R, k = e - w * R;
        const int p = pr[w], q = qr[w];
        if (q < R) {
          const double c = cs[w], s = sn[w];
          const double hp = H[p * RRS + k], hq = H[q * RRS + k];
          H[p * RRS + k] = c * hp - s * hq;
          H[q * RRS + k] = s * hp + c * hq;
        }
      }
      __syncthreads();
      // columns: H <- H J, eigenvectors Q <- Q J
      for (int e = tid; e < (RP / 2) * R; e += 256) {
        const int w = e / R, k = e - w * R;
        const int p = pr[w], q = qr[w];
        if (q < R) {
          const double c = cs[w], s = sn[w];
          const double hp = H[k * RRS + p], hq = H[k * RRS + q];
          H[k * RRS + p] = c * hp - s * hq;
          H[k * RRS + q] = s * hp + c * hq;
          const double vp = Q[k * RRS + p], vq = Q[k * RRS + q];
          Q[k * RRS + p] = c * vp - s * vq;
          Q[k * RRS + q] = s * vp + c * vq;
        }
      }
      __syncthreads();
    }
  }
  // decreasing order: rank of each eigenvalue (ties by index)
  if (tid < R) lam[tid] = H[tid * RRS + tid];
  __syncthreads();
  int pos = 0;
  if (tid < R) {
    const double v = lam[tid];
    for (int k = 0; k < R; ++k) pos += (lam[k] > v) || (lam[k] == v && k < tid);
  }
  __syncthreads();
  // T = L^-T Q (column j by thread j) written to its sorted position
  if (tid < R) {
    const int j = tid;
    double t[64];
    for (int i = R - 1; i >= 0; --i) {
      double z = Q[i * RRS + j];
      for (int k = i + 1; k < R; ++k) z -= L[k * RRS + i] * t[k];
      t[i] = z / L[i * RRS + i];
    }
    double sgn = 1.0;
    if (a.P) {
      double d = 0.0;
      for (int m = 0; m < R; ++m) d += t[m] * a.P[m * R + pos];  // the column it replaces
      sgn = d < 0.0 ? -1.0 : 1.0;
    }
    for (int i = 0; i < R; ++i) a.T[i * R + pos] = sgn * t[i];
    a.lam[pos] = lam[j];
  }
  if (tid == 0) {
    a.status[0] = bad;
    a.status[1] = sweep;
  }
}

hipError_t launch_rayleigh_ritz(const RRArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(k_rayleigh_ritz, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// max_j ||C_j - lam_j V_j|| / lam_0 (one workgroup); C = W V.
__global__ __launch_bounds__(256) void k_ritz_residual(const double* __restrict__ C,
                                                       const double* __restrict__ V,
                                                       const double* __restrict__ lam, int64_t rows,
                                                       int R, double* out) {
  __shared__ double red[256];
  double mx = 0.0;
  for (int j = 0; j < R; ++j) {
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += 256) {
      const double d = C[i * R + j] - lam[j] * V[i * R + j];
      s = fma(d, d, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    mx = fmax(mx, red[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const double l0 = fabs(lam[0]) > 0.0 ? fabs(lam[0]) : 1.0;
    *out = sqrt(mx) / l0;
  }
}

hipError_t launch_ritz_residual(const double* C, const double* V, const double* lam, int64_t rows,
                                int R, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_ritz_residual, dim3(1), dim3(256), 0, s, C, V, lam, rows, R, out);
  return hipGetLastError();
}

// Columns of V (rows x R): negate column j when its entry of largest magnitude (the
// first one on ties) is negative.  One workgroup per column.
__global__ __launch_bounds__(256) void k_sign_by_max(double* V, int64_t rows, int R) {
  __shared__ double bv[256];
  __shared__ int64_t bi[256];
  const int j = blockIdx.x;
  double best = -1.0;
  int64_t bidx = 0;
  for (int64_t i = threadIdx.x; i < rows; i += 256) {
    const double v = fabs(V[i * R + j]);
    if (v > best) {
      best = v;
      bidx = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = bidx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int64_t oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const bool neg = V[bi[0] * R + j] < 0.0;
  __syncthreads();
  if (neg)
    for (int64_t i = threadIdx.x; i < rows; i += 256) V[i * R + j] = -V[i * R + j];
}

hipError_t launch_sign_by_max(double* V, int64_t rows, int R, hipStream_t s) {
  hipLaunchKernelGGL(k_sign_by_max, dim3(R), dim3(256), 0, s, V, rows, R);
  return hipGetLastError();
}

// Y~[x][a][b] = Yp[x][a][b] + T1[x][a][b] + T2[x][b][a] (R x R trailing block):
// the first-order PP-Tucker combination, one of the two terms with its rank indices
// in the other order.  A null T1 or T2 is a term that is known to be zero.
__global__ __launch_bounds__(256) void k_pp_tucker_combine(double* out, const double* Yp,
                                                           const double* T1, const double* T2,
                                                           int64_t rows, int R) {
  const int64_t n = rows * R * R;
  const int64_t RR = (int64_t)R * R;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t x = e / RR, r = e - x * RR;
    const int64_t a = r / R, b = r - a * R;
    double v = Yp[e];
    if (T1) v += T1[e];
    if (T2) v += T2[x * RR + b * R + a];
    out[e] = v;
  }
}

// out[i][j] = in[i][j] / lam[j] (columns with lam[j] = 0 are copied).
__global__ __launch_bounds__(256) void k_scale_cols(double* out, const double* in,
                                                    const double* lam, int64_t rows, int R) {
  const int64_t n = rows * R;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const double l = lam[e % R];
    out[e] = l != 0.0 ? in[e] / l : in[e];
  }
}

hipError_t launch_scale_cols(double* out, const double* in, const double* lam, int64_t rows, int R,
                             hipStream_t s) {
  int64_t blocks = (rows * R + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0, s,
                     out, in, lam, rows, R);
  return hipGetLastError();
}

hipError_t launch_pp_tucker_combine(double* out, const double* Yp, const double* T1,
                                    const double* T2, int64_t rows, int R, hipStream_t s) {
  const int64_t n = rows * (int64_t)R * R;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_pp_tucker_combine, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0,
                     s, out, Yp, T1, T2, rows, R);
  return hipGetLastError();
}

// Core statistics: out[0] = ||Gn||^2, out[1] = ||Gn - Go||^2 (one workgroup).
__global__ __launch_bounds__(256) void k_core_stats(const double* Gn, const double* Go, int64_t n,
                                                    double* out) {
  __shared__ double r0[256], r1[256];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double g = Gn[i];
    const double d = g - Go[i];
    a = fma(g, g, a);
    b = fma(d, d, b);
  }
  r0[threadIdx.x] = a;
  r1[threadIdx.x] = b;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      r0[threadIdx.x] += r0[threadIdx.x + w];
      r1[threadIdx.x] += r1[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = r0[0];
    out[1] = r1[0];
  }
}

hipError_t launch_core_stats(const double* Gn, const double* Go, int64_t n, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_core_stats, dim3(1), dim3(256), 0, s, Gn, Go, n, out);
  return hipGetLastError();
}

}  // namespace ppk
