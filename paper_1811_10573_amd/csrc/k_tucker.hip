// Kernels of the Tucker-ALS and PP-Tucker-ALS path (Algorithms 2 and 4), FP64:
//
//  * a strided, split-K, batched FP64 GEMM for the small products of the subspace
//    iteration (V^T V, V^T W V, V^T A_prev);
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
// 64 x 64 tiles, 256 threads with 4 x 4 outputs each, K in chunks of 16 through LDS;
// workgroup z takes the z-th of ks consecutive K ranges.  A tile is read with the
// operand's unit-stride index fastest across threads.
// ---------------------------------------------------------------------------
constexpr int GT = 64, GK = 16;

__global__ __launch_bounds__(256) void k_gemm_f64(GemmArgs g, int64_t kchunk, int nz) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  const int tid = threadIdx.x;
  const int64_t m0 = (int64_t)blockIdx.y * GT, n0 = (int64_t)blockIdx.x * GT;
  const int split = (int)blockIdx.z % nz, batch = (int)blockIdx.z / nz;
  const double* Bp = g.B + batch * g.sbb;
  const int64_t kbeg = (int64_t)split * kchunk;
  const int64_t kend = kbeg + kchunk < g.K ? kbeg + kchunk : g.K;
  const int tm = (tid / 16) * 4, tn = (tid % 16) * 4;
  const bool a_kfast = g.sak == 1;
  const bool b_kfast = g.sbk == 1;
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
      As[kk][mm] = (m < g.M && k < kend) ? g.A[m * g.sam + k * g.sak] : 0.0;
    }
    for (int e = tid; e < GK * GT; e += 256) {
      const int kk = b_kfast ? e % GK : e / GT;
      const int nn = b_kfast ? e / GK : e % GT;
      const int64_t n = n0 + nn, k = k0 + kk;
      Bs[kk][nn] = (n < g.N && k < kend) ? Bp[k * g.sbk + n * g.sbn] : 0.0;
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
  double* C = g.ks > 1 ? g.part + ((int64_t)split * g.nb + batch) * g.M * g.N
                       : g.C + batch * g.M * g.N;
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
  if (g.nb < 1 || (g.ks > 1 && (g.alpha != 1.0 || g.beta != 0.0 || !g.part)) ||
      ((g.ks > 1 || g.nb > 1) && g.ldc != g.N))
    return hipErrorInvalidValue;
  const int ks = g.ks > 1 ? g.ks : 1;
  int64_t kchunk = (g.K + ks - 1) / ks;
  kchunk = (kchunk + GK - 1) / GK * GK;
  // splits that hold k-values (at most ks after the rounding of kchunk)
  const int nz = g.K > 0 ? (int)((g.K + kchunk - 1) / kchunk) : 1;
  const dim3 grid((unsigned)((g.N + GT - 1) / GT), (unsigned)((g.M + GT - 1) / GT),
                  (unsigned)(nz * g.nb));
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(256), 0, s, g, g.K > 0 ? kchunk : (int64_t)0, nz);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || ks == 1) return e;
  return launch_reduce_splits_to(g.C, 0, g.part, 0, nz, g.nb * g.M * g.N, s);
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz step (one workgroup, R <= 64).  With V the current basis (s x R),
// B = V^T V and H = V^T W V: L = chol(B), H' = L^-1 H L^-T, H' = Q diag(lam) Q^T by
// cyclic Jacobi rotations (parallel round-robin pairing), decreasing lam, and
// T = L^-T Q, so that V T are orthonormal Ritz vectors.  With P = V^T A_prev, column j
// of T is negated when (V T)_j . A_prev_j = (T^T P)_jj < 0.
//
// The Cholesky factorisation takes one barrier per column (the trailing update reads
// the unscaled pivot column while the scaled column goes to a second array), L^-1 is
// formed column by column by quads of lanes, and the three products with L^-1 are
// dense LDS products with 2 x 2 register blocks.
// ---------------------------------------------------------------------------
// The R x R arrays of the kernels below have row stride RM + 1: 65 for R <= 64, 17 in the
// small-rank kernel.

// out[a][b] = sum_k X(a, k) Y(k, b) for a, b < R with X(a, k) = Xs[a * xa + k * xk] and
// Y(k, b) = Ys[k * yk + b * yb]; 2 x 2 outputs per thread of NT; out has row stride LS.
template <int LS, int NT>
__device__ __forceinline__ void rr_product(double* out, const double* Xs, int xa, int xk,
                                           const double* Ys, int yk, int yb, int R) {
  const int Rh = (R + 1) / 2;
  for (int e = threadIdx.x; e < Rh * Rh; e += NT) {
    const int a0 = 2 * (e / Rh), b0 = 2 * (e % Rh);
    const int a1 = a0 + 1 < R ? a0 + 1 : a0, b1 = b0 + 1 < R ? b0 + 1 : b0;
    double c00 = 0.0, c01 = 0.0, c10 = 0.0, c11 = 0.0;
    for (int k = 0; k < R; ++k) {
      const double x0 = Xs[a0 * xa + k * xk], x1 = Xs[a1 * xa + k * xk];
      const double y0 = Ys[k * yk + b0 * yb], y1 = Ys[k * yk + b1 * yb];
      c00 = fma(x0, y0, c00);
      c01 = fma(x0, y1, c01);
      c10 = fma(x1, y0, c10);
      c11 = fma(x1, y1, c11);
    }
    out[a0 * LS + b0] = c00;
    if (b1 != b0) out[a0 * LS + b1] = c01;
    if (a1 != a0) out[a1 * LS + b0] = c10;
    if (a1 != a0 && b1 != b0) out[a1 * LS + b1] = c11;
  }
}

// Barrier of the NT threads that run the Rayleigh-Ritz algebra: the workgroup (256), or one
// wave (64), whose LDS operations complete in program order.
template <int NT>
__device__ __forceinline__ void rr_sync() {
  if (NT == 64) __builtin_amdgcn_wave_barrier();
  else __syncthreads();
}

// Sum of v over the NT threads (four waves, or one); every thread gets the total.
template <int NT>
__device__ __forceinline__ double rr_block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if (NT == 64) return v;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = (red[0] + red[1]) + (red[2] + red[3]);
  __syncthreads();
  return t;
}

// Maximum of v over the NT threads; every thread gets it.
template <int NT>
__device__ __forceinline__ double rr_block_max(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if (NT == 64) return v;
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  const double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
  __syncthreads();
  return t;
}

// Below this max |B - I| the inverse square root series replaces the Cholesky factor.
constexpr double kRRSeriesTol = 1e-6;

// dst[e] = src[e] for e < n into LDS, eight loads in flight per thread before the stores.
__device__ __forceinline__ void stage_rows(double* dst, const double* __restrict__ src, int n) {
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      v[q] = e < n ? src[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      if (e < n) dst[e] = v[q];
    }
  }
}

// o1 = X^T Y1 and (Y2 non-null) o2 = X^T Y2 for rows x R matrices held in LDS (row stride
// R), into LDS arrays of row stride LS.  With G the largest power of two with G R^2 <= 256
// (at least 1), thread t sums entry t % R^2 over the rows x = t / R^2 (mod G) in increasing
// order and the G partial sums are added in group order (through red, 256 doubles); with
// G = 1 a thread sums up to 16 entries.
template <int LS>
__device__ __forceinline__ void rr_project(const double* Xs, const double* Y1s, const double* Y2s,
                                           int rows, int R, double* red, double* o1, double* o2) {
  constexpr int NE = 16;  // entries per thread (R^2 <= 4096)
  const int tid = threadIdx.x;
  const int RR = R * R;
  int G = 1;
  while (2 * G * RR <= 256) G *= 2;
  const int grp = G > 1 ? tid / RR : 0;
  const int nent = G > 1 ? (tid < G * RR ? 1 : 0) : NE;
  double acc1[NE], acc2[NE];
#pragma unroll
  for (int u = 0; u < NE; ++u) acc1[u] = acc2[u] = 0.0;
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = G > 1 ? tid - grp * RR : tid + 256 * u;
    if (u < nent && e < RR) {
      const int i = e / R, k = e - i * R;
      double s1 = 0.0, s2 = 0.0;
      int x = grp;
      for (; x + 3 * G < rows; x += 4 * G) {
        double xv[4], y1[4], y2[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          xv[v] = Xs[(x + v * G) * R + i];
          y1[v] = Y1s[(x + v * G) * R + k];
          y2[v] = Y2s ? Y2s[(x + v * G) * R + k] : 0.0;
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          s1 = fma(xv[v], y1[v], s1);
          if (Y2s) s2 = fma(xv[v], y2[v], s2);
        }
      }
      for (; x < rows; x += G) {
        const double xv = Xs[x * R + i];
        s1 = fma(xv, Y1s[x * R + k], s1);
        if (Y2s) s2 = fma(xv, Y2s[x * R + k], s2);
      }
      acc1[u] = s1;
      acc2[u] = s2;
    }
  }
  if (G > 1) {
    for (int pass = 0; pass < (Y2s ? 2 : 1); ++pass) {
      if (tid < G * RR) red[tid] = pass ? acc2[0] : acc1[0];
      __syncthreads();
      if (tid < RR) {
        double s = 0.0;
        for (int q = 0; q < G; ++q) s += red[q * RR + tid];
        const int i = tid / R, k = tid - i * R;
        (pass ? o2 : o1)[i * LS + k] = s;
      }
      __syncthreads();
    }
    return;
  }
#pragma unroll
  for (int u = 0; u < NE; ++u) {
    const int e = tid + 256 * u;
    if (e < RR) {
      const int i = e / R, k = e - i * R;
      o1[i * LS + k] = acc1[u];
      if (Y2s) o2[i * LS + k] = acc2[u];
    }
  }
}

// The Rayleigh-Ritz algebra on R x R arrays of row stride LS = RM + 1, with B in L, H in H
// and Lc, Li zero: leaves T = L^-T Q (columns in Jacobi order) in L, the Ritz values in
// lam and Q in Lc; *bad = 1 when B was not positive definite.  Returns the Jacobi sweeps.
template <int RM, int NT>
__device__ __forceinline__ int rr_core(int R, double* L, double* Lc, double* Li, double* H,
                                       double* lam, double* cs, double* sn, int* pr, int* qr,
                                       double* red, int* bad) {
  constexpr int LS = RM + 1;
  static_assert(NT == 256 || (NT == 64 && RM <= 16), "four waves, or one wave for R <= 16");
  const int tid = threadIdx.x;
  const int RP = R + (R & 1);  // even, for the round-robin pairing
  double em = 0.0;
  for (int e = tid; e < R * R; e += NT) {
    const int i = e / R, k = e - i * R;
    em = fmax(em, fabs(L[i * LS + k] - (i == k ? 1.0 : 0.0)));
  }
  em = rr_block_max<NT>(em, red);
  if (em < kRRSeriesTol) {
    // V is orthonormal up to E = B - I: Li = B^-1/2 = I - E/2 + 3/8 E^2 - 5/16 E^3 (the
    // next term is O(|E|^4) < 1e-22 R^4), symmetric, so that Li B Li^T = I as with the
    // Cholesky factor below.  Horner form: Li = I + E (-I/2 + E (3/8 I - 5/16 E)).
    for (int e = tid; e < R * R; e += NT) {
      const int i = e / R, k = e - i * R;
      const double ev = L[i * LS + k] - (i == k ? 1.0 : 0.0);
      L[i * LS + k] = ev;
      Li[i * LS + k] = (i == k ? 0.375 : 0.0) - 0.3125 * ev;
    }
    rr_sync<NT>();
    rr_product<LS, NT>(Lc, L, LS, 1, Li, LS, 1, R);
    rr_sync<NT>();
    for (int i = tid; i < R; i += NT) Lc[i * LS + i] -= 0.5;
    rr_sync<NT>();
    rr_product<LS, NT>(Li, L, LS, 1, Lc, LS, 1, R);
    rr_sync<NT>();
    for (int i = tid; i < R; i += NT) Li[i * LS + i] += 1.0;
    rr_sync<NT>();
  } else {
  // Cholesky of B: Lc = L with L L^T = B (lower)
  for (int j = 0; j < R; ++j) {
    const double d0 = L[j * LS + j];
    const bool ok = d0 > 0.0 && isfinite(d0);
    if (tid == 0 && !ok) *bad = 1;
    const double d = ok ? d0 : 1.0;
    const double inv_sd = 1.0 / sqrt(d);
    const double inv_d = 1.0 / d;
    const int m = R - j - 1;
    for (int e = tid; e < m * m; e += NT) {
      const int ii = e / m, kk = e - ii * m;
      if (kk <= ii) {
        const int i = j + 1 + ii, k = j + 1 + kk;
        L[i * LS + k] -= L[i * LS + j] * L[k * LS + j] * inv_d;
      }
    }
    for (int i = j + tid; i < R; i += NT) Lc[i * LS + j] = (i == j) ? sqrt(d) : L[i * LS + j] * inv_sd;
    rr_sync<NT>();
  }
  // Li = Lc^-1, column j by the quad of lanes 4j..4j+3 (k split by k mod 4)
  {
    const int j = tid >> 2, l = tid & 3;
    if (j < R) {
      if (l == 0) Li[j * LS + j] = 1.0 / Lc[j * LS + j];
      for (int i = j + 1; i < R; ++i) {
        double s = 0.0;
        for (int k = j + l; k < i; k += 4) s = fma(Lc[i * LS + k], Li[k * LS + j], s);
        s += __shfl_xor(s, 1);
        s += __shfl_xor(s, 2);
        // every lane of the quad has the sum; lane (i - j) mod 4 stores it and is the only
        // lane that reads it again (k - j = l mod 4 above), later in program order
        if (l == ((i - j) & 3)) Li[i * LS + j] = -s / Lc[i * LS + i];
      }
    }
  }
  rr_sync<NT>();
  }
  // H' = Li H Li^T: Z = Li H into L, then H = Z Li^T
  rr_product<LS, NT>(L, Li, LS, 1, H, LS, 1, R);
  rr_sync<NT>();
  rr_product<LS, NT>(H, L, LS, 1, Li, 1, LS, R);
  rr_sync<NT>();
  for (int e = tid; e < R * R; e += NT) {  // symmetrise; eigenvectors start at I
    const int i = e / R, k = e - i * R;
    if (k < i) {
      const double v = 0.5 * (H[i * LS + k] + H[k * LS + i]);
      H[i * LS + k] = v;
      H[k * LS + i] = v;
    }
  }
  for (int e = tid; e < RM * LS; e += NT) Lc[e] = 0.0;
  rr_sync<NT>();
  double* Q = Lc;
  for (int i = tid; i < R; i += NT) Q[i * LS + i] = 1.0;
  rr_sync<NT>();
  // cyclic Jacobi, round-robin pairs (index RP-1 fixed, the others rotate)
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    double o = 0.0, dg = 0.0;
    for (int e = tid; e < R * R; e += NT) {
      const int i = e / R, k = e - i * R;
      const double v = H[i * LS + k];
      if (i == k) dg = fma(v, v, dg);
      else o = fma(v, v, o);
    }
    const double offn = rr_block_sum<NT>(o, red);
    const double diagn = rr_block_sum<NT>(dg, red);
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
          const double apq = H[p * LS + q];
          if (apq != 0.0) {
            const double theta = (H[q * LS + q] - H[p * LS + p]) / (2.0 * apq);
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
      rr_sync<NT>();
      // H <- J^T H J one 2 x 2 block (rows of pair w1, columns of pair w2) per step: the
      // pairs of a round partition the indices, so the blocks are disjoint.  A pair whose
      // partner is the padding index R has a single row or column.
      const int np = RP / 2;
      for (int e = tid; e < np * np; e += NT) {
        const int w1 = e / np, w2 = e - w1 * np;
        const double s1 = sn[w1], s2 = sn[w2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const double c1 = cs[w1], c2 = cs[w2];
        const int p1 = pr[w1], q1 = qr[w1], p2 = pr[w2], q2 = qr[w2];
        const bool r1 = q1 < R, r2 = q2 < R;
        const double hpp = H[p1 * LS + p2];
        const double hpq = r2 ? H[p1 * LS + q2] : 0.0;
        const double hqp = r1 ? H[q1 * LS + p2] : 0.0;
        const double hqq = (r1 && r2) ? H[q1 * LS + q2] : 0.0;
        // rows: p' = c1 p - s1 q, q' = s1 p + c1 q
        const double app = c1 * hpp - s1 * hqp, apq = c1 * hpq - s1 * hqq;
        const double aqp = s1 * hpp + c1 * hqp, aqq = s1 * hpq + c1 * hqq;
        // columns: p' = c2 p - s2 q, q' = s2 p + c2 q
        H[p1 * LS + p2] = c2 * app - s2 * apq;
        if (r2) H[p1 * LS + q2] = s2 * app + c2 * apq;
        if (r1) H[q1 * LS + p2] = c2 * aqp - s2 * aqq;
        if (r1 && r2) H[q1 * LS + q2] = s2 * aqp + c2 * aqq;
      }
      // eigenvectors Q <- Q J
      for (int e = tid; e < np * R; e += NT) {
        const int k = e / np, w = e - k * np;
        const double s = sn[w];
        if (s != 0.0) {
          const int p = pr[w], q = qr[w];
          const double c = cs[w];
          const double vp = Q[k * LS + p], vq = Q[k * LS + q];
          Q[k * LS + p] = c * vp - s * vq;
          Q[k * LS + q] = s * vp + c * vq;
        }
      }
      rr_sync<NT>();
    }
  }
  // T = Li^T Q into L
  if (tid < R) lam[tid] = H[tid * LS + tid];
  rr_product<LS, NT>(L, Li, 1, LS, Q, LS, 1, R);
  rr_sync<NT>();
  return sweep;
}

__global__ __launch_bounds__(256) void k_rayleigh_ritz(RRArgs a) {
  constexpr int RM = 64, LS = RM + 1;
  __shared__ double L[RM * LS];   // B, trailing updates; later scratch (Z, T)
  __shared__ double Lc[RM * LS];  // Cholesky factor; later the Jacobi eigenvectors
  __shared__ double Li[RM * LS];  // L^-1 (lower)
  __shared__ double H[RM * LS];   // H, then H' (rotated in place)
  __shared__ double lam[RM];
  __shared__ double cs[RM / 2], sn[RM / 2];
  __shared__ int pr[RM / 2], qr[RM / 2];
  __shared__ double red[4];
  __shared__ int bad;
  const int tid = threadIdx.x;
  const int R = a.R;
  for (int e = tid; e < RM * LS; e += 256) {
    Lc[e] = 0.0;
    Li[e] = 0.0;
  }
  for (int e = tid; e < R * R; e += 256) {
    const int i = e / R, k = e - i * R;
    L[i * LS + k] = a.B[e];
    H[i * LS + k] = a.H[e];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  const int sweep = rr_core<RM, 256>(R, L, Lc, Li, H, lam, cs, sn, pr, qr, red, &bad);
  // decreasing order (ties by index), sign against A_prev, written to sorted position
  if (tid < R) {
    const int j = tid;
    const double v = lam[j];
    int pos = 0;
    for (int k = 0; k < R; ++k) pos += (lam[k] > v) || (lam[k] == v && k < j);
    double sgn = 1.0;
    if (a.P) {
      double d = 0.0;
      for (int m = 0; m < R; ++m) d = fma(L[m * LS + j], a.P[m * R + pos], d);  // the column it replaces
      sgn = d < 0.0 ? -1.0 : 1.0;
    }
    for (int i = 0; i < R; ++i) a.T[i * R + pos] = sgn * L[i * LS + j];
    a.lam[pos] = v;
  }
  if (tid == 0) {
    a.status[0] = bad;
    a.status[1] = sweep;
  }
}

hipError_t launch_rayleigh_ritz(const RRArgs& a, hipStream_t s) {
  if (a.R < 1 || a.R > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_rayleigh_ritz, dim3(1), dim3(256), 0, s, a);
  return hipGetLastError();
}

// dst[e] = sum_{c < np} src[c * stride + e] for e < n into LDS, slots added in order: each
// thread issues the loads of SB slots of EB elements before adding them.
template <int EB, int SB>
__device__ __forceinline__ void stage_sum_t(double* dst, const double* __restrict__ src, int np,
                                            int64_t stride, int n) {
  for (int e0 = threadIdx.x; e0 < n; e0 += EB * 256) {
    double acc[EB];
#pragma unroll
    for (int b = 0; b < EB; ++b) acc[b] = 0.0;
    for (int c0 = 0; c0 < np; c0 += SB) {
      double v[EB][SB];
#pragma unroll
      for (int b = 0; b < EB; ++b)
#pragma unroll
        for (int q = 0; q < SB; ++q) {
          const int e = e0 + 256 * b, c = c0 + q;
          v[b][q] = (e < n && c < np) ? src[c * stride + e] : 0.0;
        }
#pragma unroll
      for (int b = 0; b < EB; ++b)
#pragma unroll
        for (int q = 0; q < SB; ++q)
          if (c0 + q < np) acc[b] += v[b][q];
    }
#pragma unroll
    for (int b = 0; b < EB; ++b) {
      const int e = e0 + 256 * b;
      if (e < n) dst[e] = acc[b];
    }
  }
}

// stage_sum_t with the shape that needs the fewest rounds of loads (uniform choice)
__device__ __forceinline__ void stage_sum(double* dst, const double* __restrict__ src, int np,
                                          int64_t stride, int n) {
  auto rounds = [&](int eb, int sb) { return ((n + 256 * eb - 1) / (256 * eb)) * ((np + sb - 1) / sb); };
  if (rounds(2, 16) <= rounds(8, 8)) stage_sum_t<2, 16>(dst, src, np, stride, n);
  else stage_sum_t<8, 8>(dst, src, np, stride, n);
}

// dst1[e] = src1[e] and (src2 non-null) dst2[e] = src2[e] for e < n into LDS, sixteen loads
// in flight per thread before the stores.
__device__ __forceinline__ void stage_two(double* dst1, const double* __restrict__ src1,
                                          double* dst2, const double* __restrict__ src2, int n) {
  for (int e0 = threadIdx.x; e0 < n; e0 += 8 * 256) {
    double v[8], w[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      v[q] = e < n ? src1[e] : 0.0;
      w[q] = (src2 && e < n) ? src2[e] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      if (e < n) {
        dst1[e] = v[q];
        if (src2) dst2[e] = w[q];
      }
    }
  }
}

// The whole subspace step after C = W V for R <= 16 in one workgroup, with V, C and A_prev
// resident in LDS (rows x R each, at most kRRSmallElems): C is the sum of npart partial
// slots in slot order (or C itself), then the projections, the Rayleigh-Ritz algebra, the
// sorted and signed T and lam, and the Ritz update: U = V T, V <- C T diag(lam)^-1 and
// *residual = max_j ||C T_j - lam_j U_j|| / |lam_0| (column sums of squares by interleaved
// row groups added in group order).
__global__ __launch_bounds__(256) void k_rr_small(RRArgs a) {
  constexpr int RM = 16, LS = RM + 1;
  __shared__ double L[RM * LS], Lc[RM * LS], Li[RM * LS], H[RM * LS], P[RM * LS], Tf[RM * LS];
  __shared__ double lam[RM], lams[RM];
  __shared__ double cs[RM / 2], sn[RM / 2];
  __shared__ int pr[RM / 2], qr[RM / 2];
  __shared__ double red[256];
  __shared__ int bad;
  extern __shared__ double dyn[];
  const int tid = threadIdx.x;
  const int R = a.R;
  const int rows = (int)a.rows;
  const int n = rows * R;
  double* Vs = dyn;
  double* Cs = Vs + n;
  double* As = Cs + n;
  if (a.cpart) {
    stage_sum(Cs, a.cpart, a.npart, a.pstride, n);
    stage_two(Vs, a.V, As, a.Ap, n);
  } else {
    stage_two(Vs, a.V, Cs, a.C, n);
    if (a.Ap) stage_rows(As, a.Ap, n);
  }
  for (int e = tid; e < RM * LS; e += 256) {
    Lc[e] = 0.0;
    Li[e] = 0.0;
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  rr_project<LS>(Vs, Vs, Cs, rows, R, red, L, H);
  if (a.Ap) rr_project<LS>(Vs, As, nullptr, rows, R, red, P, nullptr);
  __syncthreads();
  // the algebra in wave 0 (R <= 16: no workgroup barriers), the other waves wait
  int sweep = 0;
  if (tid < 64) sweep = rr_core<RM, 64>(R, L, Lc, Li, H, lam, cs, sn, pr, qr, red, &bad);
  __syncthreads();
  if (tid < R) {
    const int j = tid;
    const double v = lam[j];
    int pos = 0;
    for (int k = 0; k < R; ++k) pos += (lam[k] > v) || (lam[k] == v && k < j);
    double sgn = 1.0;
    if (a.Ap) {
      double d = 0.0;
      for (int m = 0; m < R; ++m) d = fma(L[m * LS + j], P[m * LS + pos], d);
      sgn = d < 0.0 ? -1.0 : 1.0;
    }
    for (int i = 0; i < R; ++i) {
      const double t = sgn * L[i * LS + j];
      Tf[i * LS + pos] = t;
      a.T[i * R + pos] = t;
    }
    lams[pos] = v;
    a.lam[pos] = v;
  }
  if (tid == 0) {
    a.status[0] = bad;
    a.status[1] = sweep;
  }
  __syncthreads();
  double* D = As;  // A_prev is no longer needed
  for (int e = tid; e < n; e += 256) {
    const int x = e / R, j = e - x * R;
    double u = 0.0, ct = 0.0;
    for (int m = 0; m < R; ++m) {
      const double t = Tf[m * LS + j];
      u = fma(Vs[x * R + m], t, u);
      ct = fma(Cs[x * R + m], t, ct);
    }
    const double d = ct - lams[j] * u;
    D[e] = d * d;
    a.U[e] = u;
    a.Vout[e] = lams[j] != 0.0 ? ct / lams[j] : ct;
  }
  __syncthreads();
  const int G = 256 / R;
  const int g = tid / R, j = tid - g * R;
  double s = 0.0;
  if (g < G)
    for (int x = g; x < rows; x += G) s += D[x * R + j];
  red[tid] = s;
  __syncthreads();
  if (tid == 0) {
    double mx = 0.0;
    for (int jj = 0; jj < R; ++jj) {
      double t = 0.0;
      for (int q = 0; q < G; ++q) t += red[q * R + jj];
      mx = fmax(mx, sqrt(t));
    }
    const double l0 = fabs(lams[0]) > 0.0 ? fabs(lams[0]) : 1.0;
    *a.residual = mx / l0;
  }
}

bool rr_small_fits(int64_t rows, int R) { return R >= 1 && R <= 16 && rows * R <= kRRSmallElems; }

hipError_t launch_rr_small(const RRArgs& a, hipStream_t s) {
  if (!rr_small_fits(a.rows, a.R) || !a.V || !a.Vout || !a.U || !a.residual || (!a.C && !a.cpart) ||
      (a.cpart && (a.npart < 1 || a.npart > kRRSmallParts)))
    return hipErrorInvalidValue;
  const size_t lds = (size_t)3 * a.rows * a.R * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_rr_small),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_rr_small, dim3(1), dim3(256), lds, s, a);
  return hipGetLastError();
}

// Ritz update over a block of RU rows: U = V T (the Ritz vectors), CT = C T (W applied
// to them), the per-column partial sums of ||CT_j - lam_j U_j||^2 into part[block][j],
// and V <- CT diag(lam)^-1 (the next basis; columns with lam_j = 0 keep CT_j).
constexpr int RU = 32;

__global__ __launch_bounds__(256) void k_ritz_update(double* V, const double* C, const double* T,
                                                     const double* lam, double* U, double* part,
                                                     int64_t rows, int R) {
  __shared__ double Ts[64 * 64];
  __shared__ double Vs[RU * 65], Cs[RU * 65], D[RU * 65];
  __shared__ double ls[64];
  const int tid = threadIdx.x;
  const int64_t r0 = (int64_t)blockIdx.x * RU;
  const int nr = (int)((rows - r0) < RU ? (rows - r0) : RU);
  for (int e = tid; e < R * R; e += 256) Ts[e] = T[e];
  if (tid < R) ls[tid] = lam[tid];
  for (int e = tid; e < RU * R; e += 256) {
    const int i = e / R, j = e - i * R;
    const bool ok = i < nr;
    Vs[i * 65 + j] = ok ? V[(r0 + i) * R + j] : 0.0;
    Cs[i * 65 + j] = ok ? C[(r0 + i) * R + j] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < RU * R; e += 256) {
    const int i = e / R, j = e - i * R;
    double u = 0.0, ct = 0.0;
    for (int m = 0; m < R; ++m) {
      const double t = Ts[m * R + j];
      u = fma(Vs[i * 65 + m], t, u);
      ct = fma(Cs[i * 65 + m], t, ct);
    }
    const double d = ct - ls[j] * u;
    D[i * 65 + j] = i < nr ? d * d : 0.0;
    if (i < nr) {
      U[(r0 + i) * R + j] = u;
      V[(r0 + i) * R + j] = ls[j] != 0.0 ? ct / ls[j] : ct;
    }
  }
  __syncthreads();
  if (tid < R) {
    double s = 0.0;
    for (int i = 0; i < RU; ++i) s += D[i * 65 + tid];
    part[(int64_t)blockIdx.x * R + tid] = s;
  }
}

// max_j sqrt(sum_b part[b][j]) / |lam_0| (one workgroup, blocks in a fixed order).
__global__ __launch_bounds__(64) void k_ritz_residual(const double* part, int nblocks, int R,
                                                      const double* lam, double* out) {
  const int j = threadIdx.x;
  double s = 0.0;
  if (j < R)
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * R + j];
  double m = j < R ? sqrt(s) : 0.0;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
  if (j == 0) {
    const double l0 = fabs(lam[0]) > 0.0 ? fabs(lam[0]) : 1.0;
    *out = m / l0;
  }
}

hipError_t launch_ritz_update(double* V, const double* C, const double* T, const double* lam,
                              double* U, double* part, int64_t rows, int R, double* residual,
                              hipStream_t s) {
  if (R < 1 || R > 64) return hipErrorInvalidValue;
  const int nb = (int)((rows + RU - 1) / RU);
  hipLaunchKernelGGL(k_ritz_update, dim3(nb), dim3(256), 0, s, V, C, T, lam, U, part, rows, R);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ritz_residual, dim3(1), dim3(64), 0, s, part, nb, R, lam, residual);
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

// PP-Tucker combination (Section 3.2.2): out[x][c] = base[x][c] + sum_t term_t[x][p_t(c)].
// c runs over the rank multi-index of a TTMc in canonical order (the rank indices of the
// other modes in increasing mode order, nd digits base R, the first most significant);
// a first-order term contracts its mode last, so its rank digit is the last one there:
// p_t moves digit pos_t of c to the end.
__global__ __launch_bounds__(256) void k_tucker_combine(TuckerCombine a) {
  const int64_t n = a.rows * a.cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < n; e += (int64_t)gridDim.x * 256) {
    const int64_t x = e / a.cols, c = e - x * a.cols;
    double v = a.base ? a.base[e] : 0.0;
    for (int t = 0; t < a.nterms; ++t) {
      const int64_t w = a.rpow[a.nd - 1 - a.pos[t]];  // weight of the moved digit
      const int64_t high = c / (w * a.R);
      const int64_t rem = c - high * w * a.R;
      const int64_t dp = rem / w;
      const int64_t low = rem - dp * w;
      v += a.term[t][x * a.cols + (high * w + low) * a.R + dp];
    }
    a.out[e] = v;
  }
}

hipError_t launch_tucker_combine(const TuckerCombine& a, hipStream_t s) {
  const int64_t n = a.rows * a.cols;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(k_tucker_combine, dim3((unsigned)std::max<int64_t>(1, blocks)), dim3(256), 0,
                     s, a);
  return hipGetLastError();
}

// k_tucker_combine with each term's contraction done in place (small operators): G lanes
// (a power of two <= 16, within one wave) take one output element; lane q sums the
// contracted indices k = q, q + G, .. in increasing order, the G partial sums are added
// by butterfly shuffles, and the terms are added to the base in term order.
__global__ __launch_bounds__(256) void k_tucker_pp_rhs(TuckerPPRhs a, int G) {
  const int64_t n = a.rows * a.cols;
  const int64_t gt = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t e = gt / G;
  const int q = (int)(gt - e * G);
  const bool valid = e < n;
  const int64_t ee = valid ? e : 0;
  const int64_t x = ee / a.cols, c = ee - x * a.cols;
  double v = (valid && a.base) ? a.base[ee] : 0.0;
  for (int t = 0; t < a.nterms; ++t) {
    const int64_t w = a.rpow[a.nd - 1 - a.pos[t]];  // weight of the contracted rank digit
    const int64_t high = c / (w * a.R);
    const int64_t rem = c - high * w * a.R;
    const int64_t r = rem / w;
    const int64_t rest = high * w + (rem - r * w);
    const double* o = a.op[t] + x * a.nstride[t] + rest;
    const double* f = a.F[t] + r;
    const int64_t ks = a.kstride[t] * G, len = valid ? a.klen[t] : 0;
    const int64_t fs = (int64_t)a.R * G;
    o += q * a.kstride[t];
    f += (int64_t)q * a.R;
    double acc = 0.0;
    int64_t k = q;
    for (; k + 3 * G < len; k += 4 * G) {
      const double o0 = o[0], o1 = o[ks], o2 = o[2 * ks], o3 = o[3 * ks];
      const double f0 = f[0], f1 = f[fs], f2 = f[2 * fs], f3 = f[3 * fs];
      acc = fma(o0, f0, acc);
      acc = fma(o1, f1, acc);
      acc = fma(o2, f2, acc);
      acc = fma(o3, f3, acc);
      o += 4 * ks;
      f += 4 * fs;
    }
    for (; k < len; k += G) {
      acc = fma(o[0], f[0], acc);
      o += ks;
      f += fs;
    }
    for (int off = G >> 1; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
    v += acc;
  }
  if (valid && q == 0) a.out[ee] = v;
}

int pp_rhs_lanes(int64_t elems) {
  int G = 1;
  while (G < 16 && elems * G < 98304) G *= 2;
  return G;
}

hipError_t launch_tucker_pp_rhs(const TuckerPPRhs& a, hipStream_t s) {
  const int64_t n = a.rows * a.cols;
  const int G = pp_rhs_lanes(n);
  const int64_t blocks = (n * G + 255) / 256;
  if (blocks < 1 || blocks > 0x7fffffff) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tucker_pp_rhs, dim3((unsigned)blocks), dim3(256), 0, s, a, G);
  return hipGetLastError();
}

// Norm statistics: out[0] = ||Gn||^2, out[1] = ||Gn - Go||^2 (one workgroup of 1024
// threads, two elements per thread and step; a fixed reduction order).
__global__ __launch_bounds__(1024) void k_core_stats(const double* Gn, const double* Go, int64_t n,
                                                     double* out) {
  __shared__ double r0[16], r1[16];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 2048) {
    const double g0 = Gn[i], d0 = g0 - Go[i];
    double g1 = 0.0, d1 = 0.0;
    if (i + 1024 < n) {
      g1 = Gn[i + 1024];
      d1 = g1 - Go[i + 1024];
    }
    a = fma(g0, g0, fma(g1, g1, a));
    b = fma(d0, d0, fma(d1, d1, b));
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = a;
    r1[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < 16; ++w) {
      sa += r0[w];
      sb += r1[w];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

hipError_t launch_core_stats(const double* Gn, const double* Go, int64_t n, double* out,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_core_stats, dim3(1), dim3(1024), 0, s, Gn, Go, n, out);
  return hipGetLastError();
}

// k_core_stats on (U, Ap) that also stores A = U and dA = U - Ap (one workgroup).  A may
// alias U.
__global__ __launch_bounds__(1024) void k_mode_end(const double* U, const double* __restrict__ Ap,
                                                   double* A, double* __restrict__ dA, int64_t n,
                                                   double* out) {
  __shared__ double r0[16], r1[16];
  double a = 0.0, b = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 2048) {
    const double g0 = U[i], d0 = g0 - Ap[i];
    double g1 = 0.0, d1 = 0.0;
    const bool two = i + 1024 < n;
    if (two) {
      g1 = U[i + 1024];
      d1 = g1 - Ap[i + 1024];
    }
    a = fma(g0, g0, fma(g1, g1, a));
    b = fma(d0, d0, fma(d1, d1, b));
    dA[i] = d0;
    if (A) A[i] = g0;
    if (two) {
      dA[i + 1024] = d1;
      if (A) A[i + 1024] = g1;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
  }
  if ((threadIdx.x & 63) == 0) {
    r0[threadIdx.x >> 6] = a;
    r1[threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double sa = 0.0, sb = 0.0;
    for (int w = 0; w < 16; ++w) {
      sa += r0[w];
      sb += r1[w];
    }
    out[0] = sa;
    out[1] = sb;
  }
}

hipError_t launch_mode_end(const double* U, const double* Ap, double* A, double* dA, int64_t n,
                           double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_mode_end, dim3(1), dim3(1024), 0, s, U, Ap, A, dA, n, out);
  return hipGetLastError();
}

// C = Y (Y^T V), chunk of Y's columns [j0, j0 + wc) per workgroup.  Z = Y_chunk^T V: each
// entry (j, r) summed over the rows by G interleaved groups of threads (as in rr_project),
// then out[x][r] = sum_j Y[x][j0 + j] Z[j][r] in increasing j.
constexpr int WA_NE = 16;
constexpr int WA_LDS = 18000;  // doubles of dynamic LDS at most (144 KB)
constexpr int64_t kWApplyChunks = 32;

int w_apply_width(int64_t s, int64_t m, int R) {
  if (R < 1 || R > 64 || s < 1 || m < 1) return 0;
  const int64_t free_ = WA_LDS - 256 - s * R - s;  // the chunk's rows are padded by one
  if (free_ <= 0) return 0;
  int64_t w = free_ / (s + R);
  w = std::min<int64_t>(w, 4096 / R);  // Z entries: at most 16 per thread
  w = std::min<int64_t>(w, 256);
  // about kWApplyChunks workgroups: a chunk's sums are short and run side by side
  w = std::min<int64_t>(w, (m + kWApplyChunks - 1) / kWApplyChunks);
  return w >= 1 ? (int)w : 0;
}

__global__ __launch_bounds__(256) void k_w_apply(const double* __restrict__ Y,
                                                 const double* __restrict__ V, int s, int64_t m,
                                                 int R, int w, double* __restrict__ out) {
  extern __shared__ double sm[];
  const int tid = threadIdx.x;
  const int64_t j0 = (int64_t)blockIdx.x * w;
  const int wc = (int)(m - j0 < w ? m - j0 : w);
  const int ld = wc | 1;           // odd row stride: the rows of one column in different banks
  double* Ys = sm;                 // s x wc, row stride ld
  double* Vs = Ys + s * (w + 1);   // s x R
  double* Zs = Vs + s * R;   // wc x R
  double* red = Zs + w * R;
  const int ny = s * wc;  // < 2^15 (LDS)
  for (int e0 = tid; e0 < ny; e0 += 8 * 256) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      const int x = e / wc;
      v[q] = e < ny ? Y[x * m + j0 + (e - x * wc)] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int e = e0 + 256 * q;
      if (e < ny) {
        const int x = e / wc;
        Ys[x * ld + (e - x * wc)] = v[q];
      }
    }
  }
  stage_rows(Vs, V, s * R);
  __syncthreads();
  const int ZE = wc * R;
  int G = 1;
  while (2 * G * ZE <= 256) G *= 2;
  const int grp = G > 1 ? tid / ZE : 0;
  const int nent = G > 1 ? (tid < G * ZE ? 1 : 0) : (ZE + 255) / 256;
  double acc[WA_NE];
#pragma unroll
  for (int u = 0; u < WA_NE; ++u) acc[u] = 0.0;
#pragma unroll
  for (int u = 0; u < WA_NE; ++u) {
    const int e = G > 1 ? tid - grp * ZE : tid + 256 * u;
    if (u < nent && e < ZE) {
      const int j = e / R, r = e - j * R;
      double sum = 0.0;
      int x = grp;
      for (; x + 3 * G < s; x += 4 * G) {
        double yv[4], vv[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          yv[q] = Ys[(x + q * G) * ld + j];
          vv[q] = Vs[(x + q * G) * R + r];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) sum = fma(yv[q], vv[q], sum);
      }
      for (; x < s; x += G) sum = fma(Ys[x * ld + j], Vs[x * R + r], sum);
      acc[u] = sum;
    }
  }
  if (G > 1) {
    if (tid < G * ZE) red[tid] = acc[0];
    __syncthreads();
    if (tid < ZE) {
      double z = 0.0;
      for (int q = 0; q < G; ++q) z += red[q * ZE + tid];
      Zs[tid] = z;
    }
  } else {
#pragma unroll
    for (int u = 0; u < WA_NE; ++u) {
      const int e = tid + 256 * u;
      if (e < ZE) Zs[e] = acc[u];
    }
  }
  __syncthreads();
  double* o = out + (int64_t)blockIdx.x * s * R;
  for (int e = tid; e < s * R; e += 256) {
    const int x = e / R;
    const int r = e - x * R;
    const double* yr = Ys + x * ld;
    double c = 0.0;
#pragma unroll 8
    for (int j = 0; j < wc; ++j) c = fma(yr[j], Zs[j * R + r], c);
    o[e] = c;
  }
}

hipError_t launch_w_apply_parts(const double* Y, const double* V, int64_t s, int64_t m, int R,
                                int w, double* part, hipStream_t st) {
  if (w < 1 || w != w_apply_width(s, m, R)) return hipErrorInvalidValue;
  const int64_t nchunk = (m + w - 1) / w;
  const size_t lds = (size_t)(s * (w + 1) + s * R + (int64_t)w * R + 256) * sizeof(double);
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_w_apply),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_w_apply, dim3((unsigned)nchunk), dim3(256), lds, st, Y, V, (int)s, m, R,
                     w, part);
  return hipGetLastError();
}

hipError_t launch_w_apply(const double* Y, const double* V, int64_t s, int64_t m, int R, int w,
                          double* part, double* C, hipStream_t st) {
  hipError_t e = launch_w_apply_parts(Y, V, s, m, R, w, part, st);
  if (e != hipSuccess) return e;
  return launch_reduce_splits_to(C, 0, part, 0, (int)((m + w - 1) / w), s * R, st);
}

__global__ void k_copy2(double* __restrict__ o1, double* __restrict__ o2,
                        const double* __restrict__ in, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = in[i];
    o1[i] = v;
    o2[i] = v;
  }
}

hipError_t launch_copy2(double* out1, double* out2, const double* in, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 4096 ? 4096 : blocks);
  hipLaunchKernelGGL(k_copy2, dim3((unsigned)blocks), dim3(256), 0, s, out1, out2, in, n);
  return hipGetLastError();
}

// First-level contraction at rank R <= 8 on the vector units.  The matrix-core kernel pads
// the rank to a 16-column block and the contracted extent to 32-step chunks, so at R = 5
// over K = 35 it issues 5.9 times the useful multiply-adds (on this chip the FP64 matrix
// cores and the FP64 vector units have the same peak), and at an odd Q it cannot pair rows
// into 16-byte loads.  Here each thread owns TTM_RPT rows m = p Q + q spaced by
// the workgroup width (the lanes of a wave read 64 consecutive q: one 512-byte run per load
// instruction, across slices too), walks k in steps of TTM_KU with the next step's loads
// issued before the current step's multiply-adds (the last step reloads itself: the loads
// are unconditional, so their completion can be counted), and adds the k terms of a row in
// increasing k.  The first step takes K mod TTM_KU entries (all TTM_KU when it divides K).
// F's entries are the same for every lane.
constexpr int TTM_RPT = 4, TTM_KU = 4, TTM_THREADS = 256;
constexpr int64_t TTM_ROWS_PER_BLOCK = (int64_t)TTM_RPT * TTM_THREADS;

template <int RT>
__global__ __launch_bounds__(TTM_THREADS) void k_ttm_small_r(const double* __restrict__ T,
                                                             const double* __restrict__ F,
                                                             int64_t M, int64_t K, int64_t Q,
                                                             double* __restrict__ C) {
  const int64_t m0 = (int64_t)blockIdx.x * TTM_ROWS_PER_BLOCK + threadIdx.x;
  int64_t base[TTM_RPT];
#pragma unroll
  for (int j = 0; j < TTM_RPT; ++j) {
    const int64_t m = m0 + (int64_t)j * TTM_THREADS;
    const int64_t mm = m < M ? m : M - 1;  // rows past M read row M - 1 and store nothing
    const int64_t p = mm / Q, q = mm - p * Q;
    base[j] = p * K * Q + q;
  }
  const int64_t kr = K % TTM_KU;
  const int64_t nsteps = K / TTM_KU + (kr > 0 ? 1 : 0);
  auto kb_of = [&](int64_t t) -> int64_t {
    return kr > 0 ? (t == 0 ? 0 : kr + (t - 1) * TTM_KU) : t * TTM_KU;
  };
  auto nu_of = [&](int64_t t) -> int { return (kr > 0 && t == 0) ? (int)kr : TTM_KU; };
  auto load = [&](double (&x)[TTM_KU][TTM_RPT], int64_t t) {
    const int64_t kb = kb_of(t);
    const int nu = nu_of(t);
#pragma unroll
    for (int u = 0; u < TTM_KU; ++u) {
      const int64_t off = (kb + (u < nu ? u : 0)) * Q;
#pragma unroll
      for (int j = 0; j < TTM_RPT; ++j) x[u][j] = T[base[j] + off];
    }
  };
  double acc[TTM_RPT][RT];
#pragma unroll
  for (int j = 0; j < TTM_RPT; ++j)
#pragma unroll
    for (int r = 0; r < RT; ++r) acc[j][r] = 0.0;
  double xc[TTM_KU][TTM_RPT], xn[TTM_KU][TTM_RPT];
  load(xc, 0);
  for (int64_t t = 0; t < nsteps; ++t) {
    load(xn, t + 1 < nsteps ? t + 1 : t);
    const int64_t kb = kb_of(t);
    const int nu = nu_of(t);
#pragma unroll
    for (int u = 0; u < TTM_KU; ++u) {
      if (u < nu) {
        const double* f = F + (kb + u) * RT;
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const double fr = f[r];
#pragma unroll
          for (int j = 0; j < TTM_RPT; ++j) acc[j][r] = fma(xc[u][j], fr, acc[j][r]);
        }
      }
    }
#pragma unroll
    for (int u = 0; u < TTM_KU; ++u)
#pragma unroll
      for (int j = 0; j < TTM_RPT; ++j) xc[u][j] = xn[u][j];
  }
#pragma unroll
  for (int j = 0; j < TTM_RPT; ++j) {
    const int64_t m = m0 + (int64_t)j * TTM_THREADS;
    if (m < M) {
#pragma unroll
      for (int r = 0; r < RT; ++r) C[m * RT + r] = acc[j][r];
    }
  }
}

// Odd Q > 1 (an even Q gives the matrix-core kernel its 16-byte loads, and there the two
// measured within 2% of each other; Q > 1 keeps the lanes' loads consecutive) and rows
// for at least 1024 workgroups (the kernel does not split K).
bool ttm_small_r_fits(int64_t M, int64_t K, int64_t Q, int R) {
  return R >= 1 && R <= 8 && K >= 1 && Q > 1 && (Q & 1) == 1 &&
         M >= 1024 * TTM_ROWS_PER_BLOCK && M / TTM_ROWS_PER_BLOCK < (int64_t(1) << 31);
}

hipError_t launch_ttm_small_r(const double* T, const double* F, int64_t M, int64_t K, int64_t Q,
                              int R, double* C, hipStream_t s) {
  if (!ttm_small_r_fits(M, K, Q, R) || M % Q != 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((M + TTM_ROWS_PER_BLOCK - 1) / TTM_ROWS_PER_BLOCK)), block(TTM_THREADS);
  switch (R) {
#define PPK_TTM_CASE(RV) \
  case RV: hipLaunchKernelGGL(k_ttm_small_r<RV>, grid, block, 0, s, T, F, M, K, Q, C); break;
    PPK_TTM_CASE(1) PPK_TTM_CASE(2) PPK_TTM_CASE(3) PPK_TTM_CASE(4)
    PPK_TTM_CASE(5) PPK_TTM_CASE(6) PPK_TTM_CASE(7) PPK_TTM_CASE(8)
#undef PPK_TTM_CASE
  }
  return hipGetLastError();
}

// The same contraction for a few rows over a long k (the HOSVD's C = X_(n) Z: M = s_n
// rows, K = the product of the other sizes, k = c_before * after + c_after with `after`
// the product of the sizes after n, so T[m][k] sits at (k / after) M after + m after +
// k mod after; after = K when n is first).  The matrix-core kernel pads M to 128-row
// tiles and R to 16 columns there (11.7 times the useful multiply-adds at M = 35, R = 5).
// Here workgroup z takes k in [z kper, (z + 1) kper), in blocks of TR_THREADS TR_KPT:
// thread t holds F's rows k = k0 + t + TR_THREADS i (i < TR_KPT) in registers and, row by
// row, loads T[m][k] for them (consecutive lanes on consecutive k: one 512-byte run per
// load instruction while k mod after runs on), the next row's loads issued before this
// row's multiply-adds; the R per-lane sums of a row are added across the wave by a
// butterfly and wave w's lane 0 adds them to its own LDS slot [w][m][r].  At the end the
// slots are added in wave order into part[z] (M x R); a second launch adds the
// workgroups' parts in z order.  k past the range reads a valid entry of the range with
// F's row taken as zero.
constexpr int TR_KPT = 8, TR_THREADS = 256, TR_WAVES = TR_THREADS / 64;
constexpr int64_t TR_KBLOCK = (int64_t)TR_THREADS * TR_KPT;

template <int RT>
__global__ __launch_bounds__(TR_THREADS) void k_ttm_rows_small_r(const double* __restrict__ T,
                                                                 const double* __restrict__ F,
                                                                 int M, int64_t K, int64_t after,
                                                                 int64_t kper,
                                                                 double* __restrict__ part) {
  extern __shared__ double slot[];  // [TR_WAVES][M][RT]
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  for (int e = tid; e < TR_WAVES * M * RT; e += TR_THREADS) slot[e] = 0.0;
  __syncthreads();
  const int64_t kb = (int64_t)blockIdx.x * kper;
  const int64_t ke = kb + kper < K ? kb + kper : K;
  for (int64_t k0 = kb; k0 < ke; k0 += TR_KBLOCK) {
    int64_t koff[TR_KPT];  // offset of T[0][k]
    double z[TR_KPT][RT];
#pragma unroll
    for (int i = 0; i < TR_KPT; ++i) {
      const int64_t k = k0 + tid + (int64_t)TR_THREADS * i;
      const bool ok = k < ke;
      const int64_t kc = ok ? k : ke - 1;
      const int64_t hi = kc / after;
      koff[i] = hi * M * after + (kc - hi * after);
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const double f = F[kc * RT + r];
        z[i][r] = ok ? f : 0.0;
      }
    }
    double xc[TR_KPT], xn[TR_KPT];
#pragma unroll
    for (int i = 0; i < TR_KPT; ++i) xc[i] = T[koff[i]];
    for (int m = 0; m < M; ++m) {
      const int64_t mn = (m + 1 < M ? m + 1 : m) * after;
#pragma unroll
      for (int i = 0; i < TR_KPT; ++i) xn[i] = T[mn + koff[i]];
      double a[RT];
#pragma unroll
      for (int r = 0; r < RT; ++r) a[r] = 0.0;
#pragma unroll
      for (int i = 0; i < TR_KPT; ++i)
#pragma unroll
        for (int r = 0; r < RT; ++r) a[r] = fma(xc[i], z[i][r], a[r]);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int r = 0; r < RT; ++r) a[r] += __shfl_xor(a[r], off);
      if (l == 0) {
#pragma unroll
        for (int r = 0; r < RT; ++r) slot[(w * M + m) * RT + r] += a[r];
      }
#pragma unroll
      for (int i = 0; i < TR_KPT; ++i) xc[i] = xn[i];
    }
  }
  __syncthreads();
  for (int e = tid; e < M * RT; e += TR_THREADS) {
    double sum = 0.0;
#pragma unroll
    for (int v = 0; v < TR_WAVES; ++v) sum += slot[v * M * RT + e];
    part[(int64_t)blockIdx.x * M * RT + e] = sum;
  }
}

// R <= 8, Q = 1, at most 2048 entries of output (the LDS slots: 4 x 2048 doubles, 64 KB),
// at least 2^20 k and at least 256 workgroups' worth of partial slots.
int ttm_rows_small_r_parts(int64_t M, int64_t K, int R, int max_parts) {
  if (R < 1 || R > 8 || M < 1 || M * R > 2048 || K < (int64_t(1) << 20) || max_parts < 256)
    return 0;
  const int want = max_parts < 2048 ? max_parts : 2048;
  const int64_t kper = ((K + want - 1) / want + TR_KBLOCK - 1) / TR_KBLOCK * TR_KBLOCK;
  return (int)((K + kper - 1) / kper);
}

hipError_t launch_ttm_rows_small_r(const double* T, const double* F, int64_t M, int64_t K,
                                   int64_t after, int R, int nparts, double* part, double* C,
                                   hipStream_t s) {
  if (nparts < 1 || R < 1 || R > 8 || M < 1 || M * R > 2048 || after < 1 || K % after != 0)
    return hipErrorInvalidValue;
  const int64_t kper = ((K + nparts - 1) / nparts + TR_KBLOCK - 1) / TR_KBLOCK * TR_KBLOCK;
  const int nz = (int)((K + kper - 1) / kper);
  if (nz > nparts) return hipErrorInvalidValue;
  const size_t lds = (size_t)TR_WAVES * M * R * sizeof(double);
  switch (R) {
#define PPK_TR_CASE(RV)                                                                       \
  case RV:                                                                                    \
    hipLaunchKernelGGL(k_ttm_rows_small_r<RV>, dim3((unsigned)nz), dim3(TR_THREADS), lds, s, T, \
                       F, (int)M, K, after, kper, part);                                      \
    break;
    PPK_TR_CASE(1) PPK_TR_CASE(2) PPK_TR_CASE(3) PPK_TR_CASE(4)
    PPK_TR_CASE(5) PPK_TR_CASE(6) PPK_TR_CASE(7) PPK_TR_CASE(8)
#undef PPK_TR_CASE
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_reduce_splits_to(C, 0, part, 0, nz, M * R, s);
}

}  // namespace ppk
