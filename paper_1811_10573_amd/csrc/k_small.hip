// FP64 small dense work of every mode update (Algorithm 1 / Algorithm 3 loop
// bodies): Gamma^(n) (Hadamard product of the other Grams), the second-order
// matrix W^(n) of the general PP update, the Cholesky factorisation of Gamma,
// the row-parallel triangular solves for A_new, the gradient
// G = (A_old - A_new) Gamma, dA, the Grams S = A^T A and U = A^T dA, the norms
// that feed the switching rule and the fit.  Also ||X||^2, the exact residual
// and the FP32 -> bfloat16 cast.
#include "common.h"
#include "../../include/ppals.h"

namespace ppk {

__device__ __forceinline__ double bcast_lane(double v, int lane) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), lane);
  const int hi = __builtin_amdgcn_readlane((int)(u >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Block-wide sum of one double per thread (blockDim.x == 256); result valid in all threads.
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0.0;
  const int nw = blockDim.x >> 6;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// Cholesky (lower) of the R x R matrix a (row-major, in LDS), right-looking.
// Returns -1 on success, else the 0-based index of the first pivot that is not positive
// and finite.  All threads of the block participate.
// Cholesky factorisation in place (lower) of the R x R matrix a with row stride LS (R + 1:
// consecutive rows fall in different LDS banks).  Returns -1, or the index of the first
// pivot that is not positive and finite (the matrix is then left partly factorised).
// One barrier per column: at step j every thread reads the pivot, updates the trailing
// block with column j scaled on the fly (the same roundings as scaling the column first),
// and scales column j - 1, which no longer takes part.  16 x 16 thread grid, no divisions.
__device__ int chol_lds(double* a, int R, int LS) {
  const int tid = threadIdx.x;
  const int ti = tid >> 4, tk = tid & 15;
  double prev_inv = 0.0, prev_sd = 0.0;
  __syncthreads();
  for (int j = 0; j < R; ++j) {
    const double d = a[j * LS + j];
    if (!(d > 0.0) || !isfinite(d)) return j;  // the same value in every thread
    const double sd = sqrt(d);
    const double inv = 1.0 / sd;
    if (j > 0)
      for (int i = j - 1 + tid; i < R; i += blockDim.x)
        a[i * LS + j - 1] = (i == j - 1) ? prev_sd : a[i * LS + j - 1] * prev_inv;
    for (int i = j + 1 + ti; i < R; i += 16) {
      const double lij = a[i * LS + j] * inv;
      for (int k = j + 1 + tk; k <= i; k += 16) a[i * LS + k] -= lij * (a[k * LS + j] * inv);
    }
    prev_inv = inv;
    prev_sd = sd;
    __syncthreads();
  }
  if (tid == 0) a[(R - 1) * LS + R - 1] = prev_sd;  // the last column is its diagonal
  __syncthreads();
  return -1;
}

// Cholesky status word: bits 0-1 the outcome (0 clean, 1 factorised after the diagonal
// shift, 2 failed after it), bits 8-30 one plus the first failed pivot of the unshifted
// factorisation (0: none).
__device__ __forceinline__ int chol_status_lds(int code, int pivot) { return code | ((pivot + 1) << 8); }

// One workgroup: finish mode `prev` (record entries, fit) and prepare mode `n`
// (Gamma, W, Cholesky with the diagonal-shift retry).
__global__ __launch_bounds__(256) void k_mode_begin(ModeArgs a) {
  extern __shared__ double sm[];  // R x R, row stride R + 1
  __shared__ double red[8];
  const int tid = threadIdx.x;
  const int R = a.R, RR = R * R, LS = R + 1;
  ppals_sweep_record* rec = (ppals_sweep_record*)a.rec;

  if (a.prev >= 0) {
    double g2 = 0, d2 = 0, a2 = 0, ma = 0;
    for (int64_t y = tid; y < a.prev_rows; y += blockDim.x) {
      g2 += a.rowpart[y * 4 + 0];
      d2 += a.rowpart[y * 4 + 1];
      a2 += a.rowpart[y * 4 + 2];
      ma += a.rowpart[y * 4 + 3];
    }
    g2 = block_sum(g2, red);
    d2 = block_sum(d2, red);
    a2 = block_sum(a2, red);
    ma = block_sum(ma, red);
    double fitnrm = 0.0;
    if (a.write_fit) {
      double s = 0.0;
      const double* Sp = a.S + (int64_t)a.prev * RR;
      for (int e = tid; e < RR; e += blockDim.x) s += a.gamma[e] * Sp[e];
      fitnrm = block_sum(s, red);
    }
    if (tid == 0) {
      rec->grad_norm[a.prev] = sqrt(g2);
      rec->rel_change[a.prev] = a2 > 0.0 ? sqrt(d2) / sqrt(a2) : (d2 > 0.0 ? INFINITY : 0.0);
      const int stw = a.status[a.prev];
      rec->chol_status[a.prev] = stw & 3;
      rec->chol_pivot[a.prev] = (stw >> 8) - 1;
      rec->nonfinite[a.prev] = (isfinite(g2) && isfinite(a2) && isfinite(ma)) ? 0 : 1;
      if (a.write_fit) {
        const double r2 = a.normX2 - 2.0 * ma + fitnrm;
        rec->fit_est = 1.0 - sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(a.normX2);
        rec->sweep_kind = a.sweep_kind;
      }
    }
    __syncthreads();
  }

  if (a.n < 0) return;
  const int n = a.n, N = a.N;
  for (int e = tid; e < RR; e += blockDim.x) {
    double v = 1.0;
    for (int i = 0; i < N; ++i)
      if (i != n) v *= a.S[(int64_t)i * RR + e];
    sm[(e / R) * LS + e % R] = v;
    a.gamma[e] = v;
    if (a.pp && a.second_order) {
      double w = 0.0;
      for (int i = 0; i < N; ++i) {
        if (i == n) continue;
        for (int j2 = i + 1; j2 < N; ++j2) {
          if (j2 == n) continue;
          double t = a.U[(int64_t)i * RR + e] * a.U[(int64_t)j2 * RR + e];
          for (int k = 0; k < N; ++k)
            if (k != i && k != j2 && k != n) t *= a.S[(int64_t)k * RR + e];
          w += t;
        }
      }
      a.W[e] = w;
    }
  }
  __syncthreads();
  int st = 0;
  const int piv0 = chol_lds(sm, R, LS);
  if (piv0 >= 0) {
    // retry with Gamma + delta I, delta = R 2^-52 max(diag Gamma)
    double mx = 0.0;
    for (int e = tid; e < R; e += blockDim.x) mx = fmax(mx, a.gamma[e * R + e]);
    // block max via shared
    __syncthreads();
    __shared__ double mxs[256];
    mxs[tid] = mx;
    __syncthreads();
    if (tid == 0) {
      double m2 = 0.0;
      for (int i = 0; i < (int)blockDim.x; ++i) m2 = fmax(m2, mxs[i]);
      mxs[0] = m2;
    }
    __syncthreads();
    const double delta = (double)R * 0x1p-52 * mxs[0];
    for (int e = tid; e < RR; e += blockDim.x) {
      const int i = e / R, k = e - (e / R) * R;
      sm[i * LS + k] = a.gamma[e] + (i == k ? delta : 0.0);
    }
    st = chol_lds(sm, R, LS) < 0 ? 1 : 2;
  }
  for (int e = tid; e < RR; e += blockDim.x) {
    const int i = e / R, k = e - (e / R) * R;
    a.L[e] = (k <= i) ? sm[i * LS + k] : 0.0;
  }
  if (tid == 0) a.status[n] = chol_status_lds(st, piv0);
}

// Row-parallel solve of A_new Gamma = M with Gamma = L L^T; one wave per row,
// lane k owns column k (and k + 64 when R > 64).
__global__ __launch_bounds__(256) void k_solve_rows(SolveArgs a) {
  extern __shared__ double lsm[];  // L with padded stride R+1, then 1/diag
  const int R = a.R, LS = R + 1;
  double* Ls = lsm;
  double* invd = lsm + (size_t)R * LS;
  for (int e = threadIdx.x; e < R * R; e += blockDim.x) {
    const int i = e / R, k = e - i * R;
    Ls[i * LS + k] = a.L[e];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < R; e += blockDim.x) invd[e] = 1.0 / Ls[e * LS + e];
  __syncthreads();
  const int st = *a.status & 3;
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t wave_global = (int64_t)blockIdx.x * (blockDim.x >> 6) + w;
  const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x >> 6);
  const int k0 = l, k1 = l + 64;
  const bool v0 = k0 < R, v1 = k1 < R;
  for (int64_t y = wave_global; y < a.rows; y += nwaves) {
    const int64_t rb = y * R;
    double m0 = 0, m1 = 0;
    if (a.M) {
      m0 = v0 ? a.M[rb + k0] : 0.0;
      m1 = v1 ? a.M[rb + k1] : 0.0;
    } else {
      m0 = v0 ? (double)a.M32[rb + k0] : 0.0;
      m1 = v1 ? (double)a.M32[rb + k1] : 0.0;
    }
    const double mo0 = m0, mo1 = m1;
    const double aold0 = v0 ? a.A[rb + k0] : 0.0;
    const double aold1 = v1 ? a.A[rb + k1] : 0.0;
    double x0 = aold0, x1 = aold1;
    if (st != 2) {
      // forward: L z = m (column-oriented)
      for (int j = 0; j < R; ++j) {
        const double mj = (j < 64) ? bcast_lane(m0, j) : bcast_lane(m1, j - 64);
        const double zj = mj * invd[j];
        if (v0) { if (k0 == j) m0 = zj; else if (k0 > j) m0 -= Ls[k0 * LS + j] * zj; }
        if (v1) { if (k1 == j) m1 = zj; else if (k1 > j) m1 -= Ls[k1 * LS + j] * zj; }
      }
      // backward: L^T x = z
      for (int j = R - 1; j >= 0; --j) {
        const double zj = (j < 64) ? bcast_lane(m0, j) : bcast_lane(m1, j - 64);
        const double xj = zj * invd[j];
        if (v0) { if (k0 == j) m0 = xj; else if (k0 < j) m0 -= Ls[j * LS + k0] * xj; }
        if (v1) { if (k1 == j) m1 = xj; else if (k1 < j) m1 -= Ls[j * LS + k1] * xj; }
      }
      x0 = m0;
      x1 = m1;
    }
    // gradient row g = (a_old - a_new) Gamma
    const double dd0 = aold0 - x0, dd1 = aold1 - x1;
    double g0 = 0.0, g1 = 0.0;
    for (int j = 0; j < R; ++j) {
      const double dj = (j < 64) ? bcast_lane(dd0, j) : bcast_lane(dd1, j - 64);
      if (v0) g0 = fma(dj, a.gamma[j * R + k0], g0);
      if (v1) g1 = fma(dj, a.gamma[j * R + k1], g1);
    }
    // step-size variant (Section 5.1): A_new = A_old + step (A_sol - A_old), after the
    // gradient at A_old
    if (a.step != 1.0) {
      x0 = fma(a.step, x0 - aold0, aold0);
      x1 = fma(a.step, x1 - aold1, aold1);
    }
    const double ref0 = a.Aref ? (v0 ? a.Aref[rb + k0] : 0.0) : aold0;
    const double ref1 = a.Aref ? (v1 ? a.Aref[rb + k1] : 0.0) : aold1;
    const double da0 = x0 - ref0, da1 = x1 - ref1;
    if (v0) { a.A[rb + k0] = x0; if (a.dA) a.dA[rb + k0] = da0; }
    if (v1) { a.A[rb + k1] = x1; if (a.dA) a.dA[rb + k1] = da1; }
    const double sg = wave_sum(g0 * g0 + g1 * g1);
    const double sd = wave_sum(da0 * da0 + da1 * da1);
    const double sa = wave_sum(x0 * x0 + x1 * x1);
    const double sm = wave_sum(mo0 * x0 + mo1 * x1);
    if (l == 0) {
      a.rowpart[y * 4 + 0] = sg;
      a.rowpart[y * 4 + 1] = sd;
      a.rowpart[y * 4 + 2] = sa;
      a.rowpart[y * 4 + 3] = sm;
    }
  }
}

// S_out[r][q] = sum_y A[y][r] A[y][q]; U_out[r][q] = sum_y A[y][r] dA[y][q] (blockIdx.y == 1).
__global__ __launch_bounds__(256) void k_gram(const double* __restrict__ A,
                                              const double* __restrict__ dA, int64_t rows, int R,
                                              double* __restrict__ S_out,
                                              double* __restrict__ U_out) {
  constexpr int CH = 32;
  extern __shared__ double gsm[];  // 2 * CH * R
  double* la = gsm;
  double* lb = gsm + CH * R;
  const double* Y = blockIdx.y ? dA : A;
  double* out = blockIdx.y ? U_out : S_out;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int r = e / R, q = e - (e / R) * R;
  const bool act = e < R * R;
  double acc = 0.0;
  for (int64_t y0 = 0; y0 < rows; y0 += CH) {
    const int nr = (int)min((int64_t)CH, rows - y0);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * R; t += blockDim.x) {
      la[t] = A[y0 * R + t];
      lb[t] = Y[y0 * R + t];
    }
    __syncthreads();
    if (act)
      for (int y = 0; y < nr; ++y) acc = fma(la[y * R + r], lb[y * R + q], acc);
  }
  if (act) out[e] = acc;
}

// ||X||^2 partials and final sum.
template <typename T>
__global__ __launch_bounds__(256) void k_norm2_part(const T* __restrict__ X, int64_t n,
                                                    double* __restrict__ part) {
  __shared__ double red[8];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double v = (double)X[i];
    s = fma(v, v, s);
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int n,
                                                   double* __restrict__ out) {
  __shared__ double red[8];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) *out = s;
}

__global__ void k_cast_bf16(const float* __restrict__ in, uint16_t* __restrict__ out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t u = __float_as_uint(in[i]);
    uint16_t r;
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) r = 0x7FC0;
    else r = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    out[i] = r;
  }
}

// ||X - [[A]]||^2 partials.  Rows are the leading N-1 indices; thread owns last-mode
// index xl and keeps A_N[xl][:] in registers (R <= 64); the products of the leading
// factors for a chunk of rows are staged in LDS.
struct ResArgs {
  const void* X;
  int dt;
  const double* A[PP_MAXN];
  int64_t dims[PP_MAXN];
  int N, R;
  int64_t nrows;   // prod of leading dims
  int64_t rows_per_block;
  double* part;
};
__global__ __launch_bounds__(256) void k_residual2(ResArgs a) {
  constexpr int RC = 16;  // rows staged per pass
  __shared__ double lp[RC * 64];
  __shared__ double red[8];
  const int R = a.R;
  const int64_t sN = a.dims[a.N - 1];
  const int64_t xl = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = xl < sN;
  double an[64];
#pragma unroll
  for (int r = 0; r < 64; ++r) an[r] = (act && r < R) ? a.A[a.N - 1][xl * R + r] : 0.0;
  const int64_t r0 = (int64_t)blockIdx.y * a.rows_per_block;
  const int64_t r1 = min(a.nrows, r0 + a.rows_per_block);
  double acc = 0.0;
  for (int64_t rb = r0; rb < r1; rb += RC) {
    const int nr = (int)min((int64_t)RC, r1 - rb);
    __syncthreads();
    for (int t = threadIdx.x; t < nr * 64; t += blockDim.x) {
      const int rr = t / 64, r = t - rr * 64;
      double v = 0.0;
      if (r < R) {
        int64_t row = rb + rr;
        v = 1.0;
        for (int f = a.N - 2; f >= 0; --f) {
          const int64_t d = row % a.dims[f];
          row /= a.dims[f];
          v *= a.A[f][d * R + r];
        }
      }
      lp[t] = v;
    }
    __syncthreads();
    if (act) {
      for (int rr = 0; rr < nr; ++rr) {
        double m = 0.0;
#pragma unroll
        for (int r = 0; r < 64; ++r) m = fma(lp[rr * 64 + r], an[r], m);
        const int64_t off = (rb + rr) * sN + xl;
        const double xv = a.dt == DT_F64 ? ((const double*)a.X)[off] : (double)((const float*)a.X)[off];
        const double d = xv - m;
        acc = fma(d, d, acc);
      }
    }
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// Generic (any R <= 128) residual: one thread per element.
__global__ __launch_bounds__(256) void k_residual2_generic(ResArgs a, int64_t total) {
  __shared__ double red[8];
  double acc = 0.0;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double m = 0.0;
    for (int r = 0; r < a.R; ++r) {
      int64_t e = idx;
      double v = 1.0;
      for (int f = a.N - 1; f >= 0; --f) {
        const int64_t d = e % a.dims[f];
        e /= a.dims[f];
        v *= a.A[f][d * a.R + r];
      }
      m += v;
    }
    const double xv = a.dt == DT_F64 ? ((const double*)a.X)[idx] : (double)((const float*)a.X)[idx];
    const double d = xv - m;
    acc = fma(d, d, acc);
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a.part[blockIdx.x] = acc;
}

__global__ void k_finish_gram_solve(const double* __restrict__ rowpart, int64_t rows,
                                    double* grad_out, int32_t* status_out, const int* status) {
  __shared__ double red[8];
  double s = 0.0, a2 = 0.0;
  for (int64_t y = threadIdx.x; y < rows; y += blockDim.x) {
    s += rowpart[y * 4];
    a2 += rowpart[y * 4 + 2];
  }
  s = block_sum(s, red);
  a2 = block_sum(a2, red);
  if (threadIdx.x == 0) {
    *grad_out = sqrt(s);
    // the Cholesky status word, plus bit 4 when the new factor or the gradient holds a
    // value that is not finite
    *status_out = *status | ((isfinite(s) && isfinite(a2)) ? 0 : 16);
  }
}

__global__ __launch_bounds__(256) void k_chol_standalone(const double* gamma, int R, double* L,
                                                         int* status) {
  extern __shared__ double sm[];  // R x R, row stride R + 1
  __shared__ double mxs;
  const int RR = R * R, LS = R + 1;
  for (int e = threadIdx.x; e < RR; e += blockDim.x) sm[(e / R) * LS + e % R] = gamma[e];
  int st = 0;
  const int piv0 = chol_lds(sm, R, LS);
  if (piv0 >= 0) {
    if (threadIdx.x == 0) {
      double m2 = 0.0;
      for (int i = 0; i < R; ++i) m2 = fmax(m2, gamma[i * R + i]);
      mxs = m2;
    }
    __syncthreads();
    const double delta = (double)R * 0x1p-52 * mxs;
    for (int e = threadIdx.x; e < RR; e += blockDim.x) {
      const int i = e / R, k = e - (e / R) * R;
      sm[i * LS + k] = gamma[e] + (i == k ? delta : 0.0);
    }
    st = chol_lds(sm, R, LS) < 0 ? 1 : 2;
  }
  for (int e = threadIdx.x; e < RR; e += blockDim.x) {
    const int i = e / R, k = e - (e / R) * R;
    L[e] = (k <= i) ? sm[i * LS + k] : 0.0;
  }
  if (threadIdx.x == 0) *status = chol_status_lds(st, piv0);
}

// ---------------------------------------------------------------------------
// Dynamic LDS above 64 KiB (rank > 90) must be requested explicitly.
template <typename K>
static hipError_t allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return hipSuccess;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(kernel),
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
}

hipError_t launch_mode_begin(const ModeArgs& a, hipStream_t s) {
  size_t lds = (size_t)a.R * (a.R + 1) * sizeof(double);
  hipError_t e = allow_lds(k_mode_begin, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mode_begin, dim3(1), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_solve_rows(const SolveArgs& a, hipStream_t s) {
  const int64_t waves = a.rows;  // one wave per row
  int64_t blocks = (waves + 3) / 4;
  if (blocks > 2048) blocks = 2048;
  if (blocks < 1) blocks = 1;
  size_t lds = ((size_t)a.R * (a.R + 1) + a.R) * sizeof(double);
  hipError_t e = allow_lds(k_solve_rows, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_solve_rows, dim3((unsigned)blocks), dim3(256), lds, s, a);
  return hipGetLastError();
}

hipError_t launch_gram(const double* A, const double* dA, int64_t rows, int R, double* S_out,
                       double* U_out, hipStream_t s) {
  const int blocks = (R * R + 255) / 256;
  size_t lds = 2 * 32 * (size_t)R * sizeof(double);
  hipLaunchKernelGGL(k_gram, dim3(blocks, dA ? 2 : 1), dim3(256), lds, s, A, dA, rows, R, S_out,
                     U_out);
  return hipGetLastError();
}

hipError_t launch_norm2(const void* X, int dt, int64_t n, double* partial, int nblocks,
                        double* out, hipStream_t s) {
  if (dt == DT_F64)
    hipLaunchKernelGGL(k_norm2_part<double>, dim3(nblocks), dim3(256), 0, s, (const double*)X, n, partial);
  else
    hipLaunchKernelGGL(k_norm2_part<float>, dim3(nblocks), dim3(256), 0, s, (const float*)X, n, partial);
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, partial, nblocks, out);
  return hipGetLastError();
}

hipError_t launch_cast_bf16(const float* in, uint16_t* out, int64_t n, hipStream_t s) {
  int64_t blocks = (n + 255) / 256;
  if (blocks > 16384) blocks = 16384;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_cast_bf16, dim3((unsigned)blocks), dim3(256), 0, s, in, out, n);
  return hipGetLastError();
}

hipError_t launch_residual2(const void* X, int dt, const double* const* A, const int64_t* dims,
                            int N, int R, double* partial, int nblocks, double* out,
                            hipStream_t s) {
  ResArgs a;
  a.X = X;
  a.dt = dt;
  for (int i = 0; i < N; ++i) { a.A[i] = A[i]; a.dims[i] = dims[i]; }
  a.N = N;
  a.R = R;
  int64_t nrows = 1;
  for (int i = 0; i < N - 1; ++i) nrows *= dims[i];
  a.nrows = nrows;
  a.part = partial;
  const int64_t sN = dims[N - 1];
  if (R <= 64) {
    const int gx = (int)((sN + 255) / 256);
    int gy = nblocks / gx;
    if (gy < 1) gy = 1;
    if (gy > nrows) gy = (int)nrows;
    a.rows_per_block = (nrows + gy - 1) / gy;
    gy = (int)((nrows + a.rows_per_block - 1) / a.rows_per_block);
    hipLaunchKernelGGL(k_residual2, dim3(gx, gy), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, partial, gx * gy, out);
  } else {
    hipLaunchKernelGGL(k_residual2_generic, dim3(nblocks), dim3(256), 0, s, a, nrows * sN);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(256), 0, s, partial, nblocks, out);
  }
  return hipGetLastError();
}

hipError_t launch_finish_gram_solve(const double* rowpart, int64_t rows, double* grad_out,
                                    int32_t* status_out, const int* status, hipStream_t s) {
  hipLaunchKernelGGL(k_finish_gram_solve, dim3(1), dim3(256), 0, s, rowpart, rows, grad_out,
                     status_out, status);
  return hipGetLastError();
}

hipError_t launch_chol_standalone(const double* gamma, int R, double* L, int* status,
                                  hipStream_t s) {
  hipError_t e = allow_lds(k_chol_standalone, (size_t)R * (R + 1) * sizeof(double));
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_chol_standalone, dim3(1), dim3(256), (size_t)R * (R + 1) * sizeof(double), s,
                     gamma, R, L, status);
  return hipGetLastError();
}

// End of an operator build in one launch (BuildReset).
__global__ void k_build_reset(BuildReset r) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i < r.off[r.N]; i += stride) {
    int n = 0;
    while (n + 1 < r.N && i >= r.off[n + 1]) ++n;
    r.Ap[i] = r.A[n][i - r.off[n]];
  }
  for (int64_t i = t0; i < r.ndA; i += stride) r.dA[i] = 0.0;
  for (int64_t i = t0; i < r.nU; i += stride) r.U[i] = 0.0;
  for (int q = 0; q < 2; ++q)
    for (int64_t i = t0; i < r.nints[q]; i += stride) r.ints[q][i] = 0;
}
hipError_t launch_build_reset(const BuildReset& r, hipStream_t s) {
  if (r.N < 1 || r.N > PP_MAXN) return hipErrorInvalidValue;
  int64_t n = r.off[r.N];
  if (r.ndA > n) n = r.ndA;
  if (r.nU > n) n = r.nU;
  int64_t blocks = (n + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 1024 ? 1024 : blocks);
  hipLaunchKernelGGL(k_build_reset, dim3((unsigned)blocks), dim3(256), 0, s, r);
  return hipGetLastError();
}

}  // namespace ppk
