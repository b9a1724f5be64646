// Learned controller for leaving the PP phase: a two-layer MLP
//   h = tanh(W1 x + b1),  y = W2 . h + b2
// regressing log10 of the relative PP right-hand-side error on the state of the
// iteration.  (Algorithm 3 leaves PP with a fixed threshold on ||dA||/||A||;
// other switching schemes are named as future work in Section 6.)
//
// All network arithmetic is FP32.  Flat parameter layout:
//   [W1 (H x d, row-major), b1 (H), W2 (H), b2 (1)].
// Reductions run in a fixed order (wave shuffles, then waves in index order), so
// the results are deterministic.
#include "common.h"
#include "../../include/ppals.h"

namespace ppk {

__device__ __forceinline__ float wsumf(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wave per sample: lane j (and j + 64, ...) evaluates hidden unit j.
__global__ __launch_bounds__(256) void k_mlp_forward(const float* __restrict__ p, int d, int H,
                                                     const float* __restrict__ X, int64_t B,
                                                     float* __restrict__ y,
                                                     float* __restrict__ hcache) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * 4 + w;
  if (b >= B) return;
  const float* W1 = p;
  const float* b1 = p + (size_t)H * d;
  const float* W2 = b1 + H;
  const float b2 = W2[H];
  float xin[MLP_MAX_IN];
#pragma unroll
  for (int i = 0; i < MLP_MAX_IN; ++i) xin[i] = i < d ? X[b * d + i] : 0.0f;
  float acc = 0.0f;
  for (int j = l; j < H; j += 64) {
    float z = b1[j];
#pragma unroll
    for (int i = 0; i < MLP_MAX_IN; ++i)
      if (i < d) z = fmaf(W1[j * d + i], xin[i], z);
    const float hj = tanhf(z);
    if (hcache) hcache[b * H + j] = hj;
    acc = fmaf(W2[j], hj, acc);
  }
  acc = wsumf(acc);
  if (l == 0) y[b] = acc + b2;
}

// Gradient of L = (1/B) sum_b (y_b - t_b)^2.  Block j < H: the parameters of hidden
// unit j (W1[j][:], b1[j], W2[j]); block H: b2 and the loss.
__global__ __launch_bounds__(256) void k_mlp_backward(const float* __restrict__ p, int d, int H,
                                                      const float* __restrict__ X,
                                                      const float* __restrict__ hcache,
                                                      const float* __restrict__ y,
                                                      const float* __restrict__ t, int64_t B,
                                                      float* __restrict__ g,
                                                      float* __restrict__ loss) {
  __shared__ float red[4][MLP_MAX_IN + 2];
  const int tid = threadIdx.x, w = tid >> 6, l = tid & 63;
  const int j = blockIdx.x;
  const float invB = 1.0f / (float)B;
  float acc[MLP_MAX_IN + 2];
#pragma unroll
  for (int k = 0; k < MLP_MAX_IN + 2; ++k) acc[k] = 0.0f;
  if (j < H) {
    const float w2 = p[(size_t)H * d + H + j];
    for (int64_t b = tid; b < B; b += blockDim.x) {
      const float dy = 2.0f * (y[b] - t[b]) * invB;
      const float hj = hcache[b * H + j];
      const float dz = dy * w2 * (1.0f - hj * hj);
#pragma unroll
      for (int i = 0; i < MLP_MAX_IN; ++i)
        if (i < d) acc[i] = fmaf(dz, X[b * d + i], acc[i]);
      acc[MLP_MAX_IN] += dz;                       // b1[j]
      acc[MLP_MAX_IN + 1] = fmaf(dy, hj, acc[MLP_MAX_IN + 1]);  // W2[j]
    }
  } else {
    for (int64_t b = tid; b < B; b += blockDim.x) {
      const float r = y[b] - t[b];
      acc[0] += 2.0f * r * invB;                   // b2
      acc[1] = fmaf(r, r * invB, acc[1]);          // loss
    }
  }
#pragma unroll
  for (int k = 0; k < MLP_MAX_IN + 2; ++k) {
    const float v = wsumf(acc[k]);
    if (l == 0) red[w][k] = v;
  }
  __syncthreads();
  if (tid < MLP_MAX_IN + 2) {
    const float v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
    if (j < H) {
      if (tid < d) g[(size_t)j * d + tid] = v;
      else if (tid == MLP_MAX_IN) g[(size_t)H * d + j] = v;
      else if (tid == MLP_MAX_IN + 1) g[(size_t)H * d + H + j] = v;
    } else {
      if (tid == 0) g[(size_t)H * d + 2 * H] = v;
      else if (tid == 1 && loss) *loss = v;
    }
  }
}

// Adam (Kingma & Ba, 2015) with bias corrections c1 = 1 - beta1^t, c2 = 1 - beta2^t.
__global__ void k_mlp_adam(float* __restrict__ p, const float* __restrict__ g,
                           float* __restrict__ m, float* __restrict__ v, int64_t P, float lr,
                           float beta1, float beta2, float eps, float c1, float c2) {
  for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < P;
       k += (int64_t)gridDim.x * blockDim.x) {
    const float gk = g[k];
    const float mk = fmaf(beta1, m[k], (1.0f - beta1) * gk);
    const float vk = fmaf(beta2, v[k], (1.0f - beta2) * gk * gk);
    m[k] = mk;
    v[k] = vk;
    p[k] -= lr * (mk / c1) / (sqrtf(vk / c2) + eps);
  }
}

// Controller decision after a PP sweep: features of the iterate from the sweep
// record (FP64: log10(rel_change_i + 1e-12), log1p(sweep), -log10(1 - fit + 1e-16)),
// rounded to FP32, the network's prediction of log10 of the right-hand-side error,
// and the decision to leave the PP phase (prediction >= log10_tau).  One wave.
__global__ __launch_bounds__(64) void k_mlp_decide(const float* __restrict__ p, int H, int N,
                                                   ppals_sweep_record* rec, int sweep,
                                                   double log10_tau) {
  const int l = threadIdx.x;
  const int d = N + 2;
  const float* W1 = p;
  const float* b1 = p + (size_t)H * d;
  const float* W2 = b1 + H;
  float xin[MLP_MAX_IN];
#pragma unroll
  for (int i = 0; i < MLP_MAX_IN; ++i) {
    double f = 0.0;
    if (i < N) f = log10(rec->rel_change[i] + 1e-12);
    else if (i == N) f = log1p((double)sweep);
    else if (i == N + 1) f = -log10(1.0 - rec->fit_est + 1e-16);
    xin[i] = (float)f;
  }
  float acc = 0.0f;
  for (int j = l; j < H; j += 64) {
    float z = b1[j];
#pragma unroll
    for (int i = 0; i < MLP_MAX_IN; ++i)
      if (i < d) z = fmaf(W1[j * d + i], xin[i], z);
    acc = fmaf(W2[j], tanhf(z), acc);
  }
  acc = wsumf(acc);
  if (l == 0) {
    const double pred = (double)(acc + W2[H]);
    rec->ctrl_pred = pred;
    rec->ctrl_leave = pred >= log10_tau ? 1 : 0;
  }
}

// Relative right-hand-side error of one mode: out[0] += sum (Mt - M)^2,
// out[1] += sum M^2 (one workgroup, fixed reduction order).
__global__ __launch_bounds__(1024) void k_rhs_err(const double* __restrict__ Mt,
                                                  const double* __restrict__ M, int64_t count,
                                                  double* out) {
  __shared__ double red[16][2];
  double a = 0.0, b = 0.0;
  for (int64_t k = threadIdx.x; k < count; k += blockDim.x) {
    const double e = Mt[k] - M[k];
    a = fma(e, e, a);
    b = fma(M[k], M[k], b);
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off);
    b += __shfl_xor(b, off);
  }
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) {
    red[w][0] = a;
    red[w][1] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double s0 = 0.0, s1 = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
      s0 += red[q][0];
      s1 += red[q][1];
    }
    out[0] = s0;
    out[1] = s1;
  }
}

// err = max over modes of sqrt(num_n / den_n) (sums laid out as N pairs).
__global__ void k_rhs_err_max(const double* sums, int N, double* err) {
  if (threadIdx.x != 0) return;
  double e = 0.0;
  for (int n = 0; n < N; ++n) {
    const double num = sums[2 * n], den = sums[2 * n + 1];
    const double r = den > 0.0 ? sqrt(num / den) : (num > 0.0 ? INFINITY : 0.0);
    e = fmax(e, r);
  }
  *err = e;
}

hipError_t launch_mlp_forward(const float* p, int d, int H, const float* X, int64_t B, float* y,
                              float* hcache, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((B + 3) / 4)), dim3(256), 0, s, p, d, H, X, B, y,
                     hcache);
  return hipGetLastError();
}
hipError_t launch_mlp_backward(const float* p, int d, int H, const float* X, const float* hcache,
                               const float* y, const float* t, int64_t B, float* g, float* loss,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_backward, dim3(H + 1), dim3(256), 0, s, p, d, H, X, hcache, y, t, B, g,
                     loss);
  return hipGetLastError();
}
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int64_t P, float lr,
                           float beta1, float beta2, float eps, float c1, float c2, hipStream_t s) {
  int64_t blocks = (P + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 1024) blocks = 1024;
  hipLaunchKernelGGL(k_mlp_adam, dim3((unsigned)blocks), dim3(256), 0, s, p, g, m, v, P, lr, beta1,
                     beta2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t launch_mlp_decide(const float* p, int H, int N, void* rec, int sweep, double log10_tau,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_decide, dim3(1), dim3(64), 0, s, p, H, N, (ppals_sweep_record*)rec,
                     sweep, log10_tau);
  return hipGetLastError();
}
hipError_t launch_rhs_err(const double* Mt, const double* M, int64_t count, double* out,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_err, dim3(1), dim3(1024), 0, s, Mt, M, count, out);
  return hipGetLastError();
}
hipError_t launch_rhs_err_max(const double* sums, int N, double* err, hipStream_t s) {
  hipLaunchKernelGGL(k_rhs_err_max, dim3(1), dim3(64), 0, s, sums, N, err);
  return hipGetLastError();
}

}  // namespace ppk
