// Column-wise (Khatri-Rao) multi-TTV contractions: the later levels of the
// dimension trees (Section 2.5: "batched matrix-vector products") and the
// first-order pairwise perturbation terms of the general PP update
// (Section 3.2.1): for every job
//
//   out[s][p][q][r] = sum_{x in split s} T[p][x][q][r] * F[x][r]
//
// T is an intermediate with the rank index fastest (FP64 or FP32), F an X x R
// FP64 matrix (a factor, a Khatri-Rao block or dA), out FP64 partial slots.
// These kernels are HBM-bound: each workgroup streams a contiguous slab of T with
// TTV_THREADS threads; when Q*R < TTV_THREADS the threads are split into G groups that
// read G consecutive x-rows at once and are reduced through LDS.  Accumulation is FP64.
#include "common.h"
#include "tail_bodies.h"
#include <algorithm>

namespace ppk {

template <typename T>
__device__ __forceinline__ double ttv_body(const T* __restrict__ src, const double* __restrict__ F,
                                           int64_t QR, int R, int r, int64_t x0, int64_t x1,
                                           int G) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int64_t x = x0;
  const int64_t step = G;
  for (; x + 3 * step < x1; x += 4 * step) {
    const double t0 = (double)src[x * QR];
    const double t1 = (double)src[(x + step) * QR];
    const double t2 = (double)src[(x + 2 * step) * QR];
    const double t3 = (double)src[(x + 3 * step) * QR];
    a0 = fma(t0, F[x * R + r], a0);
    a1 = fma(t1, F[(x + step) * R + r], a1);
    a2 = fma(t2, F[(x + 2 * step) * R + r], a2);
    a3 = fma(t3, F[(x + 3 * step) * R + r], a3);
  }
  for (; x < x1; x += step) a0 = fma((double)src[x * QR], F[x * R + r], a0);
  return (a0 + a1) + (a2 + a3);
}

__global__ __launch_bounds__(TTV_THREADS) __attribute__((amdgpu_num_vgpr(64))) void k_ttv(TtvBatch b) {
  __shared__ double red[TTV_THREADS];
  if (b.gate && *b.gate == 0) return;
  int64_t bid = blockIdx.x;
  int jid = 0;
  while (jid < b.njobs - 1 && bid >= b.job[jid].blocks) {
    bid -= b.job[jid].blocks;
    ++jid;
  }
  const TtvJob J = b.job[jid];
  const int R = b.R;
  const int64_t QR = J.Q * R;
  const int64_t jb = bid % J.jblocks;
  const int64_t rest = bid / J.jblocks;
  const int64_t p = rest % J.P;
  const int split = (int)(rest / J.P);
  const int64_t xs = (J.X + J.xsplit - 1) / J.xsplit;
  const int64_t x0 = (int64_t)split * xs;
  const int64_t x1 = min(J.X, x0 + xs);

  const int t = threadIdx.x;
  const int gi = t / J.Jb;
  const int jj = t - gi * J.Jb;
  const int64_t j = jb * J.Jb + jj;
  const bool active = gi < J.G && j < QR;
  double acc = 0.0;
  if (active && x0 < x1) {
    const int r = (int)(j % R);
    if (J.t_is_f32) {
      const float* src = (const float*)J.T + p * J.X * QR + j;
      acc = ttv_body<float>(src, J.F, QR, R, r, x0 + gi, x1, J.G);
    } else {
      const double* src = (const double*)J.T + p * J.X * QR + j;
      acc = ttv_body<double>(src, J.F, QR, R, r, x0 + gi, x1, J.G);
    }
  }
  if (J.G > 1) {
    red[t] = acc;
    __syncthreads();
    if (gi == 0 && j < QR) {
      double s = acc;
      for (int g = 1; g < J.G; ++g) s += red[g * J.Jb + jj];
      acc = s;
    }
  }
  if (gi == 0 && j < QR) J.out[(int64_t)split * J.out_split_stride + p * QR + j] = acc;
}

// Vector multi-TTV (TTV_VTHREADS threads, jobs of kinds TTV_SLAB and TTV_ROWS).  Each
// lane streams 16-byte vectors of T (VEC = 4 FP32 or 2 FP64 elements) and accumulates
// in FP64.
template <typename T> struct TtvVecT;
template <> struct TtvVecT<float> {
  static constexpr int VEC = 4;
  typedef float4 V;
  __device__ static __forceinline__ void get(const V& v, double (&o)[4]) {
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
  }
};
// Two FP32 elements per 8-byte vector (TTV_ROWS2).
struct TtvVec2F {
  static constexpr int VEC = 2;
  typedef float2 V;
  __device__ static __forceinline__ void get(const V& v, double (&o)[2]) {
    o[0] = v.x; o[1] = v.y;
  }
};
template <> struct TtvVecT<double> {
  static constexpr int VEC = 2;
  typedef double2 V;
  __device__ static __forceinline__ void get(const V& v, double (&o)[2]) {
    o[0] = v.x; o[1] = v.y;
  }
};
constexpr int TTV_U = 8;                         // vectors in flight per lane
constexpr int TTV_W = TTV_VTHREADS / 64;         // waves per workgroup

// TTV_SLAB: workgroup (pair of slabs p, p + 1; split); wave w takes iterations w, w + TTV_W,
// ... of its split, each covering S = VEC * lanes consecutive elements (a whole number of
// rank rows), so lane l always holds ranks (VEC l + c) mod R.  The weights share the
// slabs' flat index and are loaded once for both slabs.  Partial sums meet in LDS.
template <typename T>
__device__ __forceinline__ void ttv_slab(const TtvJob& J, int R, int64_t bid, double* red) {
  using TV = TtvVecT<T>;
  constexpr int VEC = TV::VEC;
  constexpr int PB = TTV_SLAB_PB;
  constexpr int U = TTV_U / PB;
  const int64_t pg = bid / J.xsplit;
  const int split = (int)(bid - pg * J.xsplit);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int L = J.lanes;
  const int64_t n = J.X * R;
  const int S = VEC * L;
  const int64_t niter = n / S;
  const int64_t per = (niter + J.xsplit - 1) / J.xsplit;
  const int64_t it0 = (int64_t)split * per, it1 = min(niter, it0 + per);
  const T* src[PB];
#pragma unroll
  for (int b = 0; b < PB; ++b) src[b] = (const T*)J.T + min(pg * PB + b, J.P - 1) * n;
  const double* F = J.F;
  double acc[PB][VEC];
#pragma unroll
  for (int b = 0; b < PB; ++b)
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[b][c] = 0.0;
  if (lane < L) {
    int64_t it = it0 + w;
    for (; it + (U - 1) * TTV_W < it1; it += U * TTV_W) {
      typename TV::V tv[U][PB];
      double fv[U][VEC];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = (it + u * TTV_W) * S + VEC * lane;
#pragma unroll
        for (int b = 0; b < PB; ++b) tv[u][b] = *reinterpret_cast<const typename TV::V*>(src[b] + e);
        if (J.f_vec) {
#pragma unroll
          for (int c = 0; c < VEC; c += 2) {
            const double2 f2 = *reinterpret_cast<const double2*>(F + e + c);
            fv[u][c] = f2.x;
            fv[u][c + 1] = f2.y;
          }
        } else {
#pragma unroll
          for (int c = 0; c < VEC; ++c) fv[u][c] = F[e + c];
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int b = 0; b < PB; ++b) {
          double t[VEC];
          TV::get(tv[u][b], t);
#pragma unroll
          for (int c = 0; c < VEC; ++c) acc[b][c] = fma(t[c], fv[u][c], acc[b][c]);
        }
    }
    for (; it < it1; it += TTV_W) {
      const int64_t e = it * S + VEC * lane;
#pragma unroll
      for (int b = 0; b < PB; ++b) {
        double t[VEC];
        TV::get(*reinterpret_cast<const typename TV::V*>(src[b] + e), t);
#pragma unroll
        for (int c = 0; c < VEC; ++c) acc[b][c] = fma(t[c], F[e + c], acc[b][c]);
      }
    }
    if (w == 0 && split == J.xsplit - 1) {  // the elements after the last whole iteration
      const int64_t e = niter * S + VEC * lane;
#pragma unroll
      for (int b = 0; b < PB; ++b)
#pragma unroll
        for (int c = 0; c < VEC; ++c)
          if (e + c < n) acc[b][c] = fma((double)src[b][e + c], F[e + c], acc[b][c]);
    }
#pragma unroll
    for (int b = 0; b < PB; ++b)
#pragma unroll
      for (int c = 0; c < VEC; ++c) red[(w * PB + b) * 256 + VEC * lane + c] = acc[b][c];
  }
  __syncthreads();
  for (int t = threadIdx.x; t < PB * R; t += TTV_VTHREADS) {
    const int b = t / R, r = t - b * R;
    const int64_t p = pg * PB + b;
    if (p < J.P) {
      double sum = 0.0;
      for (int ww = 0; ww < TTV_W; ++ww)
        for (int k = r; k < S; k += R) sum += red[(ww * PB + b) * 256 + k];
      J.out[(int64_t)split * J.out_split_stride + p * R + r] = sum;
    }
  }
}

// TTV_ROWS: workgroup (jb, p, split) covers VEC * TTV_VTHREADS consecutive j of the rows
// x in [x0, x1); F's rows x0..x1-1 are staged in LDS first.
template <typename T, typename TV = TtvVecT<T>>
__device__ __forceinline__ void ttv_rows(const TtvJob& J, int R, int64_t bid, double* fl) {
  constexpr int VEC = TV::VEC;
  const int64_t QR = J.Q * R;
  const int64_t jb = bid % J.jblocks;
  const int64_t rest = bid / J.jblocks;
  const int64_t p = rest % J.P;
  const int split = (int)(rest / J.P);
  const int64_t x0 = (int64_t)split * J.xs;
  const int64_t x1 = min(J.X, x0 + J.xs);
  const int nf = (int)((x1 - x0) * R);
  for (int i = threadIdx.x; i < nf; i += TTV_VTHREADS) fl[i] = J.F[x0 * R + i];
  __syncthreads();
  const int64_t j = (jb * TTV_VTHREADS + threadIdx.x) * VEC;
  if (j >= QR) return;
  int rc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) rc[c] = (int)((j + c) % R);
  const T* src = (const T*)J.T + p * J.X * QR + j;
  double acc[VEC];
#pragma unroll
  for (int c = 0; c < VEC; ++c) acc[c] = 0.0;
  int64_t x = x0;
  for (; x + TTV_U - 1 < x1; x += TTV_U) {
    typename TV::V tv[TTV_U];
#pragma unroll
    for (int u = 0; u < TTV_U; ++u) tv[u] = *reinterpret_cast<const typename TV::V*>(src + (x + u) * QR);
#pragma unroll
    for (int u = 0; u < TTV_U; ++u) {
      double t[VEC];
      TV::get(tv[u], t);
      const double* fr = fl + (x + u - x0) * R;
#pragma unroll
      for (int c = 0; c < VEC; ++c) acc[c] = fma(t[c], fr[rc[c]], acc[c]);
    }
  }
  for (; x < x1; ++x) {
    double t[VEC];
    TV::get(*reinterpret_cast<const typename TV::V*>(src + x * QR), t);
    const double* fr = fl + (x - x0) * R;
#pragma unroll
    for (int c = 0; c < VEC; ++c) acc[c] = fma(t[c], fr[rc[c]], acc[c]);
  }
  double* o = J.out + (int64_t)split * J.out_split_stride + p * QR + j;
#pragma unroll
  for (int c = 0; c < VEC; ++c) o[c] = acc[c];
}

__global__ __launch_bounds__(TTV_VTHREADS) void k_ttv_vec(TtvBatch b) {
  __shared__ double red[TTV_W * TTV_SLAB_PB * 256];
  extern __shared__ double fl[];
  if (b.gate && *b.gate == 0) return;
  int64_t bid = blockIdx.x;
  int jid = 0;
  while (jid < b.njobs - 1 && bid >= b.job[jid].blocks) {
    bid -= b.job[jid].blocks;
    ++jid;
  }
  const TtvJob& J = b.job[jid];
  if (J.kind == TTV_SLAB) {
    if (J.t_is_f32) ttv_slab<float>(J, b.R, bid, red);
    else ttv_slab<double>(J, b.R, bid, red);
  } else if (J.kind == TTV_ROWS2) {
    ttv_rows<float, TtvVec2F>(J, b.R, bid, fl);
  } else {
    if (J.t_is_f32) ttv_rows<float>(J, b.R, bid, fl);
    else ttv_rows<double>(J, b.R, bid, fl);
  }
}

// One launch per mode of a PP sweep for the mode's contractions, the Grams of the previous
// mode and the head of this mode, so that the solve after it depends on one kernel on one
// stream (a dependency between streams costs several microseconds each way).  Workgroups
// 0 .. ngram-1 take the Gram tiles, nsplit row ranges of each (four waves each; they are
// dispatched first, and the last range of a tile to finish adds the partial tiles); the last
// of them to finish, told by a device-scope counter that it resets, then runs the head
// from the Gamma and W tiles the others left in global memory.  With ngram == 0 (first
// mode of a sweep) workgroup 0 runs the head alone.  The other workgroups run the
// contraction jobs exactly as k_ttv_vec does.  All roles share one dynamic LDS block.
constexpr int TAIL_GRAM_WAVES = TTV_VTHREADS / 64;

template <int NM>
__global__ __launch_bounds__(TTV_VTHREADS) void k_ttv_tail(TtvBatch b, GramArgs g, HeadArgs h,
                                                           int ngram, int* ctr) {
  extern __shared__ double dyn[];
  __shared__ int last;
  const int nrole = ngram > 0 ? ngram : 1;
  // In a launch whose Gram role takes the threshold test (g.gate_out), Gram workgroup 0
  // may close the gate while the launch runs; the Gram role skips the check, so that every
  // Gram workgroup is counted (its work repeats what is already there when the gate was
  // closed before the launch, and workgroup 0 then leaves the record alone).
  const bool gram_role = ngram > 0 && (int)blockIdx.x < nrole;
  if (!(gram_role && g.gate_out) && b.gate && *b.gate == 0) return;
  if ((int)blockIdx.x < nrole) {
    if (ngram > 0) {
      double* racc = dyn;
      double* tiles = racc + GRAM_RACC(TAIL_GRAM_WAVES);
      const int nsplit = g.nsplit > 1 ? g.nsplit : 1;
      gram_body<TAIL_GRAM_WAVES, true>(g, blockIdx.x / nsplit, blockIdx.x % nsplit, racc, tiles,
                                       tiles + 256, tiles + 512);
      // The head needs only the Gamma tiles, written through with device-scope atomic
      // stores: waiting for this workgroup's stores to complete orders them before the
      // count, with no release fence (which would write back every dirty line of this
      // XCD's L2, while the contraction workgroups keep filling it).
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (threadIdx.x == 0) last = atomicAdd(ctr, 1) == ngram - 1;
      __syncthreads();
      if (!last) return;
      // every workgroup has counted: reset for the next launch (zeroed once per build),
      // at the same device scope as the counts
      if (threadIdx.x == 0) __hip_atomic_store(ctr, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    head_body<NM, true>(h, dyn, dyn + 64 * CH64_LS, dyn + 64 * CH64_LS + 128);
    return;
  }
  int64_t bid = (int64_t)blockIdx.x - nrole;
  int jid = 0;
  while (jid < b.njobs - 1 && bid >= b.job[jid].blocks) {
    bid -= b.job[jid].blocks;
    ++jid;
  }
  const TtvJob& J = b.job[jid];
  double* red = dyn;
  double* fl = dyn + TTV_W * TTV_SLAB_PB * 256;
  if (J.kind == TTV_SLAB) {
    if (J.t_is_f32) ttv_slab<float>(J, b.R, bid, red);
    else ttv_slab<double>(J, b.R, bid, red);
  } else if (J.kind == TTV_ROWS2) {
    ttv_rows<float, TtvVec2F>(J, b.R, bid, fl);
  } else {
    if (J.t_is_f32) ttv_rows<float>(J, b.R, bid, fl);
    else ttv_rows<double>(J, b.R, bid, fl);
  }
}

// out[idx] = (base ? base[idx] : 0) + sum_slots partial[slot][idx]
//            + (W ? sum_l A[y][l] W[l][r] : 0),   idx = y*R + r
__global__ __launch_bounds__(256) void k_combine(double* __restrict__ out, int64_t count, int R,
                                                 const double* __restrict__ base,
                                                 const double* __restrict__ partial, int nslots,
                                                 int64_t slot_stride, const double* __restrict__ A,
                                                 const double* __restrict__ W) {
  extern __shared__ double lw[];
  if (W) {
    for (int e = threadIdx.x; e < R * R; e += blockDim.x) lw[e] = W[e];
    __syncthreads();
  }
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = base ? base[idx] : 0.0;
    for (int k = 0; k < nslots; ++k) s += partial[(int64_t)k * slot_stride + idx];
    if (W) {
      const int64_t y = idx / R;
      const int r = (int)(idx - y * R);
      const double* ar = A + y * R;
      double v = 0.0;
      for (int l2 = 0; l2 < R; ++l2) v = fma(ar[l2], lw[l2 * R + r], v);
      s += v;
    }
    out[idx] = s;
  }
}

// Khatri-Rao block in FP64: out[k][r] = prod_f A_f[digit_f(k)][r] (first factor slowest)
__global__ void k_krp_f64(KrpDesc krp, int64_t K, double* __restrict__ out) {
  const int64_t total = K * krp.R;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int r = (int)(idx % krp.R);
    int64_t kr = idx / krp.R, dig[PP_MAXN];
    for (int f = krp.nf - 1; f >= 0; --f) {
      dig[f] = kr % krp.dim[f];
      kr /= krp.dim[f];
    }
    double v = krp.A[0][dig[0] * krp.R + r];
    for (int f = 1; f < krp.nf; ++f) v *= krp.A[f][dig[f] * krp.R + r];
    out[idx] = v;
  }
}

__global__ void k_sub(double* __restrict__ out, const double* __restrict__ a,
                      const double* __restrict__ b, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = b ? a[i] - b[i] : a[i];
}
__global__ void k_fill(double* __restrict__ out, double v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = v;
}
static int ew_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}
hipError_t launch_sub(double* out, const double* a, const double* b, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(ew_blocks(n)), dim3(256), 0, s, out, a, b, n);
  return hipGetLastError();
}
hipError_t launch_copy(double* out, const double* a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_sub, dim3(ew_blocks(n)), dim3(256), 0, s, out, a, (const double*)nullptr, n);
  return hipGetLastError();
}
// Byte-range copy: 16-byte vectors, four in flight per thread, then the last bytes one
// at a time (both pointers 16-byte aligned).
__global__ void k_copy16(uint4* __restrict__ out, const uint4* __restrict__ in, int64_t nv,
                         unsigned char* __restrict__ ob, const unsigned char* __restrict__ ib,
                         int64_t tail) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + 3 * stride < nv; i += 4 * stride) {
    const uint4 a = in[i], b = in[i + stride], c = in[i + 2 * stride], d = in[i + 3 * stride];
    out[i] = a;
    out[i + stride] = b;
    out[i + 2 * stride] = c;
    out[i + 3 * stride] = d;
  }
  for (; i < nv; i += stride) out[i] = in[i];
  if (blockIdx.x == 0)
    for (int64_t t = threadIdx.x; t < tail; t += blockDim.x) ob[t] = ib[t];
}
hipError_t launch_copy_bytes(void* out, const void* in, size_t bytes, hipStream_t s) {
  if ((((uintptr_t)out) | ((uintptr_t)in)) & 15) return hipErrorInvalidValue;
  const int64_t nv = (int64_t)(bytes / 16), tail = (int64_t)(bytes % 16);
  int64_t blocks = (nv / 4 + 255) / 256;
  blocks = blocks < 1 ? 1 : (blocks > 8192 ? 8192 : blocks);
  hipLaunchKernelGGL(k_copy16, dim3((unsigned)blocks), dim3(256), 0, s, (uint4*)out,
                     (const uint4*)in, nv, (unsigned char*)out + nv * 16,
                     (const unsigned char*)in + nv * 16, tail);
  return hipGetLastError();
}
hipError_t launch_fill(double* out, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_fill, dim3(ew_blocks(n)), dim3(256), 0, s, out, v, n);
  return hipGetLastError();
}

// Jobs of the scalar kind go to k_ttv, the others to k_ttv_vec (one launch each).
hipError_t launch_ttv(const TtvBatch& b, hipStream_t s) {
  TtvBatch sb = b, vb = b;
  sb.njobs = vb.njobs = 0;
  int64_t stotal = 0, vtotal = 0;
  size_t lds = 0;
  for (int i = 0; i < b.njobs; ++i) {
    const TtvJob& J = b.job[i];
    if (J.blocks <= 0) continue;
    if (J.kind == TTV_SCALAR) {
      sb.job[sb.njobs++] = J;
      stotal += J.blocks;
    } else {
      if ((uintptr_t)J.T % 16 != 0) return hipErrorInvalidValue;  // vector loads of T
      TtvJob& V = vb.job[vb.njobs++];
      V = J;
      V.f_vec = (uintptr_t)J.F % 16 == 0;
      vtotal += J.blocks;
      if (J.kind == TTV_ROWS || J.kind == TTV_ROWS2)
        lds = std::max(lds, (size_t)J.xs * b.R * sizeof(double));
    }
  }
  if (stotal > 0) {
    hipLaunchKernelGGL(k_ttv, dim3((unsigned)stotal), dim3(TTV_THREADS), 0, s, sb);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (vtotal > 0) {
    if (lds > 65536) {
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ttv_vec),
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_ttv_vec, dim3((unsigned)vtotal), dim3(TTV_VTHREADS), lds, s, vb);
    return hipGetLastError();
  }
  return hipSuccess;
}

bool ttv_tail_fusable(const TtvBatch& b) {
  if (b.R > 64) return false;
  for (int i = 0; i < b.njobs; ++i) {
    const TtvJob& J = b.job[i];
    if (J.blocks <= 0) continue;
    if (J.kind == TTV_SCALAR || (uintptr_t)J.T % 16 != 0) return false;
  }
  return true;
}

hipError_t launch_ttv_tail(const TtvBatch& b, const GramArgs* g, const HeadArgs& h, int* ctr,
                           hipStream_t s) {
  if (!ttv_tail_fusable(b) || h.R != b.R || h.N < 2 || h.N > PP_MAXN) return hipErrorInvalidValue;
  TtvBatch vb = b;
  vb.njobs = 0;
  int64_t vtotal = 0;
  size_t ttv_lds = (size_t)TTV_W * TTV_SLAB_PB * 256;
  size_t fl = 0;
  for (int i = 0; i < b.njobs; ++i) {
    const TtvJob& J = b.job[i];
    if (J.blocks <= 0) continue;
    TtvJob& V = vb.job[vb.njobs++];
    V = J;
    V.f_vec = (uintptr_t)J.F % 16 == 0;
    vtotal += J.blocks;
    if (J.kind == TTV_ROWS || J.kind == TTV_ROWS2) fl = std::max(fl, (size_t)J.xs * b.R);
  }
  const int NBR = (b.R + 15) / 16;
  const int ngram = g ? NBR * NBR * (g->nsplit > 1 ? g->nsplit : 1) : 0;
  if (g && g->nsplit > 1 && (!g->gpart || !g->gctr)) return hipErrorInvalidValue;
  const size_t gram_lds = (size_t)GRAM_RACC(TAIL_GRAM_WAVES) + 512 +
                          (g && g->gamma_out ? (size_t)std::max(1, g->N - 2) * 512 : 0);
  const size_t lds = std::max({ttv_lds + fl, gram_lds, (size_t)HEAD_LDS}) * sizeof(double);
  GramArgs ga{};
  if (g) ga = *g;
  const dim3 grid((unsigned)((ngram > 0 ? ngram : 1) + vtotal)), block(TTV_VTHREADS);
#define PPK_TAIL_CASE(NMV)                                                                        \
  case NMV: {                                                                                     \
    if (lds > 65536) {                                                                            \
      hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_ttv_tail<NMV>),          \
                                         hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);   \
      if (e != hipSuccess) return e;                                                              \
    }                                                                                             \
    hipLaunchKernelGGL(k_ttv_tail<NMV>, grid, block, lds, s, vb, ga, h, ngram, ctr);              \
    break;                                                                                        \
  }
  switch (h.N) {
    PPK_TAIL_CASE(2) PPK_TAIL_CASE(3) PPK_TAIL_CASE(4) PPK_TAIL_CASE(5)
    PPK_TAIL_CASE(6) PPK_TAIL_CASE(7) PPK_TAIL_CASE(8)
  }
#undef PPK_TAIL_CASE
  return hipGetLastError();
}

hipError_t launch_combine(double* out, int64_t count, int R, const double* base,
                          const double* partial, int nslots, int64_t slot_stride, const double* A,
                          const double* W, hipStream_t s) {
  int64_t blocks = (count + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  size_t lds = W ? (size_t)R * R * sizeof(double) : 0;
  if (lds > 65536) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_combine),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(256), lds, s, out, count, R, base,
                     partial, nslots, slot_stride, A, W);
  return hipGetLastError();
}

hipError_t launch_krp_f64(const KrpDesc& krp, int64_t K, double* out, hipStream_t s) {
  int64_t total = K * krp.R;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_krp_f64, dim3((unsigned)blocks), dim3(256), 0, s, krp, K, out);
  return hipGetLastError();
}

}  // namespace ppk
