// First-level contraction of the dimension trees (Section 2.5): the input tensor X
// contracted with one factor matrix (or with the Khatri-Rao product of a block of
// factors) as a dense GEMM on the gfx950 matrix cores.
//
//   C[g][r] = sum_k X[addr(g, k)] * B[k][r],   g in [0, M), k in [0, K), r in [0, R)
//   addr(g, k) = (g / Q) * K * Q + k * Q + (g % Q)
//
// X is viewed as P x K x Q (P*Q = M); the output keeps the uncontracted modes in
// increasing order with the rank index fastest.  Q == 1 means the contracted block
// is the fastest-varying one (rows of X are K-contiguous); otherwise consecutive g
// are contiguous in memory for a fixed k.
//
// Tiling: a 256-thread workgroup (4 waves of 64) owns BM consecutive rows g and
// 16*NB columns; each wave owns 16*MB rows.  MFMA shapes: f64 16x16x4, f32 16x16x4,
// bf16 16x16x32 with f32 accumulation.  B (prepared by k_prep_operand in an
// MFMA-ready order) is staged through LDS in chunks of KC k-values, double buffered;
// X streams from HBM straight into registers one chunk ahead.
#include "common.h"

namespace ppk {

template <int DT> struct L1T;
template <> struct L1T<DT_F64> {
  using T = double; using Acc = double; using V = d4;
  static constexpr int KSTEP = 4, KC = 32, E = 1, NSTEP = 8, VW = 2;
};
template <> struct L1T<DT_F32> {
  using T = float; using Acc = float; using V = f4;
  static constexpr int KSTEP = 4, KC = 32, E = 1, NSTEP = 8, VW = 4;
};
template <> struct L1T<DT_BF16> {
  using T = uint16_t; using Acc = float; using V = f4;
  static constexpr int KSTEP = 32, KC = 64, E = 8, NSTEP = 2, VW = 8;
};

typedef double dv2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<double> { typedef dv2 type; static constexpr int n = 2; };
template <> struct Vec16<float> { typedef f4 type; static constexpr int n = 4; };

__device__ __forceinline__ uint32_t pack2(uint16_t lo, uint16_t hi) {
  return (uint32_t)lo | ((uint32_t)hi << 16);
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return 0x7FC0;  // NaN
  uint32_t lsb = (u >> 16) & 1u;
  return (uint16_t)((u + 0x7FFFu + lsb) >> 16);
}

// ---------------------------------------------------------------------------
// Operand preparation: B (Khatri-Rao product of nf factors, FP64 math) converted to
// the contraction type and written in the MFMA-ready order
//   [slice][chunk][t][c][lane 0..63][e 0..E-1]
// lane = j + 16*kk; column = slice*16*NB + 16*c + j; k within the chunk:
//   f64/f32, natural order:   k = 4*t + kk
//   f64/f32, K-contiguous X:  k = 8*kk + t   (each lane streams 8 consecutive k)
//   bf16:                     k = 32*t + 8*kk + e
// Entries with k >= K or column >= R are zero.
// ---------------------------------------------------------------------------
template <int DT>
__global__ void k_prep_operand(KrpDesc krp, Level1Geom g, typename L1T<DT>::T* __restrict__ out) {
  using TR = L1T<DT>;
  const int64_t nchunk = g.Kpad / TR::KC;
  const int64_t per_chunk = (int64_t)TR::NSTEP * g.NB * 64 * TR::E;
  const int64_t total = (int64_t)g.nslices * nchunk * per_chunk;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    int64_t rem = idx;
    const int e = (int)(rem % TR::E); rem /= TR::E;
    const int lane = (int)(rem % 64); rem /= 64;
    const int c = (int)(rem % g.NB); rem /= g.NB;
    const int t = (int)(rem % TR::NSTEP); rem /= TR::NSTEP;
    const int64_t chunk = rem % nchunk;
    const int slice = (int)(rem / nchunk);
    const int j = lane % 16, kk = lane / 16;
    int kl;
    if (DT == DT_BF16) kl = 32 * t + 8 * kk + e;
    else kl = g.kc_mode ? (8 * kk + t) : (4 * t + kk);
    const int64_t k = chunk * TR::KC + kl;
    const int col = slice * 16 * g.NB + 16 * c + j;
    double v = 0.0;
    if (k < g.K && col < g.R) {
      int64_t kr = k, dig[PP_MAXN];
      for (int f = krp.nf - 1; f >= 0; --f) {
        dig[f] = kr % krp.dim[f];
        kr /= krp.dim[f];
      }
      v = krp.A[0][dig[0] * krp.R + col];
      for (int f = 1; f < krp.nf; ++f) v *= krp.A[f][dig[f] * krp.R + col];
    }
    if (DT == DT_F64) out[idx] = (typename TR::T)v;
    else if (DT == DT_F32) out[idx] = (typename TR::T)(float)v;
    else out[idx] = (typename TR::T)f32_to_bf16_rne((float)v);
  }
}

// The Khatri-Rao entries are formed as ((a_1 a_2) a_3) ..., first factor first, in FP64.

// ---------------------------------------------------------------------------
// MFMA wrappers
// ---------------------------------------------------------------------------
__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// 16 independent 4x4x1 outer products (block l/4: rows from lanes 4(l/4)..+3 of a, columns
// from the same lanes of b; register v of lane l holds row v, column l%4 of its block)
__device__ __forceinline__ f4 mfma_tail(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_4x4x1f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(bf16x8 a, bf16x8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Row of accumulator register r for lane l in a 16x16 output block.
template <int DT>
__device__ __forceinline__ int acc_row(int l, int r) {
  return DT == DT_F64 ? (4 * r + (l >> 4)) : (4 * (l >> 4) + r);
}

// Copy one B chunk global -> registers -> LDS: NVEC 16-byte vectors per chunk,
// thread t moves vectors t, t + 256, ...
template <int NVEC>
struct BStage {
  static constexpr int PER = (NVEC + 255) / 256;
  uint4 v[PER > 0 ? PER : 1];
  __device__ __forceinline__ void load(const uint4* __restrict__ src) {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int i = (int)threadIdx.x + 256 * s;
      v[s] = (NVEC % 256 == 0 || i < NVEC) ? src[i] : make_uint4(0, 0, 0, 0);
    }
  }
  __device__ __forceinline__ void store(uint4* dst) const {
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int i = (int)threadIdx.x + 256 * s;
      if (NVEC % 256 == 0 || i < NVEC) dst[i] = v[s];
    }
  }
};

// ---------------------------------------------------------------------------
// FP64 / FP32 register-path kernel.
//   KCM: rows K-contiguous (Q == 1): each lane streams 8 consecutive k of one row.
//   !KCM, VEC: rows contiguous for fixed k; one 16-byte load gives VW = MB rows.
//   !KCM, !VEC: scalar loads.
// ---------------------------------------------------------------------------
// Zeros read in place of X entries outside the tensor (64 bytes covers the widest read).
__device__ __attribute__((aligned(16))) double l1_zero[8];

// n / d for n < 2^31 with the precomputed multiplier of d (Level1Geom).
__device__ __forceinline__ uint32_t l1_magic_div(uint32_t n, uint64_t mag, int sh) {
  return (uint32_t)(((uint64_t)n * mag) >> (32 + sh));
}

template <int DT, int MB, int NB, bool KCM, bool VEC, bool TAIL = false, bool STR = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(DT == DT_F32 && (KCM || VEC) ? 3 : 1))) void k_level1_reg(const typename L1T<DT>::T* __restrict__ X,
                                                    const typename L1T<DT>::T* __restrict__ B,
                                                    Level1Geom g,
                                                    typename L1T<DT>::Acc* __restrict__ C,
                                                    int64_t c_split_stride) {
  using TR = L1T<DT>;
  using T = typename TR::T;
  using V = typename TR::V;
  constexpr int NSTEP = TR::NSTEP;  // 8
  constexpr int KC = TR::KC;        // 32
  constexpr int BM = 4 * 16 * MB;
  constexpr int CHUNK_ELEMS = KC * 16 * NB;
  static_assert(!( !KCM && VEC) || MB == TR::VW, "vector path needs MB == VW");
  static_assert(!STR || (!KCM && !VEC && !TAIL), "strided addressing uses the scalar loads");
  __shared__ __attribute__((aligned(16))) T ldsB[2][CHUNK_ELEMS];

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, i = l & 15, kk = l >> 4;
  const int64_t g0w = (int64_t)blockIdx.x * BM + (int64_t)w * 16 * MB;
  const int slice = blockIdx.y;
  const int z = blockIdx.z;
  const int64_t kb0 = (int64_t)z * g.kchunk;
  const int64_t kb1 = min(g.K, kb0 + g.kchunk);
  if (kb0 >= kb1) return;
  const int nch = (int)((kb1 - kb0 + KC - 1) / KC);
  const int64_t nchunk_tot = g.Kpad / KC;
  const uint4* Bslice = reinterpret_cast<const uint4*>(B + ((int64_t)slice * nchunk_tot) * CHUNK_ELEMS);
  constexpr int NVEC = CHUNK_ELEMS * (int)sizeof(T) / 16;
  const int64_t gM = g.M, gK = g.K, gQ = g.Q;
  const int gR = g.R;

  // Per-lane row bases.
  //   KCM:            m-block b -> row g0w + 16 b + i, base g*K
  //   !KCM && VEC:    rows g0w + VW*i + b (b < VW), base of the vector start
  //   !KCM && !VEC:   m-block b -> row g0w + 16 b + i, base p*K*Q + q
  int64_t base[MB];
  bool rowok[MB];
  if (KCM) {
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int64_t gr = g0w + 16 * b + i;
      rowok[b] = gr < gM;
      base[b] = rowok[b] ? gr * gK : 0;
    }
  } else if (VEC) {
    const int64_t gv = g0w + (int64_t)TR::VW * i;
    rowok[0] = gv < gM;
    const int64_t p = gv / gQ, q = gv - p * gQ;
    base[0] = rowok[0] ? p * gK * gQ + q : 0;
#pragma unroll
    for (int b = 1; b < MB; ++b) { rowok[b] = rowok[0]; base[b] = base[0]; }
  } else if (STR) {
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int64_t gr = g0w + 16 * b + i;
      rowok[b] = gr < gM;
      const int64_t q = gr / g.mrad2, m2 = gr - q * g.mrad2;
      const int64_t m0 = q / g.mrad, m1 = q - m0 * g.mrad;
      base[b] = rowok[b] ? m0 * g.ms0 + m1 * g.ms1 + m2 * g.ms2 : 0;
    }
  } else {
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int64_t gr = g0w + 16 * b + i;
      rowok[b] = gr < gM;
      const int64_t p = gr / gQ, q = gr - p * gQ;
      base[b] = rowok[b] ? p * gK * gQ + q : 0;
    }
  }

  // X registers for one chunk: xr[b][t] = A-operand of m-block b at step t.
  T xc[MB][NSTEP], xn[MB][NSTEP];

  // Loads are unconditional: an invalid row or k reads zeros from l1_zero instead.  A
  // guarded load becomes a branch, around which the number of outstanding loads is not
  // known, and a zero select right after the load makes it wait there; either way the
  // wait for the current chunk would also wait for the next chunk's prefetch.
  const T* zero = reinterpret_cast<const T*>(l1_zero);
  auto load_x = [&](T (&xr)[MB][NSTEP], int64_t kbase) {
    if (KCM) {
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        const int64_t k0 = kbase + 8 * kk;
        if (VEC) {
          const bool ok = rowok[b] && (k0 < kb1);
          using VT = typename Vec16<T>::type;
          constexpr int VN = Vec16<T>::n;
          const VT* src = reinterpret_cast<const VT*>(ok ? X + base[b] + k0 : zero);
#pragma unroll
          for (int v = 0; v < 8 / VN; ++v) {
            const VT val = src[v];
#pragma unroll
            for (int e = 0; e < VN; ++e) xr[b][v * VN + e] = val[e];
          }
        } else {
#pragma unroll
          for (int t = 0; t < NSTEP; ++t) {
            const int64_t k = k0 + t;
            xr[b][t] = *((rowok[b] && k < kb1) ? X + base[b] + k : zero);
          }
        }
      }
    } else if (VEC) {
#pragma unroll
      for (int t = 0; t < NSTEP; ++t) {
        const int64_t k = kbase + 4 * t + kk;
        using VT = typename Vec16<T>::type;
        const VT val = *reinterpret_cast<const VT*>((rowok[0] && k < kb1) ? X + base[0] + k * gQ : zero);
#pragma unroll
        for (int b = 0; b < MB; ++b) xr[b][t] = val[b];
      }
    } else if (STR) {
#pragma unroll
      for (int t = 0; t < NSTEP; ++t) {
        const int64_t k = kbase + 4 * t + kk;
        const uint32_t ku = (uint32_t)k;
        const uint32_t q2 = l1_magic_div(ku, g.kmag2, g.ksh2);
        const uint32_t k2 = ku - q2 * g.kr2;
        const uint32_t k0 = l1_magic_div(q2, g.kmag1, g.ksh1);
        const uint32_t k1 = q2 - k0 * g.kr1;
        const int64_t koff = (int64_t)k0 * g.ks0 + (int64_t)k1 * g.ks1 + (int64_t)k2 * g.ks2;
#pragma unroll
        for (int b = 0; b < MB; ++b) xr[b][t] = *((rowok[b] && k < kb1) ? X + base[b] + koff : zero);
      }
    } else {
#pragma unroll
      for (int t = 0; t < NSTEP; ++t) {
        const int64_t k = kbase + 4 * t + kk;
#pragma unroll
        for (int b = 0; b < MB; ++b) xr[b][t] = *((rowok[b] && k < kb1) ? X + base[b] + k * gQ : zero);
      }
    }
  };

  // TAIL (FP32, at most four useful columns in the last 16-column block): the last block
  // runs on the 4x4x1 matrix-core shape (16 blocks of 4 x 4 outer products, the same
  // MACs per cycle) with the X register of the 16x16x4 steps as its B operand: lane l
  // holds X[row(l%16)][k(l/16)], so block l/4 multiplies rows 4((l/4)%4) + 0..3 of the
  // 16-row block by the four tail columns at the k of group l/16.  The four k groups are
  // summed across lanes at the end.  This cuts the matrix-core time of the last block by
  // a factor of four.
  constexpr int NBF = TAIL ? NB - 1 : NB;  // blocks on the 16x16x4 shape
  static_assert(!TAIL || DT == DT_F32, "tail path is FP32 only");
  V acc[MB][NB];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[b][c] = V{0, 0, 0, 0};

  // Prologue: chunk 0 of B into LDS buffer 0, X chunk 0 into the prefetch registers.
  // Each chunk first takes the prefetched X (xc = xn: the only wait for global loads
  // before the matrix cores start) and then issues the next chunk's B and X loads, B
  // first, so that storing B into LDS after the MFMAs waits for B alone.
  const int64_t chunk0 = kb0 / KC;
  // FP32: B chunks go from global memory straight into LDS (16 bytes per lane, no
  // registers), which keeps the kernel within 168 registers per lane, three waves per
  // SIMD: wave w moves vectors 64 w .. 64 w + 63 of each 256-vector round, which land at
  // consecutive LDS addresses from a wave-uniform base.  FP64 (two waves per SIMD either
  // way) stages B through registers, stored to LDS after the chunk's matrix-core work.
  constexpr bool DMA_B = DT == DT_F32;
  BStage<DMA_B ? 0 : NVEC> st;
  auto load_b = [&](int64_t chunk, int bufi) {
    if constexpr (DMA_B) {
#pragma unroll
      for (int r = 0; r < (NVEC + 255) / 256; ++r) {
        const int v = 256 * r + tid;
        if (NVEC % 256 == 0 || v < NVEC)
          __builtin_amdgcn_global_load_lds(
              (const void*)(Bslice + chunk * NVEC + v),
              (__attribute__((address_space(3))) void*)(reinterpret_cast<uint4*>(ldsB[bufi]) + 256 * r + 64 * w),
              16, 0, 0);
      }
    } else {
      st.load(Bslice + chunk * NVEC);
    }
  };
  load_b(chunk0, 0);
  if constexpr (!DMA_B) st.store(reinterpret_cast<uint4*>(ldsB[0]));
  load_x(xn, kb0);
  if constexpr (DMA_B) __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();

  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int t = 0; t < NSTEP; ++t) xc[b][t] = xn[b][t];
    if (more) {
      load_b(chunk0 + ch + 1, buf ^ 1);
      load_x(xn, kb0 + (int64_t)(ch + 1) * KC);
    }
    const T* lb = ldsB[buf];
#pragma unroll
    for (int t = 0; t < NSTEP; ++t) {
      T bop[NB];
#pragma unroll
      for (int c = 0; c < NBF; ++c) bop[c] = lb[(t * NB + c) * 64 + l];
      // tail: lane l takes column 16 (NB - 1) + l%4 of its own k group
      if constexpr (TAIL) bop[NB - 1] = lb[(t * NB + NB - 1) * 64 + (l & 48) + (l & 3)];
#pragma unroll
      for (int b = 0; b < MB; ++b) {
#pragma unroll
        for (int c = 0; c < NBF; ++c) acc[b][c] = mfma(xc[b][t], bop[c], acc[b][c]);
        if constexpr (TAIL) acc[b][NB - 1] = mfma_tail(bop[NB - 1], xc[b][t], acc[b][NB - 1]);
      }
    }
    if constexpr (DMA_B) {
      // the next chunk's B (and X) loads are complete before any wave reads that buffer
      __builtin_amdgcn_s_waitcnt(0);
    } else {
      if (more) st.store(reinterpret_cast<uint4*>(ldsB[buf ^ 1]));
    }
    __syncthreads();
  }

  // Store: accumulator register r of lane l holds row acc_row(l, r), column l % 16.
  typename TR::Acc* Cz = C + (int64_t)z * c_split_stride;
  if constexpr (TAIL) {
    // tail block: register v of lane l holds column 16 (NB - 1) + v of row l%16 (in the
    // row order of the 16x16x4 operand), partial over k group l/16
#pragma unroll
    for (int b = 0; b < MB; ++b)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        float sv = acc[b][NB - 1][v];
        sv += __shfl_xor(sv, 16);
        sv += __shfl_xor(sv, 32);
        const int col = slice * 16 * NB + 16 * (NB - 1) + v;
        const int64_t gr = (!KCM && VEC) ? (g0w + (int64_t)TR::VW * i + b) : (g0w + 16 * b + i);
        if (l < 16 && col < gR && gr < gM) Cz[gr * gR + col] = sv;
      }
  }
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NBF; ++c) {
      const int col = slice * 16 * NB + 16 * c + i;
      if (col >= gR) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rho = acc_row<DT>(l, r);
        const int64_t gr = (!KCM && VEC) ? (g0w + (int64_t)TR::VW * rho + b) : (g0w + 16 * b + rho);
        if (gr < gM) Cz[gr * gR + col] = acc[b][c][r];
      }
    }
}

// ---------------------------------------------------------------------------
// BF16 kernel.  K-contiguous rows: each lane loads its 8 consecutive bf16 per
// step directly (the native 16x16x32 operand order).  Otherwise X tiles pass
// through LDS ([k][BM] with a padded stride) and each lane gathers its 8 k-values.
// ---------------------------------------------------------------------------
template <int MB, int NB, bool KCM, bool VEC>
__global__ __launch_bounds__(256) void k_level1_bf16(const uint16_t* __restrict__ X,
                                                     const uint16_t* __restrict__ B,
                                                     Level1Geom g, float* __restrict__ C,
                                                     int64_t c_split_stride) {
  constexpr int KC = 64, NSTEP = 2;
  constexpr int BM = 4 * 16 * MB;
  constexpr int CHUNK_ELEMS = KC * 16 * NB;
  constexpr int XS = BM + 8;  // padded LDS row stride (elements) of the X tile
  __shared__ __attribute__((aligned(16))) uint16_t ldsB[2][CHUNK_ELEMS];
  __shared__ __attribute__((aligned(16))) uint16_t ldsX[KCM ? 1 : 2][KCM ? 8 : KC * XS];

  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63, i = l & 15, kk = l >> 4;
  const int64_t g0 = (int64_t)blockIdx.x * BM;
  const int64_t g0w = g0 + (int64_t)w * 16 * MB;
  const int slice = blockIdx.y;
  const int z = blockIdx.z;
  const int64_t kb0 = (int64_t)z * g.kchunk;
  const int64_t kb1 = min(g.K, kb0 + g.kchunk);
  if (kb0 >= kb1) return;
  const int nch = (int)((kb1 - kb0 + KC - 1) / KC);
  const int64_t nchunk_tot = g.Kpad / KC;
  const uint4* Bslice = reinterpret_cast<const uint4*>(B + ((int64_t)slice * nchunk_tot) * CHUNK_ELEMS);
  constexpr int NVEC = CHUNK_ELEMS * 2 / 16;
  const int64_t gM = g.M, gK = g.K, gQ = g.Q;
  const int gR = g.R;

  // K-contiguous: registers hold xr[b][t] = 8 bf16 (one uint4).
  // Otherwise: registers hold this thread's share of the next X tile.
  constexpr int XV = KCM ? (MB * NSTEP) : (KC * BM / 8 / 256);  // uint4 per thread
  uint4 xc[XV], xn[XV];

  int64_t kbase_row[MB];
  bool rowok[MB];
  if (KCM) {
#pragma unroll
    for (int b = 0; b < MB; ++b) {
      const int64_t gr = g0w + 16 * b + i;
      rowok[b] = gr < gM;
      kbase_row[b] = rowok[b] ? gr * gK : 0;
    }
  }

  auto load_x = [&](uint4 (&xr)[XV], int64_t kbase) {
    if (KCM) {
#pragma unroll
      for (int b = 0; b < MB; ++b)
#pragma unroll
        for (int t = 0; t < NSTEP; ++t) {
          const int64_t k0 = kbase + 32 * t + 8 * kk;
          if (VEC) {
            const bool ok = rowok[b] && k0 < kb1;
            xr[b * NSTEP + t] = ok ? *reinterpret_cast<const uint4*>(X + kbase_row[b] + k0)
                                   : make_uint4(0, 0, 0, 0);
          } else {
            uint16_t h[8];
#pragma unroll
            for (int e = 0; e < 8; ++e)
              h[e] = (rowok[b] && k0 + e < kb1) ? X[kbase_row[b] + k0 + e] : (uint16_t)0;
            xr[b * NSTEP + t] = make_uint4(pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]),
                                           pack2(h[6], h[7]));
          }
        }
    } else {
      // tile rows k (KC of them) x BM consecutive g; vector v covers 8 consecutive g
#pragma unroll
      for (int s = 0; s < XV; ++s) {
        const int v = tid + 256 * s;
        const int krow = v / (BM / 8);
        const int gcol = (v % (BM / 8)) * 8;
        const int64_t k = kbase + krow;
        const int64_t gv = g0 + gcol;
        if (VEC) {
          const bool ok = (gv < gM) && (k < kb1);
          const int64_t p = gv / gQ, q = gv - p * gQ;
          xr[s] = ok ? *reinterpret_cast<const uint4*>(X + p * gK * gQ + k * gQ + q)
                     : make_uint4(0, 0, 0, 0);
        } else {
          uint16_t h[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int64_t ge = gv + e;
            const int64_t p = ge / gQ, q = ge - p * gQ;
            h[e] = (ge < gM && k < kb1) ? X[p * gK * gQ + k * gQ + q] : (uint16_t)0;
          }
          xr[s] = make_uint4(pack2(h[0], h[1]), pack2(h[2], h[3]), pack2(h[4], h[5]),
                             pack2(h[6], h[7]));
        }
      }
    }
  };
  auto store_xtile = [&](const uint4 (&xr)[XV], int buf) {
    if (!KCM) {
#pragma unroll
      for (int s = 0; s < XV; ++s) {
        const int v = tid + 256 * s;
        const int krow = v / (BM / 8);
        const int gcol = (v % (BM / 8)) * 8;
        *reinterpret_cast<uint4*>(&ldsX[buf][krow * XS + gcol]) = xr[s];
      }
    }
  };

  f4 acc[MB][NB];
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NB; ++c) acc[b][c] = f4{0, 0, 0, 0};

  const int64_t chunk0 = kb0 / KC;
  BStage<NVEC> st;
  st.load(Bslice + chunk0 * NVEC);
  st.store(reinterpret_cast<uint4*>(ldsB[0]));
  load_x(xc, kb0);
  store_xtile(xc, 0);
  __syncthreads();

  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    const bool more = ch + 1 < nch;
    if (more) {
      load_x(xn, kb0 + (int64_t)(ch + 1) * KC);
      st.load(Bslice + (chunk0 + ch + 1) * NVEC);
    }
    const uint16_t* lb = ldsB[buf];
#pragma unroll
    for (int t = 0; t < NSTEP; ++t) {
      bf16x8 bop[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        bop[c] = __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4*>(&lb[((t * NB + c) * 64 + l) * 8]));
#pragma unroll
      for (int b = 0; b < MB; ++b) {
        bf16x8 aop;
        if (KCM) {
          aop = __builtin_bit_cast(bf16x8, xc[b * NSTEP + t]);
        } else {
          const uint16_t* lx = ldsX[buf];
          const int rho = w * 16 * MB + 16 * b + i;
          const uint16_t* col = lx + (32 * t + 8 * kk) * XS + rho;
          const uint4 packed = make_uint4(pack2(col[0], col[XS]), pack2(col[2 * XS], col[3 * XS]),
                                          pack2(col[4 * XS], col[5 * XS]),
                                          pack2(col[6 * XS], col[7 * XS]));
          aop = __builtin_bit_cast(bf16x8, packed);
        }
#pragma unroll
        for (int c = 0; c < NB; ++c) acc[b][c] = mfma(aop, bop[c], acc[b][c]);
      }
    }
    if (more) {
      st.store(reinterpret_cast<uint4*>(ldsB[buf ^ 1]));
      store_xtile(xn, buf ^ 1);
    }
    __syncthreads();
    if (more && KCM) {
#pragma unroll
      for (int s = 0; s < XV; ++s) xc[s] = xn[s];
    }
  }

  float* Cz = C + (int64_t)z * c_split_stride;
#pragma unroll
  for (int b = 0; b < MB; ++b)
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      const int col = slice * 16 * NB + 16 * c + i;
      if (col >= gR) continue;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rho = 4 * (l >> 4) + r;
        const int64_t gr = g0w + 16 * b + rho;
        if (gr < gM) Cz[gr * gR + col] = acc[b][c][r];
      }
    }
}

// ---------------------------------------------------------------------------
// Split-K reduction: out[i] = sum_s partial[s][i] (in the accumulation type)
// ---------------------------------------------------------------------------
template <typename TO, typename TP>
__global__ void k_reduce_splits(TO* __restrict__ out, const TP* __restrict__ part, int nsplit,
                                int64_t count) {
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < count;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += (double)part[(int64_t)k * count + idx];
    out[idx] = (TO)s;
  }
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline int grid_for(int64_t n, int per = 256, int cap = 8192) {
  int64_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (int)b;
}

hipError_t launch_prep_operand(const KrpDesc& krp, const Level1Geom& g, int dt, void* out,
                               hipStream_t s) {
  int64_t total = (int64_t)g.nslices * g.Kpad * 16 * g.NB;
  dim3 grid(grid_for(total)), block(256);
  if (dt == DT_F64) hipLaunchKernelGGL(k_prep_operand<DT_F64>, grid, block, 0, s, krp, g, (double*)out);
  else if (dt == DT_F32) hipLaunchKernelGGL(k_prep_operand<DT_F32>, grid, block, 0, s, krp, g, (float*)out);
  else hipLaunchKernelGGL(k_prep_operand<DT_BF16>, grid, block, 0, s, krp, g, (uint16_t*)out);
  return hipGetLastError();
}

template <int DT, int MB, bool KCM, bool VEC>
static void launch_reg_nb(const void* X, const void* B, const Level1Geom& g, void* C,
                          int64_t stride, hipStream_t s) {
  using TR = L1T<DT>;
  using T = typename TR::T;
  using Acc = typename TR::Acc;
  constexpr int BM = 4 * 16 * MB;
  dim3 grid((unsigned)((g.M + BM - 1) / BM), g.nslices, g.ksplit), block(256);
  // FP32 with one column slice whose last 16-column block holds 1..4 useful columns
  if constexpr (DT == DT_F32) {
    const int rem = g.R - 16 * (g.NB - 1);
    if (g.nslices == 1 && g.NB >= 2 && rem >= 1 && rem <= 4) {
      switch (g.NB) {
        case 2: hipLaunchKernelGGL((k_level1_reg<DT, MB, 2, KCM, VEC, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); return;
        case 3: hipLaunchKernelGGL((k_level1_reg<DT, MB, 3, KCM, VEC, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); return;
        default: hipLaunchKernelGGL((k_level1_reg<DT, MB, 4, KCM, VEC, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); return;
      }
    }
  }
  switch (g.NB) {
    case 1: hipLaunchKernelGGL((k_level1_reg<DT, MB, 1, KCM, VEC>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
    case 2: hipLaunchKernelGGL((k_level1_reg<DT, MB, 2, KCM, VEC>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
    case 3: hipLaunchKernelGGL((k_level1_reg<DT, MB, 3, KCM, VEC>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
    default: hipLaunchKernelGGL((k_level1_reg<DT, MB, 4, KCM, VEC>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
  }
}

// Strided addressing (direct operator build): scalar loads, no tail shape.
template <int DT, int MB>
static void launch_reg_str(const void* X, const void* B, const Level1Geom& g, void* C,
                           int64_t stride, hipStream_t s) {
  using TR = L1T<DT>;
  using T = typename TR::T;
  using Acc = typename TR::Acc;
  constexpr int BM = 4 * 16 * MB;
  dim3 grid((unsigned)((g.M + BM - 1) / BM), g.nslices, g.ksplit), block(256);
  switch (g.NB) {
    case 1: hipLaunchKernelGGL((k_level1_reg<DT, MB, 1, false, false, false, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
    case 2: hipLaunchKernelGGL((k_level1_reg<DT, MB, 2, false, false, false, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
    case 3: hipLaunchKernelGGL((k_level1_reg<DT, MB, 3, false, false, false, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
    default: hipLaunchKernelGGL((k_level1_reg<DT, MB, 4, false, false, false, true>), grid, block, 0, s, (const T*)X, (const T*)B, g, (Acc*)C, stride); break;
  }
}

template <int MB, bool KCM, bool VEC>
static void launch_bf16_nb(const void* X, const void* B, const Level1Geom& g, void* C,
                           int64_t stride, hipStream_t s) {
  constexpr int BM = 4 * 16 * MB;
  dim3 grid((unsigned)((g.M + BM - 1) / BM), g.nslices, g.ksplit), block(256);
  const uint16_t* x = (const uint16_t*)X;
  const uint16_t* b = (const uint16_t*)B;
  float* c = (float*)C;
  switch (g.NB) {
    case 1: hipLaunchKernelGGL((k_level1_bf16<MB, 1, KCM, VEC>), grid, block, 0, s, x, b, g, c, stride); break;
    case 2: hipLaunchKernelGGL((k_level1_bf16<MB, 2, KCM, VEC>), grid, block, 0, s, x, b, g, c, stride); break;
    case 3: hipLaunchKernelGGL((k_level1_bf16<MB, 3, KCM, VEC>), grid, block, 0, s, x, b, g, c, stride); break;
    default: hipLaunchKernelGGL((k_level1_bf16<MB, 4, KCM, VEC>), grid, block, 0, s, x, b, g, c, stride); break;
  }
}

// Vector loads need 16-byte aligned, fully valid vectors:
//   K-contiguous rows: K % 8 == 0;  otherwise Q % VW == 0 (VW rows per vector).
static bool vec_ok(int dt, const Level1Geom& g) {
  if (g.kc_mode) return g.K % 8 == 0;
  const int vw = dt == DT_F64 ? 2 : (dt == DT_F32 ? 4 : 8);
  return g.Q % vw == 0;
}

hipError_t launch_level1(const void* X, int dt, const void* B, const Level1Geom& g, void* C,
                         void* partial, hipStream_t s, hipEvent_t after_gemm) {
  const bool split = g.ksplit > 1;
  void* dst = split ? partial : C;
  const int64_t stride = split ? g.M * (int64_t)g.R : 0;
  const bool vec = vec_ok(dt, g);
  if (g.strided) {
    if (dt == DT_F64) launch_reg_str<DT_F64, 2>(X, B, g, dst, stride, s);
    else if (dt == DT_F32) launch_reg_str<DT_F32, 4>(X, B, g, dst, stride, s);
    else return hipErrorInvalidValue;  // the BF16 kernel has no strided addressing
  } else if (dt == DT_F64) {
    if (g.kc_mode) { if (vec) launch_reg_nb<DT_F64, 2, true, true>(X, B, g, dst, stride, s); else launch_reg_nb<DT_F64, 2, true, false>(X, B, g, dst, stride, s); }
    else { if (vec) launch_reg_nb<DT_F64, 2, false, true>(X, B, g, dst, stride, s); else launch_reg_nb<DT_F64, 2, false, false>(X, B, g, dst, stride, s); }
  } else if (dt == DT_F32) {
    if (g.kc_mode) { if (vec) launch_reg_nb<DT_F32, 4, true, true>(X, B, g, dst, stride, s); else launch_reg_nb<DT_F32, 4, true, false>(X, B, g, dst, stride, s); }
    else { if (vec) launch_reg_nb<DT_F32, 4, false, true>(X, B, g, dst, stride, s); else launch_reg_nb<DT_F32, 4, false, false>(X, B, g, dst, stride, s); }
  } else {
    if (g.kc_mode) { if (vec) launch_bf16_nb<4, true, true>(X, B, g, dst, stride, s); else launch_bf16_nb<4, true, false>(X, B, g, dst, stride, s); }
    else { if (vec) launch_bf16_nb<2, false, true>(X, B, g, dst, stride, s); else launch_bf16_nb<2, false, false>(X, B, g, dst, stride, s); }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (after_gemm) {
    e = hipEventRecord(after_gemm, s);
    if (e != hipSuccess) return e;
  }
  if (!split) return hipSuccess;
  const int64_t count = g.M * (int64_t)g.R;
  if (dt == DT_F64)
    hipLaunchKernelGGL((k_reduce_splits<double, double>), dim3(grid_for(count)), dim3(256), 0, s,
                       (double*)C, (const double*)partial, g.ksplit, count);
  else
    hipLaunchKernelGGL((k_reduce_splits<float, float>), dim3(grid_for(count)), dim3(256), 0, s,
                       (float*)C, (const float*)partial, g.ksplit, count);
  return hipGetLastError();
}

hipError_t launch_reduce_splits_to(void* out, int out_f32, const void* partial, int part_f32,
                                   int nsplit, int64_t count, hipStream_t s) {
  dim3 grid(grid_for(count)), block(256);
  if (out_f32 && part_f32) hipLaunchKernelGGL((k_reduce_splits<float, float>), grid, block, 0, s, (float*)out, (const float*)partial, nsplit, count);
  else if (out_f32) hipLaunchKernelGGL((k_reduce_splits<float, double>), grid, block, 0, s, (float*)out, (const double*)partial, nsplit, count);
  else if (part_f32) hipLaunchKernelGGL((k_reduce_splits<double, float>), grid, block, 0, s, (double*)out, (const float*)partial, nsplit, count);
  else hipLaunchKernelGGL((k_reduce_splits<double, double>), grid, block, 0, s, (double*)out, (const double*)partial, nsplit, count);
  return hipGetLastError();
}

}  // namespace ppk
