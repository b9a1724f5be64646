// Device bodies of the per-mode tail steps that more than one kernel runs: the head of a
// mode (Gamma, W, the Cholesky factor and the solve operands) and the Gram tiles of the
// updated factor.  Each takes its LDS from the caller, so that a kernel can give the
// same LDS to different roles of its workgroups.
#pragma once
#include "common.h"
#include "tail_dev.h"
#include "../../include/ppals.h"

namespace ppk {

constexpr int NPART = 5;  // per-block norm partials of the solve

// Gamma^(n)[e] = prod_{i != n} S^(i)[e]
__device__ __forceinline__ double gamma_entry(const double* S, int N, int n, int64_t RR, int e) {
  double sv[PP_MAXN];
#pragma unroll
  for (int i = 0; i < PP_MAXN; ++i) sv[i] = (i < N && i != n) ? S[i * RR + e] : 1.0;
  double v = 1.0;
#pragma unroll
  for (int i = 0; i < PP_MAXN; ++i) v *= sv[i];
  return v;
}

constexpr int HEAD_THREADS = 256;

// Head of mode n (one workgroup of four waves): Gamma^(n), W^(n) (PP), the Cholesky
// factor (wave 0, one diagonal-shift retry) and the solve operands.  Small enough to be
// co-resident with the contraction kernels that run meanwhile on the other stream.  NM
// is the tensor order; thread t takes row t / 4 and columns t % 4 + 4 j, a batch of CB
// columns at a time with the loads of every other mode's S (and U) issued together.
// The body runs in a workgroup of HEAD_THREADS threads; the caller provides the LDS:
// Lm (64 x CH64_LS doubles: Gamma, zero-padded to 64 x 64), cb (128 doubles) and red
// (HEAD_THREADS / 64 doubles).
constexpr int HEAD_LDS = 64 * CH64_LS + 128 + HEAD_THREADS / 64;  // doubles

// COH: Gamma was left by workgroups of the same launch (other XCDs' caches); it is read
// with device-scope atomic loads, which bypass the non-coherent L2.
__device__ __forceinline__ double coh_load(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coh_store(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NM, bool COH = false>
__device__ __forceinline__ void head_body(const HeadArgs& h, double* Lm, double* cb, double* red) {
  constexpr int NO = NM - 1;                 // modes other than n
  constexpr int CB = 16 / NO > 1 ? 16 / NO : 2;
  __builtin_amdgcn_s_setprio(3);  // latency-bound: first in line for issue beside streaming kernels
  const int tid = threadIdx.x;
  const int R = h.R, RR = R * R;
  const int n = h.n;
  const bool wterm = h.pp && h.second_order;
  for (int e = tid; e < 64 * CH64_LS; e += HEAD_THREADS) {
    const int r = e / CH64_LS, c = e - r * CH64_LS;
    if (r >= R || c >= R) Lm[e] = 0.0;
  }
  const int row = tid >> 2, c0 = tid & 3;
  double dmax = 0.0;
  if (h.gamma_ready) {
    if (row < R) {
      double gv[16];
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = c0 + 4 * j;
        const double* gp = h.gamma + row * R + (c < R ? c : 0);
        gv[j] = COH ? coh_load(gp) : *gp;
      }
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const int c = c0 + 4 * j;
        if (c < R) {
          Lm[row * CH64_LS + c] = gv[j];
          if (row == c) dmax = fmax(dmax, gv[j]);
        }
      }
    }
  } else if (row < R) {
    for (int j0 = 0; c0 + 4 * j0 < R; j0 += CB) {
      double sv[CB][NO], uv[CB][NO];
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int c = c0 + 4 * (j0 + j);
        const int e = row * R + (c < R ? c : 0);
#pragma unroll
        for (int k = 0; k < NO; ++k) {
          const int mk = k + (k >= n ? 1 : 0);
          sv[j][k] = h.S[(int64_t)mk * RR + e];
          uv[j][k] = wterm ? h.U[(int64_t)mk * RR + e] : 0.0;
        }
      }
#pragma unroll
      for (int j = 0; j < CB; ++j) {
        const int c = c0 + 4 * (j0 + j);
        if (c < R) {
          // Running sums over the modes k != n: P0 = prod s_k (= Gamma), P1 = sum_i u_i
          // prod_{k != i} s_k, P2 = sum_{i<j} u_i u_j prod_{k != i,j} s_k (= W).
          double P0 = 1.0, P1 = 0.0, P2 = 0.0;
#pragma unroll
          for (int k = 0; k < NO; ++k) {
            P2 = fma(P2, sv[j][k], P1 * uv[j][k]);
            P1 = fma(P1, sv[j][k], P0 * uv[j][k]);
            P0 *= sv[j][k];
          }
          const int e = row * R + c;
          h.gamma[e] = P0;
          Lm[row * CH64_LS + c] = P0;
          if (row == c) dmax = fmax(dmax, P0);
          if (wterm) h.W[e] = P2;
        }
      }
    }
  }
  for (int off = 32; off > 0; off >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, off));
  if ((tid & 63) == 0) red[tid >> 6] = dmax;
  __syncthreads();
  if (tid < 64) {  // the factorisation is wave 0's alone; the other waves wait below
    int st = 0, piv0 = -1;
    for (int attempt = 0;; ++attempt) {
      const int piv = chol_wave64(Lm, cb, R);
      if (piv < 0) break;
      if (attempt == 0) piv0 = piv;
      if (attempt == 1) {
        st = 2;
        break;
      }
      double mx = 0.0;
      for (int i = 0; i < HEAD_THREADS / 64; ++i) mx = fmax(mx, red[i]);
      const double delta = (double)R * 0x1p-52 * mx;
      for (int e = tid; e < 64 * CH64_LS; e += 64) {
        const int r = e / CH64_LS, c = e - r * CH64_LS;
        double g = 0.0;
        if (r < R && c < R) {
          if (!h.gamma_ready) g = gamma_entry(h.S, h.N, n, RR, r * R + c);
          else g = COH ? coh_load(h.gamma + r * R + c) : h.gamma[r * R + c];
        }
        Lm[e] = g + (r < R && r == c ? delta : 0.0);
      }
      st = 1;
    }
    if (tid < R) cb[tid] = 1.0 / Lm[tid * CH64_LS + tid];
    if (tid == 0) h.status[n] = chol_status_word(st, piv0);
  }
  __syncthreads();
  // the solve operands: LF[k][i] = L[i][k] / L[k][k] (i > k), LB[i][k] = L[i][k] / L[i][i]
  // (k < i), zero elsewhere, then 1 / L[i][i]
  double* LF = h.pack;
  double* LB = LF + RR;
  if (row < R) {
    const double di = cb[row];
    for (int c = c0; c < R; c += 4) {
      const double v = c <= row ? Lm[row * CH64_LS + c] : 0.0;
      LF[c * R + row] = row > c ? v * cb[c] : 0.0;
      LB[row * R + c] = c < row ? v * di : 0.0;
    }
    if (c0 == 0) LB[RR + row] = di;
  }
}

// Grams of the updated factor on the matrix cores: S = A^T A and, in PP sweeps,
// U = A^T dA.  One workgroup of GW waves per 16 x 16 output tile, computing the
// tile of S and of U from one read of A's tile columns; each wave takes GRAM_U groups of
// 4 rows at a time and loads the next groups before the current matrix-core steps
// (f64 16x16x4: lane l supplies A[y0 + l/16][r0 + l%16] and B[y0 + l/16][c0 + l%16];
// accumulator register v holds tile row 4v + l/16, column l%16).  When asked, each
// workgroup also forms its tile of Gamma^(next) and W^(next) for the following mode's
// head, with the other modes' S and U tiles loaded at the start.  Block 0 also reduces the
// solve's per-block partials into the sweep record (and the fit).
// The body runs in a workgroup of GW waves on output tile `tile`; the caller provides the
// LDS: racc (GRAM_RACC(GW) doubles), tileS and tileU (256 each) and tileO ((N - 2) x 2 x
// 256, when Gamma^(next) is formed).
constexpr int GRAM_U = 4;
constexpr int GRAM_RACC(int gw) { return (gw / 2) * 2 * 4 * 64; }

// COH: the Gamma tile is stored with device-scope atomic stores (written through to the
// coherent level), for a head in another workgroup of the same launch.
//
// Row splits (a.nsplit > 1): the rows are cut into nsplit ranges and the tile is the sum of
// the ranges' partial tiles, added in range order.  With COH each range is its own
// workgroup (`split`): it writes its partial tile through to a.gpart, counts itself on the
// tile's counter a.gctr[tile], and the last of them adds the partials and goes on (the
// others return).  Without COH one workgroup computes the ranges one after another; both
// give the same bits.
template <int GW, bool COH = false>
__device__ __forceinline__ void gram_body(const GramArgs& a, int tile, int split, double* racc,
                                          double* tileS, double* tileU, double* tileO) {
  __builtin_amdgcn_s_setprio(3);
  const int tid = threadIdx.x;
  const int w = tid >> 6, l = tid & 63;
  const int R = a.R, RR = R * R;
  const int NBR = (R + 15) / 16;
  const int r0 = (tile / NBR) * 16, c0 = (tile % NBR) * 16;
  const bool has_u = a.dA != nullptr;
  // this thread's tile entry for Gamma^(next): the other modes' S and U, loaded up front
  const bool want_g = a.gamma_out != nullptr;
  const int te_r = r0 + ((tid & 255) >> 4), te_c = c0 + (tid & 15);
  const bool te_ok = want_g && te_r < R && te_c < R;
  const int ky = l >> 4, cc = l & 15;
  const bool oka = r0 + cc < R, okb = c0 + cc < R;
  const int64_t rows = a.rows;
  if (want_g) {
    // thread t takes entry t % 256 of the other modes o = t / 256, t / 256 + GW / 4, ...
    // (S and U; other mode o = the o-th mode that is neither this one nor the next)
    const int e = te_ok ? te_r * R + te_c : 0;
    for (int o = tid >> 8; o < a.N - 2; o += GW * 64 / 256) {
      int k = -1;
      for (int q = 0, cnt = 0; q < a.N; ++q)
        if (q != a.mode && q != a.next && cnt++ == o) k = q;
      if (k >= 0) {
        const double sv = a.S_all[(int64_t)k * RR + e];
        const double uv = a.wterm ? a.U_all[(int64_t)k * RR + e] : 0.0;
        tileO[(o * 2 + 0) * 256 + (tid & 255)] = sv;
        tileO[(o * 2 + 1) * 256 + (tid & 255)] = uv;
      }
    }
  }
  // The tile of S (waves 0) and U (wave 1) over rows [ys, ye): sum[v] = tile row 4v + l/16,
  // column l%16.
  constexpr int HW = GW / 2;
  auto tile_sum = [&](int64_t ys, int64_t ye, double (&sum)[4]) {
    d4 accS = {0.0, 0.0, 0.0, 0.0}, accU = {0.0, 0.0, 0.0, 0.0};
    double xa[GRAM_U], xb[GRAM_U], xd[GRAM_U];
    auto load = [&](int64_t y0, double (&va)[GRAM_U], double (&vb)[GRAM_U], double (&vd)[GRAM_U]) {
#pragma unroll
      for (int u = 0; u < GRAM_U; ++u) {
        const int64_t y = y0 + 4 * u + ky;
        const bool in = y < ye;
        va[u] = (in && oka) ? a.A[y * R + r0 + cc] : 0.0;
        vb[u] = (in && okb) ? a.A[y * R + c0 + cc] : 0.0;
        vd[u] = (in && okb && has_u) ? a.dA[y * R + c0 + cc] : 0.0;
      }
    };
    const int64_t step = (int64_t)4 * GRAM_U * GW;
    int64_t y0 = ys + (int64_t)w * 4 * GRAM_U;
    load(y0, xa, xb, xd);
    for (; y0 < ye; y0 += step) {
      double na[GRAM_U], nb[GRAM_U], nd[GRAM_U];
      const bool more = y0 + step < ye;
      if (more) load(y0 + step, na, nb, nd);
#pragma unroll
      for (int u = 0; u < GRAM_U; ++u) {
        accS = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xb[u], accS, 0, 0, 0);
        if (has_u) accU = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u], xd[u], accU, 0, 0, 0);
      }
      if (more) {
#pragma unroll
        for (int u = 0; u < GRAM_U; ++u) {
          xa[u] = na[u];
          xb[u] = nb[u];
          xd[u] = nd[u];
        }
      }
    }
    // two-stage reduction over the waves: the upper half adds into the lower half
    if (w >= HW) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        racc[(((w - HW) * 2 + 0) * 4 + v) * 64 + l] = accS[v];
        racc[(((w - HW) * 2 + 1) * 4 + v) * 64 + l] = accU[v];
      }
    }
    __syncthreads();
    if (w < HW) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        racc[((w * 2 + 0) * 4 + v) * 64 + l] += accS[v];
        racc[((w * 2 + 1) * 4 + v) * 64 + l] += accU[v];
      }
    }
    __syncthreads();
    if (w < 2) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = 0.0;
        for (int q = 0; q < HW; ++q) t += racc[((q * 2 + w) * 4 + v) * 64 + l];
        sum[v] = t;
      }
    }
    __syncthreads();  // racc is free again
  };
  const int nsplit = a.nsplit > 1 ? a.nsplit : 1;
  const int64_t per = (rows + nsplit - 1) / nsplit;
  double tot[4] = {0.0, 0.0, 0.0, 0.0};
  if (COH && nsplit > 1) {
    __shared__ int last_split;
    const int64_t ys = (int64_t)split * per;
    tile_sum(ys, ys + per < rows ? ys + per : rows, tot);
    double* gp = a.gpart + (int64_t)tile * nsplit * 512;
    const int pe = w * 256 + (4 * 0 + ky) * 16 + cc;  // entry of register v = 0
    if (w < 2) {
#pragma unroll
      for (int v = 0; v < 4; ++v) coh_store(gp + split * 512 + pe + 64 * v, tot[v]);
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    if (tid == 0) last_split = atomicAdd(a.gctr + tile, 1) == nsplit - 1;
    __syncthreads();
    if (!last_split) return;
    if (tid == 0) __hip_atomic_store(a.gctr + tile, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (w < 2) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        double t = coh_load(gp + pe + 64 * v);
        for (int q = 1; q < nsplit; ++q) t += coh_load(gp + q * 512 + pe + 64 * v);
        tot[v] = t;
      }
    }
  } else {
    for (int q = 0; q < nsplit; ++q) {
      double part[4];
      const int64_t ys = (int64_t)q * per;
      tile_sum(ys, ys + per < rows ? ys + per : rows, part);
#pragma unroll
      for (int v = 0; v < 4; ++v) tot[v] = q == 0 ? part[v] : tot[v] + part[v];
    }
  }
  if (w < 2 && (w == 0 || has_u)) {
    double* out = w ? a.U_out : a.S_out;
    double* tl = w ? tileU : tileS;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int tr = 4 * v + ky, tc = cc;
      const int r = r0 + tr, c = c0 + tc;
      if (r < R && c < R) out[r * R + c] = tot[v];
      tl[tr * 16 + tc] = tot[v];
    }
  }
  if (want_g) {
    __syncthreads();
    if (te_ok && tid < 256) {
      // Running sums over the modes k != next (order of k as in the head): P0 = Gamma,
      // P2 = W (second-order term)
      double P0 = 1.0, P1 = 0.0, P2 = 0.0;
      int o = 0;
      for (int k = 0; k < a.N; ++k) {
        if (k == a.next) continue;
        double sk, uk;
        if (k == a.mode) {
          sk = tileS[tid];
          uk = has_u ? tileU[tid] : 0.0;
        } else {
          sk = tileO[(o * 2 + 0) * 256 + tid];
          uk = tileO[(o * 2 + 1) * 256 + tid];
          ++o;
        }
        P2 = fma(P2, sk, P1 * uk);
        P1 = fma(P1, sk, P0 * uk);
        P0 *= sk;
      }
      const int e = te_r * R + te_c;
      if (COH) coh_store(a.gamma_out + e, P0);
      else a.gamma_out[e] = P0;
      if (a.wterm) a.W_out[e] = P2;
    }
  }
  if (tile != 0) return;
  // a launch that takes the threshold test with the gate already closed (only this
  // workgroup writes it) leaves the record as it is
  if (a.gate_out && *a.gate_out == 0) return;
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
      const int stw = *a.status;
      rec->chol_status[a.mode] = stw & 3;
      rec->chol_pivot[a.mode] = (stw >> 8) - 1;
      rec->nonfinite[a.mode] = (isfinite(g2) && isfinite(a2) && isfinite(sums[3])) ? 0 : 1;
      if (a.write_fit) {
        const double r2 = a.normX2 - 2.0 * sums[3] + sums[4];
        rec->fit_est = 1.0 - sqrt(r2 > 0.0 ? r2 : 0.0) / sqrt(a.normX2);
        rec->sweep_kind = a.sweep_kind;
        if (a.ring) {
          // the sweep's record is complete: file it, then decide whether the next sweep runs
          ppals_sweep_record* ring = (ppals_sweep_record*)a.ring;
          const int k = *a.ring_ctr;
          ring[k] = *rec;
          *a.ring_ctr = k + 1;
          bool open = true;
          for (int q = 0; q < a.N; ++q) open = open && rec->rel_change[q] < a.eps;
          *a.gate_out = open ? 1 : 0;
          rec->sweep_kind = open ? PPALS_SWEEP_PP_APPROX : -1;
        }
      }
    }
  }
}

}  // namespace ppk
