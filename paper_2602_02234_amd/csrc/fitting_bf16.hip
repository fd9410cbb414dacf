// Fitting net of the bfloat16 path: per-atom energy and dE/dD (see fitting.hip for
// the model).  The energy is read off the fitting net directly, so its products
// carry the path's largest rounding sensitivity; each one runs on bf16 MFMA with
// both operands split into two bf16 terms, x = x_hi + x_lo, and three products
// x_hi w_hi + x_hi w_lo + x_lo w_hi accumulated in fp32 (the dropped lo*lo term is
// 2^-16 relative).  16 atoms per workgroup, two workgroups per CU; the hidden width
// 240 is padded to 256 along k.  dE/dD overwrites D in place.
#include "dp_internal.h"

namespace dp {
namespace {

constexpr int KH = 256;       // padded hidden width along k
constexpr int LDA = KH + 8;   // LDS row stride (floats) of the hidden activations
constexpr int NWT = 8;        // waves
constexpr int NT = FH / 16;   // 15 hidden column tiles

__device__ __forceinline__ bf8 ld8g(const bf16_t *p) { return *(const bf8 *)p; }

// Splits 8 fp32 values into bf16 hi and lo parts.
__device__ __forceinline__ void split8(const float4 a, const float4 b, bf8 &hi, bf8 &lo) {
  const float v[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)v[e];
    hi[e] = h;
    lo[e] = (__bf16)(v[e] - (float)h);
  }
}

__device__ __forceinline__ f4 mma3(const bf8 &xh, const bf8 &xl, const bf8 &yh, const bf8 &yl, f4 acc) {
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xl, yh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yl, acc, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(xh, yh, acc, 0, 0, 0);
}

// acc = A(16 x K) . B_t^T for the column tiles t = wave + NWT u (< NT), u < 2; A fp32
// rows at a (stride lda, K a multiple of 32), B split bf16 in fragment order at bh/bl.
// The operands of step k + 32 are loaded before the products of step k.
__device__ __forceinline__ void mm_split2(f4 (&acc)[2], const float *a, int lda, const bf16_t *bh, const bf16_t *bl,
                                          int K) {
  const int l = lane_id(), r = l & 15, q = l >> 4, wv = wave_id();
  const bool t1 = wv + NWT < NT;
  const int S = K / 32;
  acc[0] = acc[1] = f4{0.f, 0.f, 0.f, 0.f};
  const float *ar = a + r * lda + 8 * q;
  const size_t o0 = (size_t)wv * S * 512 + 8 * l, o1 = (size_t)min(wv + NWT, NT - 1) * S * 512 + 8 * l;
  float4 pa0 = *(const float4 *)ar, pa1 = *(const float4 *)(ar + 4);
  bf8 ph0 = ld8g(bh + o0), pl0 = ld8g(bl + o0), ph1 = ld8g(bh + o1), pl1 = ld8g(bl + o1);
  for (int k0 = 0, st = 0; k0 < K; k0 += 32, ++st) {
    const float4 a0 = pa0, a1 = pa1;
    const bf8 h0 = ph0, l0 = pl0, h1 = ph1, l1 = pl1;
    if (k0 + 32 < K) {
      const int k = k0 + 32;
      const size_t f = (size_t)(st + 1) * 512;
      pa0 = *(const float4 *)(ar + k);
      pa1 = *(const float4 *)(ar + k + 4);
      ph0 = ld8g(bh + o0 + f); pl0 = ld8g(bl + o0 + f);
      ph1 = ld8g(bh + o1 + f); pl1 = ld8g(bl + o1 + f);
    }
    __builtin_amdgcn_sched_barrier(0);
    bf8 xh, xl;
    split8(a0, a1, xh, xl);
    acc[0] = mma3(xh, xl, h0, l0, acc[0]);
    if (t1) acc[1] = mma3(xh, xl, h1, l1, acc[1]);
  }
}

// The dE/dD product for the column tiles t = wave + NWT u, U0 <= u < U1 (< ND / 16),
// A from LDS (K = 256), B in fragment order.
template <int U0, int U1>
__device__ __forceinline__ void mm_split_dd(f4 (&acc)[U1 - U0], const float *a, int lda, const bf16_t *bh,
                                            const bf16_t *bl, bool zero = true) {
  const int l = lane_id(), r = l & 15, q = l >> 4, wv = wave_id();
  if (zero) {
#pragma unroll
    for (int u = 0; u < U1 - U0; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
  }
  for (int k0 = 0; k0 < KH; k0 += 32) {
    bf8 xh, xl;
    const float *ar = a + r * lda + k0 + 8 * q;
    split8(*(const float4 *)ar, *(const float4 *)(ar + 4), xh, xl);
#pragma unroll
    for (int u = U0; u < U1; ++u) {
      const int t = wv + NWT * u;
      if (t < ND / 16) {
        const size_t o = ((size_t)t * (KH / 32) + k0 / 32) * 512 + 8 * l;
        acc[u - U0] = mma3(xh, xl, ld8g(bh + o), ld8g(bl + o), acc[u - U0]);
      }
    }
  }
}

// NH fitting heads on the same descriptor: each head's forward gives E_i^h (kept in
// Eh[i][h] when NH > 1) and E_i = sum_h hw_h E_i^h; the backward of every head with a
// non-zero weight runs with dE/dy3 = hw_h F4^h, and dE/dD = sum_h dE/dpre1^h F1^hT.
template <int NH>
__global__ void __launch_bounds__(NWT * 64) __attribute__((amdgpu_waves_per_eu(4)))
k_fit_b16(Tables w, WeightsB16 wp, const int *__restrict__ types, int c0, int n, float *__restrict__ D,
          double *__restrict__ Ei, double *__restrict__ Eh, int backward) {
  // y1, t2: the first two layers' outputs; y2: the third layer's input, later dE/dy2;
  // X: dE/dpre3, dE/dpre2, dE/dpre1 in turn (Xs: dE/dpre1 of each head, NH > 1).
  // Columns 240..255 stay zero.
  __shared__ __align__(16) float y1[16 * LDA], t2[16 * LDA], y2[16 * LDA], X[16 * LDA];
  __shared__ __align__(16) float Xs[NH > 1 ? NH : 1][NH > 1 ? 16 * LDA : 4];
  __shared__ double ep[16][16];  // per-row energy partials, one per column tile
  __shared__ double eacc[16];
  const int a0 = c0 + blockIdx.x * 16;
  const int l = lane_id(), q = l >> 4, cl = l & 15, wv = wave_id();
  for (int x = threadIdx.x; x < 16 * (KH - FH); x += NWT * 64) {
    const int r = x / (KH - FH), c = FH + x % (KH - FH);
    y1[r * LDA + c] = t2[r * LDA + c] = y2[r * LDA + c] = X[r * LDA + c] = 0.f;
  }
  if (threadIdx.x < 16) eacc[threadIdx.x] = 0.0;
  f4 acc[2];
#pragma unroll 1
  for (int h = 0; h < NH; ++h) {
    const float hw = (float)w.hw[h];
    const bool bwd = backward && w.hw[h] != 0.0;
    // y1 = tanh(D F1 + c1); the D allocation has 16 spare rows, so rows >= n of the
    // last batch are read in bounds (their results are discarded)
    mm_split2(acc, D + (size_t)a0 * ND, ND, wp.F1T[h][0], wp.F1T[h][1], ND);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = wv + NWT * u;
      if (t < NT)
        for (int ii = 0; ii < 4; ++ii)
          y1[(4 * q + ii) * LDA + 16 * t + cl] = tanhf(acc[u][ii] + w.c1[h][16 * t + cl]);
    }
    __syncthreads();
    mm_split2(acc, y1, LDA, wp.F2T[h][0], wp.F2T[h][1], KH);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = wv + NWT * u;
      if (t < NT)
        for (int ii = 0; ii < 4; ++ii) {
          const int r = 4 * q + ii, c = 16 * t + cl;
          const float tt = tanhf(acc[u][ii] + w.c2[h][c]);
          t2[r * LDA + c] = tt;
          y2[r * LDA + c] = tt + y1[r * LDA + c];
        }
    }
    __syncthreads();
    // y3 = tanh(y2 F3 + c3) + y2 stays in registers: E_i = y3 . F4 + c4 + ebias(t_i) as
    // per-tile partials, and dE/dpre3 = hw F4 (1 - t3^2) goes to X
    mm_split2(acc, y2, LDA, wp.F3T[h][0], wp.F3T[h][1], KH);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = wv + NWT * u;
      if (t < NT)
        for (int ii = 0; ii < 4; ++ii) {
          const int r = 4 * q + ii, c = 16 * t + cl;
          const float tt = tanhf(acc[u][ii] + w.c3[h][c]);
          X[r * LDA + c] = hw * w.F4[h][c] * (1.f - tt * tt);
          double p = (double)(tt + y2[r * LDA + c]) * w.F4d[h][c];
          p += __shfl_xor(p, 1);
          p += __shfl_xor(p, 2);
          p += __shfl_xor(p, 4);
          p += __shfl_xor(p, 8);
          if (cl == 0) ep[r][t] = p;
        }
    }
    __syncthreads();
    if ((int)threadIdx.x < 16 && a0 + (int)threadIdx.x < n) {
      const int r = threadIdx.x;
      int ty = types[a0 + r];
      ty = ty < 0 ? 0 : (ty >= NTYPES ? NTYPES - 1 : ty);
      double e = 0.0;
      for (int t = 0; t < NT; ++t) e += ep[r][t];
      e += w.c4[h] + w.ebias[h][ty];
      eacc[r] += w.hw[h] * e;
      if (NH > 1) Eh[(size_t)(a0 + r) * MAXH + h] = e;
    }
    if (bwd) {
      // dy2 = dpre3 F3^T + hw F4 (into y2, free since the third layer);  dpre2 = dy2 (1 - t2^2)
      mm_split2(acc, X, LDA, wp.F3[h][0], wp.F3[h][1], KH);
      __syncthreads();  // every wave has read X
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = wv + NWT * u;
        if (t < NT)
          for (int ii = 0; ii < 4; ++ii) {
            const int r = 4 * q + ii, c = 16 * t + cl;
            const float dy2 = acc[u][ii] + hw * w.F4[h][c];
            const float tt = t2[r * LDA + c];
            y2[r * LDA + c] = dy2;
            X[r * LDA + c] = dy2 * (1.f - tt * tt);
          }
      }
      __syncthreads();
      // dy1 = dpre2 F2^T + dy2;  dpre1 = dy1 (1 - y1^2)
      mm_split2(acc, X, LDA, wp.F2[h][0], wp.F2[h][1], KH);
      __syncthreads();
      float *xo = NH > 1 ? Xs[h] : X;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int t = wv + NWT * u;
        if (t < NT)
          for (int ii = 0; ii < 4; ++ii) {
            const int r = 4 * q + ii, c = 16 * t + cl;
            const float dy1 = acc[u][ii] + y2[r * LDA + c];
            const float yy = y1[r * LDA + c];
            xo[r * LDA + c] = dy1 * (1.f - yy * yy);
          }
      }
      if (NH > 1)
        for (int x = threadIdx.x; x < 16 * (KH - FH); x += NWT * 64) {
          const int r = x / (KH - FH), c = FH + x % (KH - FH);
          xo[r * LDA + c] = 0.f;
        }
    }
    __syncthreads();  // the next head overwrites y1, t2, y2, X
  }
  if ((int)threadIdx.x < 16 && a0 + (int)threadIdx.x < n) Ei[a0 + threadIdx.x] = eacc[threadIdx.x];
  if (!backward) return;
  // dE/dD = sum over heads of dpre1 F1^T  (100 column tiles, in two passes over k)
  {
    f4 dacc[7];
    bool first = true;
#pragma unroll 1
    for (int h = 0; h < NH; ++h)
      if (w.hw[h] != 0.0) {
        mm_split_dd<0, 7>(dacc, NH > 1 ? Xs[h] : X, LDA, wp.F1[h][0], wp.F1[h][1], first);
        first = false;
      }
    if (first)
      for (int u = 0; u < 7; ++u) dacc[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 7; ++u) {
      const int t = wv + NWT * u;
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii;
        if (a0 + r < n) D[(size_t)(a0 + r) * ND + 16 * t + cl] = dacc[u][ii];
      }
    }
  }
  {
    f4 dacc[6];
    bool first = true;
#pragma unroll 1
    for (int h = 0; h < NH; ++h)
      if (w.hw[h] != 0.0) {
        mm_split_dd<7, 13>(dacc, NH > 1 ? Xs[h] : X, LDA, wp.F1[h][0], wp.F1[h][1], first);
        first = false;
      }
    if (first)
      for (int u = 0; u < 6; ++u) dacc[u] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int u = 0; u < 6; ++u) {
      const int t = wv + NWT * (u + 7);
      if (t < ND / 16)
        for (int ii = 0; ii < 4; ++ii) {
          const int r = 4 * q + ii;
          if (a0 + r < n) D[(size_t)(a0 + r) * ND + 16 * t + cl] = dacc[u][ii];
        }
    }
  }
}

}  // namespace

void launch_fitting_b16(const Tables &w, const WeightsB16 &wp, const Workspace &ws, const int *types, int c0, int c1,
                        bool backward, hipStream_t st) {
  const dim3 grid((c1 - c0 + 15) / 16), block(NWT * 64);
  const int n = c1;
  const int b = backward ? 1 : 0;
  switch (w.nheads) {
    case 1: hipLaunchKernelGGL(k_fit_b16<1>, grid, block, 0, st, w, wp, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
    case 2: hipLaunchKernelGGL(k_fit_b16<2>, grid, block, 0, st, w, wp, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
    case 3: hipLaunchKernelGGL(k_fit_b16<3>, grid, block, 0, st, w, wp, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
    default: hipLaunchKernelGGL(k_fit_b16<4>, grid, block, 0, st, w, wp, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
  }
}

}  // namespace dp
