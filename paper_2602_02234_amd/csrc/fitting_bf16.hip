// Fitting net of the bfloat16 path: per-atom energy and dE/dD (see fitting.hip for
// the model).  The energy is read off the fitting net directly, so its products
// carry the path's largest rounding sensitivity; each one runs on bf16 MFMA with
// both operands split into two bf16 terms, x = x_hi + x_lo, and three products
// x_hi w_hi + x_hi w_lo + x_lo w_hi accumulated in fp32 (the dropped lo*lo term is
// 2^-16 relative).  16 atoms per workgroup; the hidden width 240 is padded to 256
// along k.  dE/dD overwrites D in place.
#include "dp_internal.h"

namespace dp {
namespace {

constexpr int KH = 256;       // padded hidden width along k
constexpr int LDA = KH + 8;   // LDS row stride (floats) of the hidden activations
constexpr int NWT = 8;        // waves

__device__ __forceinline__ bf8 ld8g(const bf16_t *p) { return *(const bf8 *)p; }

// Splits 8 fp32 values into bf16 hi and lo parts.
__device__ __forceinline__ void split8(const float *p, bf8 &hi, bf8 &lo) {
  const float4 a = *(const float4 *)p, b = *(const float4 *)(p + 4);
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

// acc = A(16 x K) . B_t^T for the column tiles t = wave, wave + NWT, ... (< ntiles);
// A fp32 rows at a (stride lda, K multiple of 32), B split bf16 [col][k] at bh/bl (stride ldb).
template <int MAXT>
__device__ __forceinline__ void mm_split(f4 (&acc)[MAXT], const float *a, int lda, const bf16_t *bh,
                                         const bf16_t *bl, int ldb, int K, int ntiles) {
  const int l = lane_id(), r = l & 15, q = l >> 4, wv = wave_id();
#pragma unroll
  for (int u = 0; u < MAXT; ++u) acc[u] = f4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf8 xh, xl;
    split8(a + r * lda + k0 + 8 * q, xh, xl);
#pragma unroll
    for (int u = 0; u < MAXT; ++u) {
      const int t = wv + NWT * u;
      if (t < ntiles) {
        const size_t o = (size_t)(16 * t + r) * ldb + k0 + 8 * q;
        acc[u] = mma3(xh, xl, ld8g(bh + o), ld8g(bl + o), acc[u]);
      }
    }
  }
}

__global__ void __launch_bounds__(NWT * 64)
k_fit_b16(Weights<bf16_t> w, WeightsB16 wp, const int *__restrict__ types, int n, float *__restrict__ D,
          double *__restrict__ Ei, int backward) {
  __shared__ __align__(16) float y1[16 * LDA], t2[16 * LDA], y2[16 * LDA], t3[16 * LDA], bA[16 * LDA],
      bB[16 * LDA];
  const int a0 = blockIdx.x * 16;
  const int l = lane_id(), q = l >> 4, cl = l & 15, wv = wave_id();
  constexpr int NT = FH / 16;  // 15 hidden column tiles
  for (int x = threadIdx.x; x < 16 * (KH - FH); x += NWT * 64) {
    const int r = x / (KH - FH), c = FH + x % (KH - FH);
    y1[r * LDA + c] = t2[r * LDA + c] = y2[r * LDA + c] = t3[r * LDA + c] = bA[r * LDA + c] = bB[r * LDA + c] = 0.f;
  }
  __syncthreads();
  f4 acc[2];
  // y1 = tanh(D F1 + c1); the D allocation has 16 spare rows, so rows >= n of the
  // last batch are read in bounds (their results are discarded)
  mm_split<2>(acc, D + (size_t)a0 * ND, ND, wp.F1T[0], wp.F1T[1], ND, ND, NT);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wv + NWT * u;
    if (t < NT)
      for (int ii = 0; ii < 4; ++ii) y1[(4 * q + ii) * LDA + 16 * t + cl] = tanhf(acc[u][ii] + w.c1[16 * t + cl]);
  }
  __syncthreads();
  mm_split<2>(acc, y1, LDA, wp.F2T[0], wp.F2T[1], KH, KH, NT);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wv + NWT * u;
    if (t < NT)
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii, c = 16 * t + cl;
        const float tt = tanhf(acc[u][ii] + w.c2[c]);
        t2[r * LDA + c] = tt;
        y2[r * LDA + c] = tt + y1[r * LDA + c];
      }
  }
  __syncthreads();
  mm_split<2>(acc, y2, LDA, wp.F3T[0], wp.F3T[1], KH, KH, NT);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wv + NWT * u;
    if (t < NT)
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii, c = 16 * t + cl;
        const float tt = tanhf(acc[u][ii] + w.c3[c]);
        t3[r * LDA + c] = tt;
        bA[r * LDA + c] = tt + y2[r * LDA + c];
      }
  }
  __syncthreads();
  if ((int)threadIdx.x < 16 && a0 + (int)threadIdx.x < n) {
    const int r = threadIdx.x;
    int ty = types[a0 + r];
    ty = ty < 0 ? 0 : (ty >= NTYPES ? NTYPES - 1 : ty);
    double e = 0.0;
    for (int o = 0; o < FH; ++o) e += (double)bA[r * LDA + o] * (double)w.F4[o];
    Ei[a0 + r] = e + (double)w.c4 + (double)w.ebias[ty];
  }
  if (!backward) return;
  __syncthreads();
  for (int x = threadIdx.x; x < 16 * FH; x += NWT * 64) {
    const int r = x / FH, o = x % FH;
    const float tt = t3[r * LDA + o];
    bB[r * LDA + o] = w.F4[o] * (1.f - tt * tt);  // dpre3
  }
  __syncthreads();
  // dy2 = dpre3 F3^T + F4;  dpre2 = dy2 (1 - t2^2)
  mm_split<2>(acc, bB, LDA, wp.F3[0], wp.F3[1], KH, KH, NT);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wv + NWT * u;
    if (t < NT)
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii, c = 16 * t + cl;
        const float dy2 = acc[u][ii] + w.F4[c];
        const float tt = t2[r * LDA + c];
        bA[r * LDA + c] = dy2;
        t3[r * LDA + c] = dy2 * (1.f - tt * tt);
      }
  }
  __syncthreads();
  // dy1 = dpre2 F2^T + dy2;  dpre1 = dy1 (1 - y1^2)
  mm_split<2>(acc, t3, LDA, wp.F2[0], wp.F2[1], KH, KH, NT);
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int t = wv + NWT * u;
    if (t < NT)
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii, c = 16 * t + cl;
        const float dy1 = acc[u][ii] + bA[r * LDA + c];
        const float yy = y1[r * LDA + c];
        bB[r * LDA + c] = dy1 * (1.f - yy * yy);
      }
  }
  __syncthreads();
  // dE/dD = dpre1 F1^T  (100 column tiles)
  f4 dacc[13];
  mm_split<13>(dacc, bB, LDA, wp.F1[0], wp.F1[1], KH, KH, ND / 16);
#pragma unroll
  for (int u = 0; u < 13; ++u) {
    const int t = wv + NWT * u;
    if (t < ND / 16)
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii;
        if (a0 + r < n) D[(size_t)(a0 + r) * ND + 16 * t + cl] = dacc[u][ii];
      }
  }
}

}  // namespace

void launch_fitting_b16(const Weights<bf16_t> &w, const WeightsB16 &wp, const Workspace &ws, const int *types, int n,
                        bool backward, hipStream_t st) {
  hipLaunchKernelGGL(k_fit_b16, dim3((n + 15) / 16), dim3(NWT * 64), 0, st, w, wp, types, n, ws.D, ws.Ei,
                     backward ? 1 : 0);
}

}  // namespace dp
