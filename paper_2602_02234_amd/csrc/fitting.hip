// Fitting net on gfx950: per-atom energy from the descriptor and, for the
// backward pass, dE_i/dD (paper, Section II: a fitting net maps each atom's
// representation to its energy; E is the sum of the atomic energies).
//   y1 = tanh(D F1 + c1);  y2 = tanh(y1 F2 + c2) + y1;  y3 = tanh(y2 F3 + c3) + y2
//   E_i = y3 . F4 + c4 + ebias[t_i]    (per fitting head; see k_fit)
// Batched over 16 atoms per workgroup so each weight fragment is fetched once per
// 16 atoms; the 1600 -> 240 products and their transposes run on MFMA.
// dE/dD overwrites D in place (each workgroup owns its 16 rows).
#include "dp_internal.h"

namespace dp {
namespace {

constexpr int LDF = FH + 4;

// NH fitting heads on the same descriptor: each head's forward gives E_i^h (kept in
// Eh[i][h] when NH > 1) and E_i = sum_h hw_h E_i^h; every head with a non-zero weight runs
// its backward with dE/dy3 = hw_h F4^h, and dE/dD = sum_h dE/dpre1^h F1^hT.
template <typename T, int NH>
__global__ void __launch_bounds__(NTHREADS)
k_fit(Weights<T> w, const int *__restrict__ types, int c0, int n, float *__restrict__ D, double *__restrict__ Ei,
      double *__restrict__ Eh, int backward) {
  __shared__ float y1[16 * LDF], t2[16 * LDF], y2[16 * LDF], t3[16 * LDF], bA[16 * LDF], bB[16 * LDF];
  __shared__ float bS[NH > 1 ? NH : 1][NH > 1 ? 16 * LDF : 4];  // dE/dpre1 of each head (NH > 1)
  __shared__ double eacc[16];
  const int a0 = c0 + blockIdx.x * 16;
  const int wv = wave_id();
  constexpr int NT = FH / 16;  // 15 column tiles of the hidden width
  if (threadIdx.x < 16) eacc[threadIdx.x] = 0.0;
#pragma unroll 1
  for (int h = 0; h < NH; ++h) {
    const float hw = (float)w.hw[h];
    // layer 1: y1 = tanh(D F1 + c1)
    for (int t = wv; t < NT; t += NW) {
      const int c0 = t * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return (a0 + r < n) ? D[(size_t)(a0 + r) * ND + k] : 0.f; },
                   [&](int c, int k) { return ldw(w.F1T[h], (c0 + c) * ND + k); }, ND);
      const int col = c0 + acc_col();
      for (int i = 0; i < 4; ++i) y1[acc_row(i) * LDF + col] = tanhf(acc[i] + w.c1[h][col]);
    }
    __syncthreads();
    for (int t = wv; t < NT; t += NW) {
      const int c0 = t * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return y1[r * LDF + k]; },
                   [&](int c, int k) { return ldw(w.F2T[h], (c0 + c) * FH + k); }, FH);
      const int col = c0 + acc_col();
      for (int i = 0; i < 4; ++i) {
        const int r = acc_row(i);
        const float tt = tanhf(acc[i] + w.c2[h][col]);
        t2[r * LDF + col] = tt;
        y2[r * LDF + col] = tt + y1[r * LDF + col];
      }
    }
    __syncthreads();
    for (int t = wv; t < NT; t += NW) {
      const int c0 = t * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return y2[r * LDF + k]; },
                   [&](int c, int k) { return ldw(w.F3T[h], (c0 + c) * FH + k); }, FH);
      const int col = c0 + acc_col();
      for (int i = 0; i < 4; ++i) {
        const int r = acc_row(i);
        const float tt = tanhf(acc[i] + w.c3[h][col]);
        t3[r * LDF + col] = tt;
        bA[r * LDF + col] = tt + y2[r * LDF + col];
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < 16 && a0 + (int)threadIdx.x < n) {
      const int r = threadIdx.x;
      int ty = types[a0 + r];
      ty = ty < 0 ? 0 : (ty >= NTYPES ? NTYPES - 1 : ty);
      double e = 0.0;  // the last layer's dot product in float64, with float64 F4, c4, ebias
      for (int o = 0; o < FH; ++o) e += (double)bA[r * LDF + o] * w.F4d[h][o];
      e += w.c4[h] + w.ebias[h][ty];
      eacc[r] += w.hw[h] * e;
      if (NH > 1) Eh[(size_t)(a0 + r) * MAXH + h] = e;
    }
    if (backward && w.hw[h] != 0.0) {
      for (int q = threadIdx.x; q < 16 * FH; q += NTHREADS) {
        const int r = q / FH, o = q % FH;
        const float tt = t3[r * LDF + o];
        bB[r * LDF + o] = hw * w.F4[h][o] * (1.f - tt * tt);
      }
      __syncthreads();
      // dy2 = dpre3 F3^T + dy3  (dy3 = hw F4);  dpre2 = dy2 (1 - t2^2)
      for (int t = wv; t < NT; t += NW) {
        const int c0 = t * 16;
        f4 acc = {0, 0, 0, 0};
        Mma<T>::tile(acc, [&](int r, int k) { return bB[r * LDF + k]; },
                     [&](int c, int k) { return ldw(w.F3[h], (c0 + c) * FH + k); }, FH);
        const int col = c0 + acc_col();
        for (int i = 0; i < 4; ++i) {
          const int r = acc_row(i);
          const float dy2 = acc[i] + hw * w.F4[h][col];
          const float tt = t2[r * LDF + col];
          bA[r * LDF + col] = dy2;
          t3[r * LDF + col] = dy2 * (1.f - tt * tt);
        }
      }
      __syncthreads();
      // dy1 = dpre2 F2^T + dy2;  dpre1 = dy1 (1 - y1^2)
      float *bo = NH > 1 ? bS[h] : bB;
      for (int t = wv; t < NT; t += NW) {
        const int c0 = t * 16;
        f4 acc = {0, 0, 0, 0};
        Mma<T>::tile(acc, [&](int r, int k) { return t3[r * LDF + k]; },
                     [&](int c, int k) { return ldw(w.F2[h], (c0 + c) * FH + k); }, FH);
        const int col = c0 + acc_col();
        for (int i = 0; i < 4; ++i) {
          const int r = acc_row(i);
          const float dy1 = acc[i] + bA[r * LDF + col];
          const float yy = y1[r * LDF + col];
          bo[r * LDF + col] = dy1 * (1.f - yy * yy);
        }
      }
    }
    __syncthreads();  // the next head overwrites the activations
  }
  if ((int)threadIdx.x < 16 && a0 + (int)threadIdx.x < n) Ei[a0 + threadIdx.x] = eacc[threadIdx.x];
  if (!backward) return;
  // dE/dD = sum over heads of dpre1 F1^T, written over D
  for (int t = wv; t < ND / 16; t += NW) {
    const int c0 = t * 16;
    f4 acc = {0, 0, 0, 0};
    for (int h = 0; h < NH; ++h)
      if (w.hw[h] != 0.0) {
        const float *bi = NH > 1 ? bS[h] : bB;
        Mma<T>::tile(acc, [&](int r, int k) { return bi[r * LDF + k]; },
                     [&](int c, int k) { return ldw(w.F1[h], (c0 + c) * FH + k); }, FH);
      }
    const int col = c0 + acc_col();
    for (int i = 0; i < 4; ++i) {
      const int r = acc_row(i);
      if (a0 + r < n) D[(size_t)(a0 + r) * ND + col] = acc[i];
    }
  }
}

}  // namespace

template <typename T>
void launch_fitting(const Weights<T> &w, const Workspace &ws, const int *types, int c0, int c1, bool backward,
                    hipStream_t st) {
  const dim3 grid((c1 - c0 + 15) / 16), block(NTHREADS);
  const int n = c1;
  const int b = backward ? 1 : 0;
  switch (w.nheads) {
    case 1: hipLaunchKernelGGL((k_fit<T, 1>), grid, block, 0, st, w, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
    case 2: hipLaunchKernelGGL((k_fit<T, 2>), grid, block, 0, st, w, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
    case 3: hipLaunchKernelGGL((k_fit<T, 3>), grid, block, 0, st, w, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
    default: hipLaunchKernelGGL((k_fit<T, 4>), grid, block, 0, st, w, types, c0, n, ws.D, ws.Ei, ws.Eh, b); break;
  }
}
template void launch_fitting<float>(const Weights<float> &, const Workspace &, const int *, int, int, bool,
                                    hipStream_t);

}  // namespace dp
