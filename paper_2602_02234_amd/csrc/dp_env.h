// Per-atom environment (shared by the descriptor kernels of both precisions).
//   Delta = x_j - x_i (minimum image), r = |Delta|, u = (r - rcs) / (rc - rcs),
//   sw = 1 below rcs, u^3 (-6u^2 + 15u - 10) + 1 up to rc, 0 beyond (quintic, C2);
//   s = sw / r, rhat = Delta / r, Rt = (s, s rhat).  Padded tokens (j >= n) are zero.
#pragma once
#include "dp_internal.h"

namespace dp {

__device__ __forceinline__ int clamp_type(int t) { return t < 0 ? 0 : (t >= NTYPES ? NTYPES - 1 : t); }

struct Env {
  float s[NPMAX], sw[NPMAX], dsw[NPMAX], r[NPMAX];
  float rh[NPMAX * 3];
  float Rt[NPMAX * 4];
  int tj[NPMAX];
};

__device__ inline void build_env(Env &e, const double *__restrict__ X, const int *__restrict__ types,
                                 const int *__restrict__ nlist, int i, int n, int natoms, const Grid &g, float rc,
                                 float rcs) {
  for (int j = threadIdx.x; j < NPMAX; j += blockDim.x) {
    float s = 0.f, sw = 0.f, dsw = 0.f, r = 1.f, hx = 0.f, hy = 0.f, hz = 0.f;
    int tj = 0;
    if (j < n) {
      int nj = nlist[(size_t)i * SEL + j];
      if (nj < 0 || nj >= natoms) nj = i;  // never read outside the coordinate array
      tj = clamp_type(types[nj]);
      double d[3];
      for (int a = 0; a < 3; ++a) {
        double v = X[3 * nj + a] - X[3 * i + a];
        if (g.periodic) v -= g.L[a] * rint(v * g.invL[a]);
        d[a] = v;
      }
      const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
      r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float u = (r - rcs) / (rc - rcs);
      if (r < rcs) {
        sw = 1.f;
      } else if (r < rc) {
        sw = u * u * u * (-6.f * u * u + 15.f * u - 10.f) + 1.f;
        dsw = -30.f * u * u * (1.f - u) * (1.f - u) / (rc - rcs);
      }
      s = sw / r;
      hx = dx / r; hy = dy / r; hz = dz / r;
    }
    e.s[j] = s; e.sw[j] = sw; e.dsw[j] = dsw; e.r[j] = r;
    e.rh[3 * j] = hx; e.rh[3 * j + 1] = hy; e.rh[3 * j + 2] = hz;
    e.Rt[4 * j] = s; e.Rt[4 * j + 1] = s * hx; e.Rt[4 * j + 2] = s * hy; e.Rt[4 * j + 3] = s * hz;
    e.tj[j] = tj;
  }
}

__device__ __forceinline__ float gate(const Env &e, int j, int k) {
  return e.rh[3 * j] * e.rh[3 * k] + e.rh[3 * j + 1] * e.rh[3 * k + 1] + e.rh[3 * j + 2] * e.rh[3 * k + 2];
}

// The last step of the backward pass for one token: combine the gradients that reached
// s (through the embedding input and Rt), rhat (through Rt and the gate) and sw (through
// the softmax weights) into g = dE_i / dDelta_ij.
__device__ __forceinline__ float4 pair_gradient(const Env &e, int j, float ds_emb, const float *dRt, const float *drh,
                                                float dswa) {
  const float s = e.s[j], sw = e.sw[j], rr = e.r[j];
  const float hx = e.rh[3 * j], hy = e.rh[3 * j + 1], hz = e.rh[3 * j + 2];
  const float ds = ds_emb + dRt[0] + dRt[1] * hx + dRt[2] * hy + dRt[3] * hz;
  const float gx = drh[0] + s * dRt[1];
  const float gy = drh[1] + s * dRt[2];
  const float gz = drh[2] + s * dRt[3];
  const float dswt = dswa + ds / rr;
  const float dr = -ds * sw / (rr * rr) + dswt * e.dsw[j];
  const float proj = gx * hx + gy * hy + gz * hz;
  return make_float4((gx - proj * hx) / rr + dr * hx, (gy - proj * hy) / rr + dr * hy, (gz - proj * hz) / rr + dr * hz,
                     0.f);
}

}  // namespace dp
