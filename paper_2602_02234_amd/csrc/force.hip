// Force assembly, virial and the compensated float64 reductions on gfx950.
//   F_i = sum_{j in N(i)} g_ij - sum_{j : i in N(j)} g_ji     (F = -dE/dx)
//   Xi_ab = - sum_i sum_{j in N(i)} Delta_ij,a g_ij,b
// The second force term is gathered through rev[][] (slot of i in the list of
// j), so no floating-point atomics are needed while lists are symmetric; an
// atom whose list overflowed can leave a pair one-sided, and only those pairs
// are scattered with float64 atomics afterwards.  E and Xi are reduced per
// system in float64 with Neumaier compensation in a fixed order.
#include "dp_internal.h"

namespace dp {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One wavefront per atom.  mode 0: out = F;  mode 1: out = -gE * F = gE dE/dx, virial scaled by gE.
__global__ void __launch_bounds__(256) k_forces(const float4 *__restrict__ g, const int *__restrict__ nlist,
                                                const int *__restrict__ nnei, const int *__restrict__ rev,
                                                const double *__restrict__ X, Grid hg, const Grid *__restrict__ dg,
                                                int n, const double *__restrict__ gE, double *__restrict__ Fout,
                                                double *__restrict__ vpart) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  const Grid gr = dg ? *dg : hg;
  double f[3] = {0, 0, 0}, v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  const int nn = min(max(nnei[i], 0), SEL);
  for (int s = lane; s < nn; s += 64) {
    const size_t is = (size_t)i * SEL + s;
    const float4 gi = g[is];
    int j = nlist[is];
    if (j < 0 || j >= n) j = i;  // never read outside the arrays
    f[0] += gi.x; f[1] += gi.y; f[2] += gi.z;
    const int r = rev[is];
    if (r >= 0 && r < SEL) {
      const float4 gj = g[(size_t)j * SEL + r];
      f[0] -= gj.x; f[1] -= gj.y; f[2] -= gj.z;
    }
    double d[3];
    for (int a = 0; a < 3; ++a) {
      double t = X[3 * j + a] - X[3 * i + a];
      if (gr.periodic) t -= gr.L[a] * rint(t * gr.invL[a]);
      d[a] = t;
    }
    const double gg[3] = {gi.x, gi.y, gi.z};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) v[3 * a + b] -= d[a] * gg[b];
  }
  for (int a = 0; a < 3; ++a) f[a] = wave_sum(f[a]);
  for (int k = 0; k < 9; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
    const double sF = gE ? -gE[0] : 1.0;
    const double sV = gE ? gE[0] : 1.0;
    for (int a = 0; a < 3; ++a) Fout[3 * i + a] = sF * f[a];
    for (int k = 0; k < 9; ++k) vpart[9 * (size_t)i + k] = sV * v[k];
  }
}

// One-sided pairs (only after a list overflow): subtract g_ij from F_j.
__global__ void k_forces_onesided(const float4 *__restrict__ g, const int *__restrict__ nlist,
                                  const int *__restrict__ nnei, const int *__restrict__ rev, int n,
                                  const double *__restrict__ gE, double *__restrict__ Fout) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * SEL) return;
  const int i = (int)(t / SEL), s = (int)(t % SEL);
  if (s >= nnei[i] || rev[t] >= 0) return;
  const int j = nlist[t];
  if (j < 0 || j >= n) return;
  const float4 gi = g[t];
  const double sF = gE ? -gE[0] : 1.0;
  atomicAdd(&Fout[3 * j], -sF * gi.x);
  atomicAdd(&Fout[3 * j + 1], -sF * gi.y);
  atomicAdd(&Fout[3 * j + 2], -sF * gi.z);
}

struct Neu {
  double s, c;
};
__device__ __forceinline__ void neu_add(Neu &a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
  else a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ void neu_merge(Neu &a, const Neu &b) {
  neu_add(a, b.s);
  a.c += b.c;
}

// Block-wide Neumaier sum of src[k * stride] for k < count (fixed order); one block per output.
template <typename S>
__global__ void __launch_bounds__(1024) k_neumaier(const S *__restrict__ src, int count, int stride,
                                                   double *__restrict__ out, double *__restrict__ copy_out) {
  __shared__ double ss[1024], sc[1024];
  const int comp = blockIdx.x;
  Neu a{0.0, 0.0};
  for (int k = threadIdx.x; k < count; k += 1024) {
    const double x = (double)src[(size_t)k * stride + comp];
    neu_add(a, x);
    if (copy_out) copy_out[k] = x;
  }
  ss[threadIdx.x] = a.s;
  sc[threadIdx.x] = a.c;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      Neu x{ss[threadIdx.x], sc[threadIdx.x]};
      neu_merge(x, Neu{ss[threadIdx.x + h], sc[threadIdx.x + h]});
      ss[threadIdx.x] = x.s;
      sc[threadIdx.x] = x.c;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[comp] = ss[0] + sc[0];
}

}  // namespace

void launch_forces(const Workspace &ws, const double *coords, int n, const Grid &g, bool grid_on_device,
                   const double *gE, double *forces, double *virial_out, hipStream_t st) {
  const Grid *dg = grid_on_device ? ws.grid : nullptr;
  hipLaunchKernelGGL(k_forces, dim3((n + 3) / 4), dim3(256), 0, st, ws.g, ws.nlist, ws.nnei, ws.rev, coords, g, dg,
                     n, gE, forces, ws.vpart);
  const long long tot = (long long)n * SEL;
  hipLaunchKernelGGL(k_forces_onesided, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, ws.g, ws.nlist,
                     ws.nnei, ws.rev, n, gE, forces);
  if (virial_out)
    hipLaunchKernelGGL(k_neumaier<double>, dim3(9), dim3(1024), 0, st, ws.vpart, n, 9, virial_out,
                       (double *)nullptr);
}

void launch_energy(const Workspace &ws, int n, double *energy, double *atom_energy, hipStream_t st) {
  hipLaunchKernelGGL(k_neumaier<double>, dim3(1), dim3(1024), 0, st, ws.Ei, n, 1, energy, atom_energy);
}

}  // namespace dp
