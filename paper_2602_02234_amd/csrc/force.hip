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

// Outputs are written only when the step raised no error flag, so that a failed step
// leaves the caller's buffers as they were (the status is read back after the step).
__device__ __forceinline__ bool step_failed(const unsigned *flags) { return (flags[0] & FLAG_ERRORS) != 0u; }

// One wavefront per atom.  gE == NULL: out = F;  else out = -gE F = gE dE/dx, virial scaled by gE.
__global__ void __launch_bounds__(256) k_forces(const float4 *__restrict__ g, const int *__restrict__ nlist,
                                                const int *__restrict__ nnei, const int *__restrict__ rev,
                                                const double *__restrict__ X, const Grid *__restrict__ grids,
                                                const int *__restrict__ sys_of, int n, const double *__restrict__ gE,
                                                double *__restrict__ Fout, double *__restrict__ vpart,
                                                const unsigned *__restrict__ flags) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n || step_failed(flags)) return;
  const Grid gr = grids[sys_of[i]];
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
                                  const double *__restrict__ gE, double *__restrict__ Fout,
                                  const unsigned *__restrict__ flags) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * SEL || flags[2] == 0u || step_failed(flags)) return;
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

// Per-system Neumaier sums in a fixed order: block b reduces component c = b % ncomp of
// system s = b / ncomp, i.e. src[k * ncomp + c] for off[s] <= k < off[s + 1], into
// out[s * ncomp + c].  Thread t takes the elements off[s] + t, off[s] + t + 1024, ...,
// so a system's sums do not depend on which other systems share the step.
__global__ void __launch_bounds__(1024) k_seg_neumaier(const double *__restrict__ src, const int *__restrict__ off,
                                                       int ncomp, double *__restrict__ out,
                                                       double *__restrict__ copy_out,
                                                       const unsigned *__restrict__ flags) {
  __shared__ double ss[1024], sc[1024];
  if (step_failed(flags)) return;
  const int comp = blockIdx.x % ncomp, s = blockIdx.x / ncomp;
  const int k0 = off[s], k1 = off[s + 1];
  Neu a{0.0, 0.0};
  for (int k = k0 + threadIdx.x; k < k1; k += 1024) {
    const double x = src[(size_t)k * ncomp + comp];
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
  if (threadIdx.x == 0) out[(size_t)s * ncomp + comp] = ss[0] + sc[0];
}

}  // namespace

void launch_forces(const Workspace &ws, const double *coords, int n, int nsys, const double *gE, double *forces,
                   double *virial_out, hipStream_t st) {
  hipLaunchKernelGGL(k_forces, dim3((n + 3) / 4), dim3(256), 0, st, ws.g, ws.nlist, ws.nnei, ws.rev, coords,
                     ws.grids, ws.sys_of, n, gE, forces, ws.vpart, ws.flags);
  const long long tot = (long long)n * SEL;
  hipLaunchKernelGGL(k_forces_onesided, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, ws.g, ws.nlist,
                     ws.nnei, ws.rev, n, gE, forces, ws.flags);
  if (virial_out)
    hipLaunchKernelGGL(k_seg_neumaier, dim3(9 * nsys), dim3(1024), 0, st, ws.vpart, ws.sys_off, 9, virial_out,
                       (double *)nullptr, ws.flags);
}

void launch_sum(const Workspace &ws, const double *src, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_neumaier, dim3(1), dim3(1024), 0, st, src, ws.sys_off, 1, out, (double *)nullptr,
                     ws.flags);
}

void launch_energy(const Workspace &ws, int nsys, double *energy, double *atom_energy, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_neumaier, dim3(nsys), dim3(1024), 0, st, ws.Ei, ws.sys_off, 1, energy, atom_energy,
                     ws.flags);
}

}  // namespace dp
