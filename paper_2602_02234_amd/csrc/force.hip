// Force assembly, virial and the compensated float64 reductions on gfx950.
//   F_i = sum_{j in N(i)} g_ij - sum_{j : i in N(j)} g_ji     (F = -dE/dx)
//   Xi_ab = - sum_i sum_{j in N(i)} Delta_ij,a g_ij,b
// The second force term is gathered through rev[][] (slot of i in the list of
// j), so no floating-point atomics are needed.  An atom whose list overflowed can
// leave a pair one-sided; those terms are gathered by a second pass over each
// atom's cell neighbours, in a fixed order.  E and Xi are reduced per
// system in float64 with Neumaier compensation in a fixed order.
#include <algorithm>

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

// One-sided pairs (only after a list overflow, counted in flags[2] by the reverse-slot
// pass): F_i -= sum of g_ci over the atoms c with i in N(c) but c not in N(i).  Such a c
// lies within rc of i, so it is among the atoms of i's stencil cells (lists made this
// step) or of i's skin row (reused skin lists).  The terms are summed in float64 in
// ascending c, so the forces do not depend on the order the cells were filled in.
// Grid-stride over atoms: without one-sided pairs every workgroup returns at once.
__global__ void __launch_bounds__(64) k_forces_onesided(
    const float4 *__restrict__ g, const int *__restrict__ nlist, const int *__restrict__ nnei,
    const int *__restrict__ rev, const Grid *__restrict__ grids, const int *__restrict__ sys_of,
    const int *__restrict__ cell_of, const int *__restrict__ cell_start, const int *__restrict__ cell_atoms,
    const int *__restrict__ slist, const int *__restrict__ snnei, int skin_rows, int n,
    const double *__restrict__ gE, double *__restrict__ Fout, const unsigned *__restrict__ flags) {
  __shared__ int oc[CAND_CAP];
  __shared__ float4 og[CAND_CAP], sg[CAND_CAP];
  if (flags[2] == 0u || step_failed(flags)) return;
  const int lane = threadIdx.x;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    int count = 0;
    // candidate c: keep it if i is in c's list at a slot whose pair is one-sided
    auto consider = [&](int c) {
      int slot = -1;
      if (c >= 0 && c < n && c != i) {
        const int *row = nlist + (size_t)c * SEL;
        int lo = 0, hi = min(max(nnei[c], 0), SEL) - 1;
        while (lo <= hi) {
          const int mid = (lo + hi) >> 1;
          const int v = row[mid];
          if (v == i) { slot = mid; break; }
          if (v < i) lo = mid + 1; else hi = mid - 1;
        }
        if (slot >= 0 && rev[(size_t)c * SEL + slot] >= 0) slot = -1;
      }
      const unsigned long long mask = __ballot(slot >= 0);
      const int pos = count + __popcll(mask & ((1ull << lane) - 1ull));
      if (slot >= 0 && pos < CAND_CAP) {
        oc[pos] = c;
        og[pos] = g[(size_t)c * SEL + slot];
      }
      count += __popcll(mask);
    };
    if (skin_rows) {
      const int ns = min(max(snnei[i], 0), SKIN_CAP);
      for (int p = 0; p < ns; p += 64) consider(p + lane < ns ? slist[(size_t)i * SKIN_CAP + p + lane] : -1);
    } else {
      const Grid gr = grids[sys_of[i]];
      const int cell = min(max(cell_of[i] - gr.cell_base, 0), gr.ncells - 1);
      const int cz = cell % gr.nc[2], cy = (cell / gr.nc[2]) % gr.nc[1], cx = cell / (gr.nc[1] * gr.nc[2]);
      int st[3][3], ns[3];
      const int cc[3] = {cx, cy, cz};
      for (int a = 0; a < 3; ++a) {  // distinct stencil cells along each axis
        ns[a] = 0;
        for (int o = -1; o <= 1; ++o) {
          int v = cc[a] + o;
          if (gr.periodic) v = (v + gr.nc[a]) % gr.nc[a];
          else if (v < 0 || v >= gr.nc[a]) continue;
          bool dup = false;
          for (int q = 0; q < ns[a]; ++q) dup |= st[a][q] == v;
          if (!dup) st[a][ns[a]++] = v;
        }
      }
      for (int x = 0; x < ns[0]; ++x)
        for (int y = 0; y < ns[1]; ++y)
          for (int z = 0; z < ns[2]; ++z) {
            const int c = gr.cell_base + (st[0][x] * gr.nc[1] + st[1][y]) * gr.nc[2] + st[2][z];
            const int s0 = cell_start[c], s1 = cell_start[c + 1];
            for (int p = s0; p < s1; p += 64) consider(p + lane < s1 ? cell_atoms[p + lane] : -1);
          }
    }
    count = min(count, CAND_CAP);
    __syncthreads();
    for (int e = lane; e < count; e += 64) {  // the candidates are distinct: rank by index
      int rank = 0;
      for (int f = 0; f < count; ++f) rank += oc[f] < oc[e];
      sg[rank] = og[e];
    }
    __syncthreads();
    if (lane == 0 && count > 0) {
      double s[3] = {0.0, 0.0, 0.0};
      for (int e = 0; e < count; ++e) {
        s[0] += sg[e].x;
        s[1] += sg[e].y;
        s[2] += sg[e].z;
      }
      const double sF = gE ? -gE[0] : 1.0;
      for (int a = 0; a < 3; ++a) Fout[3 * i + a] -= sF * s[a];
    }
    __syncthreads();
  }
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
                   double *virial_out, bool skin_rows, hipStream_t st) {
  hipLaunchKernelGGL(k_forces, dim3((n + 3) / 4), dim3(256), 0, st, ws.g, ws.nlist, ws.nnei, ws.rev, coords,
                     ws.grids, ws.sys_of, n, gE, forces, ws.vpart, ws.flags);
  hipLaunchKernelGGL(k_forces_onesided, dim3((unsigned)std::min(n, 2048)), dim3(64), 0, st, ws.g, ws.nlist,
                     ws.nnei, ws.rev, ws.grids, ws.sys_of, ws.cell_of, ws.cell_start, ws.cell_atoms, ws.slist,
                     ws.snnei, skin_rows ? 1 : 0, n, gE, forces, ws.flags);
  if (virial_out)
    hipLaunchKernelGGL(k_seg_neumaier, dim3(9 * nsys), dim3(1024), 0, st, ws.vpart, ws.sys_off, 9, virial_out,
                       (double *)nullptr, ws.flags);
}

void launch_sum(const Workspace &ws, const double *src, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_seg_neumaier, dim3(1), dim3(1024), 0, st, src, ws.sys_off, 1, out, (double *)nullptr,
                     ws.flags);
}

void launch_energy(const Workspace &ws, const int *off, int nsys, double *energy, double *atom_energy,
                   hipStream_t st) {
  hipLaunchKernelGGL(k_seg_neumaier, dim3(nsys), dim3(1024), 0, st, ws.Ei, off, 1, energy, atom_energy, ws.flags);
}

}  // namespace dp
