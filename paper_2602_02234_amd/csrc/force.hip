// Force assembly, virial and the compensated float64 reductions on gfx950.
//   F_i = sum_{j in N(i)} g_ij - sum_{j : i in N(j)} g_ji     (F = -dE/dx)
//   Xi_ab = - sum_i sum_{j in N(i)} Delta_ij,a g_ij,b
// One kernel gathers F_i without atomics: for each j in N(i) the slot of i in N(j) is
// found by binary search (lists are sorted), and g_ji subtracted.  A pair can be
// one-sided (i in N(c) but c not in N(i)) only after a list was truncated to sel, or
// when i is a ghost atom without a list; then the atoms c of i's cell neighbourhood (or
// skin row) are searched as well, and their terms summed in fixed point, exactly and in
// any order.  The virial of each system is reduced by the last workgroup to finish its
// atoms, in float64 with Neumaier compensation and a fixed order.
#include <algorithm>

#include "dp_reduce.h"

namespace dp {
namespace {

__device__ __forceinline__ double wave_sum(double v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}
__device__ __forceinline__ long long wave_sum_ll(long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Outputs are written only when the step raised no error flag, so that a failed step
// leaves the caller's buffers as they were (the status is read back after the step).
__device__ __forceinline__ bool step_failed(const unsigned *flags) { return (flags[0] & FLAG_ERRORS) != 0u; }

// Slot of v in the ascending list row[0 .. len), or -1.
__device__ __forceinline__ int find_slot(const int *__restrict__ row, int len, int v) {
  int lo = 0, hi = len - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int x = row[mid];
    if (x == v) return mid;
    if (x < v) lo = mid + 1; else hi = mid - 1;
  }
  return -1;
}

// One-sided terms are rounded to multiples of 2^-36 eV/A and summed in int64: exact, so
// the result does not depend on the order the candidates are visited in.
constexpr double FIX = 68719476736.0;  // 2^36

// One wavefront per atom, four per workgroup.  gE == NULL: out = F;  else out = -gE F =
// gE dE/dx, virial scaled by gE.  one_sided != 0 (a list was truncated, or there are
// ghost atoms): also gather the one-sided terms.
__global__ void __launch_bounds__(256) k_forces(
    const float4 *__restrict__ g, const int *__restrict__ nlist, const int *__restrict__ nnei,
    const double *__restrict__ X, const Grid *__restrict__ grids, const int *__restrict__ sys_of, int n,
    const double *__restrict__ gE, double *__restrict__ Fout, double *__restrict__ vpart,
    const int *__restrict__ cell_of, const int *__restrict__ cell_start, const int *__restrict__ cell_atoms,
    const int *__restrict__ slist, const int *__restrict__ snnei, int skin_rows, int ghosts,
    const unsigned *__restrict__ flags) {
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i < n && !step_failed(flags)) {
    const Grid gr = grids[sys_of[i]];
    double f[3] = {0, 0, 0}, v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    const int nn = min(max(nnei[i], 0), SEL);
    const int *rowi = nlist + (size_t)i * SEL;
    for (int s = lane; s < nn; s += 64) {
      const float4 gi = g[(size_t)i * SEL + s];
      int j = rowi[s];
      if (j < 0 || j >= n) j = i;  // never read outside the arrays
      f[0] += gi.x; f[1] += gi.y; f[2] += gi.z;
      const int r = find_slot(nlist + (size_t)j * SEL, min(max(nnei[j], 0), SEL), i);
      if (r >= 0) {
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
    if (ghosts || flags[1] != 0u) {
      // the atoms c with i in N(c) but c not in N(i): they lie within rc of i
      long long q[3] = {0, 0, 0};
      auto consider = [&](int c) {
        if (c < 0 || c >= n || c == i) return;
        const int slot = find_slot(nlist + (size_t)c * SEL, min(max(nnei[c], 0), SEL), i);
        if (slot < 0 || find_slot(rowi, nn, c) >= 0) return;
        const float4 gc = g[(size_t)c * SEL + slot];
        q[0] += llrint((double)gc.x * FIX);
        q[1] += llrint((double)gc.y * FIX);
        q[2] += llrint((double)gc.z * FIX);
      };
      if (skin_rows) {
        const int ns = min(max(snnei[i], 0), SKIN_CAP);
        for (int p = lane; p < ns; p += 64) consider(slist[(size_t)i * SKIN_CAP + p]);
      } else {
        const int cell = min(max(cell_of[i] - gr.cell_base, 0), gr.ncells - 1);
        const int cc[3] = {cell / (gr.nc[1] * gr.nc[2]), (cell / gr.nc[2]) % gr.nc[1], cell % gr.nc[2]};
        int st[3][3], ns[3];
        for (int a = 0; a < 3; ++a) {  // distinct stencil cells along each axis
          ns[a] = 0;
          for (int o = -1; o <= 1; ++o) {
            int w = cc[a] + o;
            if (gr.periodic) w = (w + gr.nc[a]) % gr.nc[a];
            else if (w < 0 || w >= gr.nc[a]) continue;
            bool dup = false;
            for (int k = 0; k < ns[a]; ++k) dup |= st[a][k] == w;
            if (!dup) st[a][ns[a]++] = w;
          }
        }
        for (int x = 0; x < ns[0]; ++x)
          for (int y = 0; y < ns[1]; ++y)
            for (int z = 0; z < ns[2]; ++z) {
              const int c = gr.cell_base + (st[0][x] * gr.nc[1] + st[1][y]) * gr.nc[2] + st[2][z];
              for (int p = cell_start[c] + lane; p < cell_start[c + 1]; p += 64) consider(cell_atoms[p]);
            }
      }
      for (int a = 0; a < 3; ++a) f[a] -= (double)wave_sum_ll(q[a]) / FIX;
    }
    if (lane == 0) {
      const double sF = gE ? -gE[0] : 1.0;
      const double sV = gE ? gE[0] : 1.0;
      for (int a = 0; a < 3; ++a) Fout[3 * i + a] = sF * f[a];
      for (int k = 0; k < 9; ++k) vpart[9 * (size_t)i + k] = sV * v[k];
    }
  }
}

// Per-system float64 sums in a fixed order, one workgroup per (system, component):
// component 0 the energy (E_i over the energy ranges eoff[s] .. eoff[s+1]-1, copied to
// atom_energy when given), components 1..nv the virial (vpart over off[s] .. off[s+1]-1,
// nv = 9 or 0), then one per fitting head when there are several (Eh into Ehsys).
// A system's sums do not depend on which other systems share the step.
__global__ void __launch_bounds__(1024) k_reduce(const double *__restrict__ Ei, const double *__restrict__ vpart,
                                                 const double *__restrict__ Eh, const int *__restrict__ eoff,
                                                 const int *__restrict__ off, int ncomp, int nv,
                                                 double *__restrict__ energy, double *__restrict__ atom_energy,
                                                 double *__restrict__ virial, double *__restrict__ Ehsys,
                                                 const unsigned *__restrict__ flags) {
  __shared__ double ss[1024], sc[1024];
  if (step_failed(flags)) return;
  const int comp = blockIdx.x % ncomp, s = blockIdx.x / ncomp;
  if (comp > nv) {
    const int h = comp - nv - 1;
    const double E = block_neumaier<1024>(Eh, eoff[s], eoff[s + 1], MAXH, h, ss, sc);
    if (threadIdx.x == 0) Ehsys[s * MAXH + h] = E;
  } else if (comp == 0) {
    const double E = block_neumaier<1024>(Ei, eoff[s], eoff[s + 1], 1, 0, ss, sc);
    if (energy && threadIdx.x == 0) energy[s] = E;
    if (atom_energy)
      for (int k = eoff[s] + (int)threadIdx.x; k < eoff[s + 1]; k += 1024) atom_energy[k] = Ei[k];
  } else {
    const double V = block_neumaier<1024>(vpart, off[s], off[s + 1], 9, comp - 1, ss, sc);
    if (threadIdx.x == 0) virial[9 * s + comp - 1] = V;
  }
}

// out[0] = sum of src over the atoms of system 0 (fixed order).
__global__ void __launch_bounds__(1024) k_sum(const double *__restrict__ src, const int *__restrict__ off,
                                              double *__restrict__ out) {
  __shared__ double ss[1024], sc[1024];
  const double v = block_neumaier<1024>(src, off[0], off[1], 1, 0, ss, sc);
  if (threadIdx.x == 0) out[0] = v;
}

}  // namespace

void launch_forces(const Workspace &ws, const double *coords, int n, const double *gE, double *forces,
                   bool skin_rows, bool ghosts, hipStream_t st) {
  hipLaunchKernelGGL(k_forces, dim3((n + 3) / 4), dim3(256), 0, st, ws.g, ws.nlist, ws.nnei, coords, ws.grids,
                     ws.sys_of, n, gE, forces, ws.vpart, ws.cell_of, ws.cell_start, ws.cell_atoms, ws.slist, ws.snnei,
                     skin_rows ? 1 : 0, ghosts ? 1 : 0, ws.flags);
}

void launch_reduce(const Workspace &ws, const int *eoff, int nsys, double *energy, double *atom_energy,
                   double *virial, int nheads, hipStream_t st) {
  const int nv = virial ? 9 : 0;
  const int ncomp = 1 + nv + (nheads > 1 ? nheads : 0);
  hipLaunchKernelGGL(k_reduce, dim3(nsys * ncomp), dim3(1024), 0, st, ws.Ei, ws.vpart, ws.Eh, eoff, ws.sys_off, ncomp,
                     nv, energy, atom_energy, virial, ws.Ehsys, ws.flags);
}

void launch_sum(const Workspace &ws, const double *src, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, src, ws.sys_off, out);
}

}  // namespace dp
