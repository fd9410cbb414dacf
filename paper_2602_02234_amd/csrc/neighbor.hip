// Cell-list neighbour search on gfx950.
//
// Neighbour lists within the model cutoff over periodic boundaries (paper,
// Sections I-II: short-range work restricted to atoms within a cutoff through
// Verlet neighbour lists; Section IV: 0.6 nm model cutoff).  The inclusion rule
// is exact float64 so that the lists can be compared bit for bit with an
// independent search:  Delta = x_j - x_i;  Delta_a -= L_a * rint(Delta_a * invL_a)
// (periodic axes, half-to-even, every operation rounded separately);
// d2 = (Dx*Dx + Dy*Dy) + Dz*Dz;  neighbour iff d2 < rc*rc;  sorted by j;  with
// more than SEL qualifying, the SEL smallest by (d2, j) are kept.
//
// This file is built with -ffp-contract=off; the pragma keeps that true here.
#pragma clang fp contract(off)

#include "dp_internal.h"

namespace dp {
namespace {

__device__ __forceinline__ Grid load_grid(const Grid &g, const Grid *dg) { return dg ? *dg : g; }

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bounding box of the atoms for open boundaries; one workgroup.
__global__ void __launch_bounds__(1024) k_grid_open(const double *__restrict__ X, int n, double rc,
                                                    Grid *__restrict__ out, unsigned *__restrict__ flags) {
  __shared__ double smin[3][1024], smax[3][1024];
  double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
  bool bad = false;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      const double v = X[3 * i + a];
      if (!isfinite(v)) { bad = true; continue; }
      lo[a] = fmin(lo[a], v);
      hi[a] = fmax(hi[a], v);
    }
  }
  if (bad) atomicOr(flags, FLAG_NONFINITE);
  for (int a = 0; a < 3; ++a) { smin[a][threadIdx.x] = lo[a]; smax[a][threadIdx.x] = hi[a]; }
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s)
      for (int a = 0; a < 3; ++a) {
        smin[a][threadIdx.x] = fmin(smin[a][threadIdx.x], smin[a][threadIdx.x + s]);
        smax[a][threadIdx.x] = fmax(smax[a][threadIdx.x], smax[a][threadIdx.x + s]);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    Grid g;
    g.periodic = 0;
    int nct = 1;
    for (int a = 0; a < 3; ++a) {
      double o = smin[a][0], e = smax[a][0] - smin[a][0];
      if (!(e > 0.0)) e = 1.0;
      if (!isfinite(o)) { o = 0.0; e = 1.0; }
      int nc = (int)floor(e / (rc * (1.0 + 1e-9)));
      nc = clampi(nc, 1, MAX_CELLS_PER_DIM);
      g.origin[a] = o;
      g.L[a] = e;
      g.invL[a] = 1.0 / e;
      g.nc[a] = nc;
      g.cw[a] = e / nc;
      g.icw[a] = nc / e;
      nct *= nc;
    }
    g.ncells = nct;
    *out = g;
  }
}

__global__ void k_fill_int(int *__restrict__ p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void k_cell_assign(const double *__restrict__ X, const int *__restrict__ types, int n, int ntypes,
                              Grid hg, const Grid *__restrict__ dg, int *__restrict__ cell_of,
                              int *__restrict__ cell_count, unsigned *__restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Grid g = load_grid(hg, dg);
  const int t = types[i];
  if (t < 0 || t >= ntypes) atomicOr(flags, FLAG_TYPE);
  int c[3];
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    const double x = X[3 * i + a];
    if (!isfinite(x)) { ok = false; c[a] = 0; continue; }
    double w;
    if (g.periodic) w = x - g.L[a] * floor(x * g.invL[a]);
    else w = x - g.origin[a];
    c[a] = clampi((int)floor(w * g.icw[a]), 0, g.nc[a] - 1);
  }
  if (!ok) atomicOr(flags, FLAG_NONFINITE);
  const int cell = (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
  cell_of[i] = cell;
  atomicAdd(&cell_count[cell], 1);
}

// Exclusive scan of the cell counts; one workgroup of 1024 threads.
__global__ void __launch_bounds__(1024) k_cell_scan(const int *__restrict__ count, int *__restrict__ start,
                                                    int *__restrict__ cursor, Grid hg, const Grid *__restrict__ dg) {
  __shared__ int part[1024];
  const Grid g = load_grid(hg, dg);
  const int nc = g.ncells;
  const int per = (nc + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(nc, b + per);
  int s = 0;
  for (int c = b; c < e; ++c) s += count[c];
  part[threadIdx.x] = s;
  __syncthreads();
  // Hillis-Steele inclusive scan over the 1024 partial sums
  for (int off = 1; off < 1024; off <<= 1) {
    int v = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int c = b; c < e; ++c) {
    start[c] = run;
    cursor[c] = run;
    run += count[c];
  }
  if (threadIdx.x == 1023) start[nc] = part[1023];
}

__global__ void k_cell_fill(const int *__restrict__ cell_of, int *__restrict__ cursor, int *__restrict__ atoms, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = atomicAdd(&cursor[cell_of[i]], 1);
  atoms[p] = i;
}

// Distinct stencil cells along one axis (deduplicated when nc < 3; clipped when open).
__device__ __forceinline__ int stencil_axis(int c, int nc, int periodic, int out[3]) {
  int k = 0;
  for (int o = -1; o <= 1; ++o) {
    int v = c + o;
    if (periodic) v = (v + nc) % nc;
    else if (v < 0 || v >= nc) continue;
    bool dup = false;
    for (int q = 0; q < k; ++q) dup |= (out[q] == v);
    if (!dup) out[k++] = v;
  }
  return k;
}

// One wavefront (one workgroup of 64) per atom.
__global__ void __launch_bounds__(64) k_nlist(const double *__restrict__ X, int n, Grid hg, const Grid *__restrict__ dg,
                                              double rc2, const int *__restrict__ cell_of,
                                              const int *__restrict__ cell_start, const int *__restrict__ cell_atoms,
                                              int *__restrict__ nlist, int *__restrict__ nnei,
                                              unsigned *__restrict__ flags) {
  __shared__ int cj[CAND_CAP];
  __shared__ double cd2[CAND_CAP];
  __shared__ int keep[CAND_CAP];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int lane = threadIdx.x;
  const Grid g = load_grid(hg, dg);
  const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
  const int cell = cell_of[i];
  const int cz = cell % g.nc[2], cy = (cell / g.nc[2]) % g.nc[1], cx = cell / (g.nc[1] * g.nc[2]);
  int sx[3], sy[3], sz[3];
  const int nx = stencil_axis(cx, g.nc[0], g.periodic, sx);
  const int ny = stencil_axis(cy, g.nc[1], g.periodic, sy);
  const int nz = stencil_axis(cz, g.nc[2], g.periodic, sz);
  int count = 0;
  bool overlap = false;
  for (int a = 0; a < nx; ++a)
    for (int b = 0; b < ny; ++b)
      for (int c = 0; c < nz; ++c) {
        const int cc = (sx[a] * g.nc[1] + sy[b]) * g.nc[2] + sz[c];
        const int s0 = cell_start[cc], s1 = cell_start[cc + 1];
        for (int p = s0; p < s1; p += 64) {
          const int q = p + lane;
          int j = -1;
          double d2 = 0.0;
          bool acc = false;
          if (q < s1) {
            j = cell_atoms[q];
            if (j != i) {
              double dx = __dsub_rn(X[3 * j], xi), dy = __dsub_rn(X[3 * j + 1], yi), dz = __dsub_rn(X[3 * j + 2], zi);
              if (g.periodic) {
                dx = __dsub_rn(dx, __dmul_rn(g.L[0], rint(__dmul_rn(dx, g.invL[0]))));
                dy = __dsub_rn(dy, __dmul_rn(g.L[1], rint(__dmul_rn(dy, g.invL[1]))));
                dz = __dsub_rn(dz, __dmul_rn(g.L[2], rint(__dmul_rn(dz, g.invL[2]))));
              }
              d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
              acc = d2 < rc2;
              overlap |= (d2 == 0.0);
            }
          }
          const unsigned long long mask = __ballot(acc);
          const int pos = count + __popcll(mask & ((1ull << lane) - 1ull));
          if (acc && pos < CAND_CAP) { cj[pos] = j; cd2[pos] = d2; }
          count += __popcll(mask);
        }
      }
  if (overlap) atomicOr(flags, FLAG_OVERLAP);
  if (count > CAND_CAP) {
    if (lane == 0) atomicOr(flags, FLAG_TOO_DENSE);
    count = CAND_CAP;
  }
  __syncthreads();
  int *row = nlist + (size_t)i * SEL;
  if (count <= SEL) {
    for (int e = lane; e < count; e += 64) {
      const int j = cj[e];
      int rank = 0;
      for (int f = 0; f < count; ++f) rank += cj[f] < j;
      row[rank] = j;
    }
    for (int r = count + lane; r < SEL; r += 64) row[r] = -1;
    if (lane == 0) nnei[i] = count;
  } else {
    for (int e = lane; e < count; e += 64) {
      const int j = cj[e];
      const double d = cd2[e];
      int rank = 0;
      for (int f = 0; f < count; ++f) rank += (cd2[f] < d) || (cd2[f] == d && cj[f] < j);
      keep[e] = rank < SEL;
    }
    __syncthreads();
    for (int e = lane; e < count; e += 64) {
      if (!keep[e]) continue;
      const int j = cj[e];
      int rank = 0;
      for (int f = 0; f < count; ++f) rank += keep[f] && cj[f] < j;
      row[rank] = j;
    }
    if (lane == 0) {
      nnei[i] = SEL;
      atomicAdd(flags + 1, 1u);
    }
  }
}

// rev[i][s] = slot of i in the list of j = nlist[i][s], or -1 (lists sorted ascending).
__global__ void k_rev(const int *__restrict__ nlist, const int *__restrict__ nnei, int *__restrict__ rev, int n,
                      unsigned *__restrict__ flags) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)n * SEL) return;
  const int i = (int)(t / SEL), s = (int)(t % SEL);
  int r = -1;
  if (s < nnei[i]) {
    const int j = nlist[t];
    if (j < 0 || j >= n) {
      rev[t] = -1;
      return;
    }
    const int *row = nlist + (size_t)j * SEL;
    int lo = 0, hi = min(nnei[j], SEL) - 1;
    while (lo <= hi) {
      const int mid = (lo + hi) >> 1;
      const int v = row[mid];
      if (v == i) { r = mid; break; }
      if (v < i) lo = mid + 1; else hi = mid - 1;
    }
    if (r < 0) atomicAdd(flags + 2, 1u);
  }
  rev[t] = r;
}

}  // namespace

void launch_neighbors(const Workspace &ws, const double *coords, const int *types, int n, int ntypes, const Grid &g,
                      bool grid_on_device, double rc, hipStream_t st) {
  const Grid *dg = grid_on_device ? ws.grid : nullptr;
  if (grid_on_device)
    hipLaunchKernelGGL(k_grid_open, dim3(1), dim3(1024), 0, st, coords, n, rc, ws.grid, ws.flags);
  const int ncell_alloc = grid_on_device ? MAX_CELLS : g.ncells;
  hipLaunchKernelGGL(k_fill_int, dim3((ncell_alloc + 1 + 255) / 256), dim3(256), 0, st, ws.cell_count,
                     ncell_alloc + 1, 0);
  hipLaunchKernelGGL(k_cell_assign, dim3((n + 255) / 256), dim3(256), 0, st, coords, types, n, ntypes, g, dg,
                     ws.cell_of, ws.cell_count, ws.flags);
  hipLaunchKernelGGL(k_cell_scan, dim3(1), dim3(1024), 0, st, ws.cell_count, ws.cell_start, ws.cell_cursor, g, dg);
  hipLaunchKernelGGL(k_cell_fill, dim3((n + 255) / 256), dim3(256), 0, st, ws.cell_of, ws.cell_cursor,
                     ws.cell_atoms, n);
  hipLaunchKernelGGL(k_nlist, dim3(n), dim3(64), 0, st, coords, n, g, dg, rc * rc, ws.cell_of, ws.cell_start,
                     ws.cell_atoms, ws.nlist, ws.nnei, ws.flags);
  const long long tot = (long long)n * SEL;
  hipLaunchKernelGGL(k_rev, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, ws.nlist, ws.nnei, ws.rev, n,
                     ws.flags);
}

}  // namespace dp
