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

#include <algorithm>

#include "dp_internal.h"

namespace dp {
namespace {

__device__ __forceinline__ int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// Bounding box of the atoms of a single open-boundary system -> grids[0]; one workgroup.
__global__ void __launch_bounds__(1024) k_grid_open(const double *__restrict__ X, int n, double cutoff,
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
    g.cell_base = 0;
    int nct = 1;
    for (int a = 0; a < 3; ++a) {
      double o = smin[a][0], e = smax[a][0] - smin[a][0];
      if (!(e > 0.0)) e = 1.0;
      if (!isfinite(o)) { o = 0.0; e = 1.0; }
      int nc = (int)floor(e / (cutoff * (1.0 + 1e-9)));
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

// Start of a step: clears the status words (nflags of them), the completion counters
// (ndone) and the backward instances' atom counts, clears the cell counts (ncz entries),
// and writes sys_of[a] = s for off[s] <= a < off[s + 1], a < n.  Grid-stride; no
// workgroup depends on another.
__global__ void k_prologue(const int *__restrict__ off, int nsys, int n, int *__restrict__ sys_of,
                           int *__restrict__ cell_count, int ncz, unsigned *__restrict__ flags, int nflags,
                           int *__restrict__ done, int ndone, int *__restrict__ bcnt) {
  const int stride = gridDim.x * blockDim.x;
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < max(max(n, ncz), max(ndone, 2)); t += stride) {
    if (t < nflags) flags[t] = 0u;
    if (t < 2) bcnt[t] = 0;
    if (t < ndone) done[t] = 0;
    if (t < ncz) cell_count[t] = 0;
    if (t < n) {
      int lo = 0, hi = nsys - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= t) lo = mid; else hi = mid - 1;
      }
      sys_of[t] = lo;
    }
  }
}

// Cell of each atom and the cell counts; the last workgroup to finish then turns the
// counts into start offsets (exclusive scan over the ncells_host cells, or the cell count
// of *open_grid) and resets the fill cursors.  *blocks_done must be zero at the start.
__global__ void __launch_bounds__(1024) k_cell_assign(
    const double *__restrict__ X, const int *__restrict__ types, int n, int ntypes, const Grid *__restrict__ grids,
    const int *__restrict__ sys_of, int *__restrict__ cell_of, int *__restrict__ cell_count,
    int *__restrict__ start, int *__restrict__ cursor, int ncells_host, const Grid *__restrict__ open_grid,
    int *__restrict__ blocks_done, unsigned *__restrict__ flags) {
  __shared__ int part[1024];
  __shared__ bool is_last;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    const Grid g = grids[sys_of[i]];
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
    const int cell = g.cell_base + (c[0] * g.nc[1] + c[1]) * g.nc[2] + c[2];
    cell_of[i] = cell;
    atomicAdd(&cell_count[cell], 1);
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    is_last = atomicAdd(blocks_done, 1) == (int)gridDim.x - 1;
    __threadfence();
  }
  __syncthreads();
  if (!is_last) return;
  // exclusive scan of the cell counts by this (last) workgroup
  const int nc = open_grid ? open_grid->ncells : ncells_host;
  const int per = (nc + 1023) / 1024;
  const int b = threadIdx.x * per, e = min(nc, b + per);
  int sum = 0;
  for (int k = b; k < e; ++k) sum += cell_count[k];
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // Hillis-Steele inclusive scan of the partial sums
    const int v = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  int run = threadIdx.x ? part[threadIdx.x - 1] : 0;
  for (int k = b; k < e; ++k) {
    start[k] = run;
    cursor[k] = run;
    run += cell_count[k];
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

// The canonical float64 squared distance (every operation rounded on its own).
__device__ __forceinline__ double pair_d2(const Grid &g, double xi, double yi, double zi, const double *__restrict__ xj) {
  double dx = __dsub_rn(xj[0], xi), dy = __dsub_rn(xj[1], yi), dz = __dsub_rn(xj[2], zi);
  if (g.periodic) {
    dx = __dsub_rn(dx, __dmul_rn(g.L[0], rint(__dmul_rn(dx, g.invL[0]))));
    dy = __dsub_rn(dy, __dmul_rn(g.L[1], rint(__dmul_rn(dy, g.invL[1]))));
    dz = __dsub_rn(dz, __dmul_rn(g.L[2], rint(__dmul_rn(dz, g.invL[2]))));
  }
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

// Writes a list row from count candidates (cj, cd2) in LDS: sorted by j; with more than
// cap candidates only the cap smallest by (d2, j) are kept.  Returns true on overflow.
__device__ bool write_row(const int *cj, const double *cd2, int *keep, int count, int cap, int *row, int *nnei_out,
                          int lane) {
  if (count <= cap) {
    for (int e = lane; e < count; e += 64) {
      const int j = cj[e];
      int rank = 0;
      for (int f = 0; f < count; ++f) rank += cj[f] < j;
      row[rank] = j;
    }
    for (int r = count + lane; r < cap; r += 64) row[r] = -1;
    if (lane == 0) *nnei_out = count;
    return false;
  }
  for (int e = lane; e < count; e += 64) {
    const int j = cj[e];
    const double d = cd2[e];
    int rank = 0;
    for (int f = 0; f < count; ++f) rank += (cd2[f] < d) || (cd2[f] == d && cj[f] < j);
    keep[e] = rank < cap;
  }
  __syncthreads();
  for (int e = lane; e < count; e += 64) {
    if (!keep[e]) continue;
    const int j = cj[e];
    int rank = 0;
    for (int f = 0; f < count; ++f) rank += keep[f] && cj[f] < j;
    row[rank] = j;
  }
  if (lane == 0) *nnei_out = cap;
  return true;
}

// One wavefront (one workgroup of 64) per atom: every atom of the 27 stencil cells with
// d2 < cut2 (cell edges >= the cutoff), rows of `cap` entries.  skin = 0: the model list
// (overflow counted in flags[1]); skin = 1: the skin list (overflow sets FLAG_SKIN_FULL).
__global__ void __launch_bounds__(64) k_nlist(const double *__restrict__ X, int n, const Grid *__restrict__ grids,
                                              const int *__restrict__ sys_of, double cut2,
                                              const int *__restrict__ cell_of, const int *__restrict__ cell_start,
                                              const int *__restrict__ cell_atoms, int cap, int skin, int i0,
                                              int ncen, int *__restrict__ nlist, int *__restrict__ nnei,
                                              unsigned *__restrict__ flags) {
  __shared__ int cj[CAND_CAP];
  __shared__ double cd2[CAND_CAP];
  __shared__ int keep[CAND_CAP];
  const int i = i0 + blockIdx.x;
  if (i >= n) return;
  const int lane = threadIdx.x;
  if (i >= ncen) {  // not a centre (a ghost atom): an empty list
    if (lane == 0) nnei[i] = 0;
    return;
  }
  const Grid g = grids[sys_of[i]];
  const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
  const int cell = clampi(cell_of[i] - g.cell_base, 0, g.ncells - 1);
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
        const int cc = g.cell_base + (sx[a] * g.nc[1] + sy[b]) * g.nc[2] + sz[c];
        const int s0 = cell_start[cc], s1 = cell_start[cc + 1];
        for (int p = s0; p < s1; p += 64) {
          const int q = p + lane;
          int j = -1;
          double d2 = 0.0;
          bool acc = false;
          if (q < s1) {
            j = cell_atoms[q];
            if (j != i) {
              d2 = pair_d2(g, xi, yi, zi, X + 3 * j);
              acc = d2 < cut2;
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
  const bool ovf = write_row(cj, cd2, keep, count, cap, nlist + (size_t)i * cap, nnei + i, lane);
  if (ovf && lane == 0) {
    if (skin) atomicOr(flags, FLAG_SKIN_FULL);
    else atomicAdd(flags + 1, 1u);
  }
}

// Model list from the skin list: the entries of atom i's skin row with d2 < rc2 at the
// current coordinates, by the same rule as k_nlist (the skin row is sorted by j, and a
// wave-ordered compaction keeps that order).  Identical to a fresh search as long as
// no atom has moved by half the skin since the skin list was built.
__global__ void __launch_bounds__(64) k_filter(const double *__restrict__ X, int n, const Grid *__restrict__ grids,
                                               const int *__restrict__ sys_of, double rc2,
                                               const int *__restrict__ slist, const int *__restrict__ snnei,
                                               int *__restrict__ nlist, int *__restrict__ nnei,
                                               unsigned *__restrict__ flags) {
  __shared__ int cj[SKIN_CAP];
  __shared__ double cd2[SKIN_CAP];
  __shared__ int keep[SKIN_CAP];
  const int i = blockIdx.x;
  if (i >= n) return;
  const int lane = threadIdx.x;
  const Grid g = grids[sys_of[i]];
  const double xi = X[3 * i], yi = X[3 * i + 1], zi = X[3 * i + 2];
  const int ns = min(max(snnei[i], 0), SKIN_CAP);
  int count = 0;
  bool overlap = false;
  for (int p = 0; p < ns; p += 64) {
    const int e = p + lane;
    int j = -1;
    double d2 = 0.0;
    bool acc = false;
    if (e < ns) {
      j = slist[(size_t)i * SKIN_CAP + e];
      if (j >= 0 && j < n && j != i) {
        d2 = pair_d2(g, xi, yi, zi, X + 3 * j);
        acc = d2 < rc2;
        overlap |= (d2 == 0.0);
      }
    }
    const unsigned long long mask = __ballot(acc);
    const int pos = count + __popcll(mask & ((1ull << lane) - 1ull));
    if (acc) { cj[pos] = j; cd2[pos] = d2; }
    count += __popcll(mask);
  }
  if (overlap) atomicOr(flags, FLAG_OVERLAP);
  __syncthreads();
  const bool ovf = write_row(cj, cd2, keep, count, SEL, nlist + (size_t)i * SEL, nnei + i, lane);
  if (ovf && lane == 0) atomicAdd(flags + 1, 1u);
}

// Per-step checks of the skin path (the cell pass, which makes them otherwise, is
// skipped): finite coordinates, types in range, and every displacement since the
// skin list was built below half the skin (else FLAG_STALE).
__global__ void k_skin_check(const double *__restrict__ X, const double *__restrict__ Xref,
                             const int *__restrict__ types, int n, int ntypes, const Grid *__restrict__ grids,
                             const int *__restrict__ sys_of, double lim2, unsigned *__restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Grid g = grids[sys_of[i]];
  const int t = types[i];
  if (t < 0 || t >= ntypes) atomicOr(flags, FLAG_TYPE);
  double d2 = 0.0;
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    const double x = X[3 * i + a];
    if (!isfinite(x)) ok = false;
    double d = x - Xref[3 * i + a];
    if (g.periodic) d -= g.L[a] * rint(d * g.invL[a]);
    d2 += d * d;
  }
  if (!ok) atomicOr(flags, FLAG_NONFINITE);
  else if (!(d2 < lim2)) atomicOr(flags, FLAG_STALE);
}

__global__ void k_copy_f64(const double *__restrict__ src, double *__restrict__ dst, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[i];
}

}  // namespace

void launch_prologue(const Workspace &ws, int nsys, int n, int ncells_zero, bool clear_flags, hipStream_t st) {
  const int work = std::max(n, ncells_zero);
  const int blocks = std::max(1, std::min((work + 255) / 256, 4096));
  hipLaunchKernelGGL(k_prologue, dim3(blocks), dim3(256), 0, st, ws.sys_off, nsys, n, ws.sys_of, ws.cell_count,
                     ncells_zero, ws.flags, clear_flags ? 4 : 0, ws.done, clear_flags ? 2 * ws.cap_sys + 1 : 0,
                     ws.bcnt);
}

namespace {
__global__ void k_require_complete(unsigned *__restrict__ flags) {
  if (threadIdx.x == 0 && flags[1] != 0u) flags[0] |= FLAG_INCOMPLETE;
}
}  // namespace

void launch_require_complete(const Workspace &ws, hipStream_t st) {
  hipLaunchKernelGGL(k_require_complete, dim3(1), dim3(64), 0, st, ws.flags);
}

namespace {
__global__ void __launch_bounds__(256) k_rev_slots(const int *__restrict__ nlist, const int *__restrict__ nnei, int n,
                                                   int *__restrict__ slot) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)n * SEL) return;
  const int i = (int)(t / SEL), j = (int)(t % SEL);
  int s = -1;
  if (j < min(max(nnei[i], 0), SEL)) {
    const int nj = nlist[t];
    if (nj >= 0 && nj < n) {
      const int len = min(max(nnei[nj], 0), SEL);
      const int *row = nlist + (size_t)nj * SEL;
      int lo = 0, hi = len - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int x = row[mid];
        if (x == i) { s = mid; break; }
        if (x < i) lo = mid + 1; else hi = mid - 1;
      }
    }
  }
  slot[t] = s;
}
}  // namespace

void launch_rev_slots(const Workspace &ws, int n, int *slot, hipStream_t st) {
  const int64_t tot = (int64_t)n * SEL;
  if (tot == 0) return;
  hipLaunchKernelGGL(k_rev_slots, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, ws.nlist, ws.nnei, n, slot);
}

void launch_cells(const Workspace &ws, const double *coords, const int *types, int n, int ntypes, bool open_single,
                  int ncells_total, double cell_cutoff, hipStream_t st) {
  if (open_single)
    hipLaunchKernelGGL(k_grid_open, dim3(1), dim3(1024), 0, st, coords, n, cell_cutoff, ws.grids, ws.flags);
  // the block counter of the assign pass is the last completion counter (cleared by the prologue)
  hipLaunchKernelGGL(k_cell_assign, dim3((n + 1023) / 1024), dim3(1024), 0, st, coords, types, n, ntypes, ws.grids,
                     ws.sys_of, ws.cell_of, ws.cell_count, ws.cell_start, ws.cell_cursor, ncells_total,
                     open_single ? ws.grids : (const Grid *)nullptr, ws.done + 2 * ws.cap_sys, ws.flags);
  hipLaunchKernelGGL(k_cell_fill, dim3((n + 255) / 256), dim3(256), 0, st, ws.cell_of, ws.cell_cursor,
                     ws.cell_atoms, n);
}

void launch_nlist(const Workspace &ws, const double *coords, int n, int i0, int i1, int ncen, double cutoff, bool skin,
                  hipStream_t st) {
  hipLaunchKernelGGL(k_nlist, dim3(i1 - i0), dim3(64), 0, st, coords, n, ws.grids, ws.sys_of, cutoff * cutoff,
                     ws.cell_of, ws.cell_start, ws.cell_atoms, skin ? SKIN_CAP : SEL, skin ? 1 : 0, i0, ncen,
                     skin ? ws.slist : ws.nlist, skin ? ws.snnei : ws.nnei, ws.flags);
}

void launch_filter(const Workspace &ws, const double *coords, int n, double rc, hipStream_t st) {
  hipLaunchKernelGGL(k_filter, dim3(n), dim3(64), 0, st, coords, n, ws.grids, ws.sys_of, rc * rc, ws.slist, ws.snnei,
                     ws.nlist, ws.nnei, ws.flags);
}

void launch_skin_check(const Workspace &ws, const double *coords, const int *types, int n, int ntypes, double lim2,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_skin_check, dim3((n + 255) / 256), dim3(256), 0, st, coords, ws.xref, types, n, ntypes,
                     ws.grids, ws.sys_of, lim2, ws.flags);
}

void launch_skin_ref(const Workspace &ws, const double *coords, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_copy_f64, dim3((3 * n + 255) / 256), dim3(256), 0, st, coords, ws.xref, 3 * n);
}

}  // namespace dp
