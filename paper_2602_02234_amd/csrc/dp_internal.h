// Host/device structures shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>

#include "dp_common.h"

namespace dp {

// Cell grid over the box (periodic) or over the atoms' bounding box (open).
struct Grid {
  double origin[3];
  double L[3];      // periodic box edges, or bounding-box extent
  double invL[3];   // 1 / L (periodic minimum image)
  double cw[3];     // cell edge, >= rc (1 + 1e-9) unless there is a single cell
  double icw[3];    // 1 / cw
  int nc[3];
  int periodic;
  int ncells;
};

constexpr int MAX_CELLS_PER_DIM = 64;
constexpr int MAX_CELLS = MAX_CELLS_PER_DIM * MAX_CELLS_PER_DIM * MAX_CELLS_PER_DIM;
constexpr int CAND_CAP = 512;  // neighbours within rc one atom may have before DP_ERR_TOO_LARGE

// Status bits written by kernels into the workspace flag word.
enum : unsigned {
  FLAG_OVERLAP = 1u, FLAG_TYPE = 2u, FLAG_NONFINITE = 4u, FLAG_TOO_DENSE = 8u,
};

// Device weights; T is float (DP_FP32) or __bf16 (DP_BF16) for GEMM operands.
template <typename T> struct Weights {
  const float *w1s;   // [E1]            first embedding layer, s column
  const float *Bt;    // [NTYPES][NTYPES][E1]  type part + bias of the first layer
  const T *W2T;       // [E2][E1]
  const T *W2;        // [E1][E2]
  const float *b2;    // [E2]
  const T *W3T;       // [M][E2]
  const T *W3;        // [E2][M]
  const float *b3;    // [M]
  const T *WqkT[NATTN];  // [M][M]  (WQ WK^T / sqrt(d))^T
  const T *Wqk[NATTN];   // [M][M]
  const T *WvoT[NATTN];  // [M][M]  (WV WO)^T
  const T *Wvo[NATTN];   // [M][M]
  const float *gamma[NATTN];
  const float *beta[NATTN];
  const T *F1T;       // [FH][ND]
  const T *F1;        // [ND][FH]
  const T *F2T;       // [FH][FH]
  const T *F2;
  const T *F3T;
  const T *F3;
  const float *c1, *c2, *c3;
  const float *F4;    // [FH]
  float c4;
  const float *ebias; // [NTYPES]
};

// Extra device weights of the bfloat16 path: GEMM operands zero-padded to MFMA
// tile multiples and stored [output column][k] (k contiguous, 16-byte rows), so
// every MFMA fragment is one 16-byte load.  Feature width 100 is padded to 112,
// embedding widths 25/50 to 32/64, the fitting width 240 to 256 along k.  The
// fitting operands come as a two-term split w = hi + lo (both bf16).
struct WeightsB16 {
  const bf16_t *W2T;           // [64][32]    W2T[c][k] = W2[k][c]
  const bf16_t *W3T;           // [112][64]   W3T[m][k] = W3[k][m]
  const bf16_t *W3;            // [64][112]   W3[c][m]
  const bf16_t *W2;            // [32][64]    W2[e1][e2]
  const bf16_t *WqkT[NATTN];   // [112][112]  WqkT[c][k] = Wqk[k][c]
  const bf16_t *Wqk[NATTN];    // [112][112]
  const bf16_t *WvoT[NATTN];   // [112][112]
  const bf16_t *Wvo[NATTN];    // [112][112]
  const bf16_t *F1T[2];        // [240][1600] hi, lo
  const bf16_t *F1[2];         // [1600][256]
  const bf16_t *F2T[2];        // [240][256]
  const bf16_t *F2[2];         // [240][256]
  const bf16_t *F3T[2];        // [240][256]
  const bf16_t *F3[2];         // [240][256]
};

struct Workspace {
  int64_t cap = 0;            // atoms
  int *cell_of = nullptr;     // [cap]
  int *cell_count = nullptr;  // [MAX_CELLS + 1]
  int *cell_start = nullptr;  // [MAX_CELLS + 1]
  int *cell_cursor = nullptr; // [MAX_CELLS]
  int *cell_atoms = nullptr;  // [cap]
  int *nlist = nullptr;       // [cap][SEL]
  int *nnei = nullptr;        // [cap]
  int *rev = nullptr;         // [cap][SEL]
  float *Gsave = nullptr;     // [cap][NATTN][NPMAX][M]  inputs of each attention layer
  float *Tsave = nullptr;     // [cap][M][4]
  float *D = nullptr;         // [cap][ND]  descriptor, then dE/dD
  double *Ei = nullptr;       // [cap] atomic energies
  float4 *g = nullptr;        // [cap][SEL]  dE_i/dDelta_ij
  double *vpart = nullptr;    // [cap][9]   per-atom virial
  double *red = nullptr;      // scratch for the compensated reductions
  Grid *grid = nullptr;       // device copy of the grid (open boundaries)
  unsigned *flags = nullptr;  // [4] status words: flags, overflow count, rev misses, spare
  unsigned *flags_host = nullptr;  // pinned mirror
  double *gE = nullptr;       // [1] scale of the backward pass
};

}  // namespace dp

struct dp_model {
  int device = 0;
  int prec = 0;
  double rc = 0, rcs = 0, ln_eps = 1e-5;
  int sel = 0, ntypes = 0;
  void *wbuf = nullptr;
  dp::Weights<float> wf{};
  dp::Weights<dp::bf16_t> wb{};
  dp::WeightsB16 wp{};
  dp::Workspace ws;
  // state kept between dp_compute_device (energy only) and dp_backward_device
  int64_t fwd_natoms = 0;
  const double *fwd_coords = nullptr;
  const int32_t *fwd_types = nullptr;
  dp::Grid fwd_grid{};
  bool fwd_valid = false;
  // per-phase timing (dp_profile_enable)
  bool prof = false;
  hipEvent_t ev[8] = {};
  double prof_ms[8] = {};
  int64_t prof_calls[8] = {};
};

namespace dp {
void set_error(const std::string &s);

// Launchers (defined in the kernel translation units); all enqueue on `st`.
void launch_neighbors(const Workspace &ws, const double *coords, const int *types, int n, int ntypes,
                      const Grid &g, bool grid_on_device, double rc, hipStream_t st);
template <typename T>
void launch_descriptor_fwd(const Weights<T> &w, const Workspace &ws, const double *coords, const int *types,
                           int n, const Grid &g, bool grid_on_device, float rc, float rcs, float ln_eps,
                           hipStream_t st);
template <typename T>
void launch_fitting(const Weights<T> &w, const Workspace &ws, const int *types, int n, bool backward,
                    hipStream_t st);
void launch_descriptor_fwd_b16(const Weights<bf16_t> &w, const WeightsB16 &wp, const Workspace &ws,
                               const double *coords, const int *types, int n, const Grid &g, bool grid_on_device,
                               float rc, float rcs, float ln_eps, hipStream_t st);
void launch_descriptor_bwd_b16(const Weights<bf16_t> &w, const WeightsB16 &wp, const Workspace &ws,
                               const double *coords, const int *types, int n, const Grid &g, bool grid_on_device,
                               float rc, float rcs, float ln_eps, hipStream_t st);
void launch_fitting_b16(const Weights<bf16_t> &w, const WeightsB16 &wp, const Workspace &ws, const int *types, int n,
                        bool backward, hipStream_t st);
template <typename T>
void launch_descriptor_bwd(const Weights<T> &w, const Workspace &ws, const double *coords, const int *types,
                           int n, const Grid &g, bool grid_on_device, float rc, float rcs, float ln_eps,
                           hipStream_t st);
void launch_forces(const Workspace &ws, const double *coords, int n, const Grid &g, bool grid_on_device,
                   const double *gE, double *forces, double *virial_out, hipStream_t st);
void launch_energy(const Workspace &ws, int n, double *energy, double *atom_energy, hipStream_t st);
}  // namespace dp
