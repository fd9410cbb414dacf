// The GNN-variant descriptor (the paper's second model family, Section II: message
// passing over bonds and angles in place of attention): sizes, device weights and
// buffers, launchers.
//
// Model (the functional form the library implements; the paper gives none):
//   edges (i, j), j in N(i) (r_ij < rc); angles at i: ordered pairs (p, q), p != q, of
//   the first asel neighbours of i (list order) with r < rca;
//   n_i = TN[t_i];  e_ij = tanh(s_ij We0 + be0), s = sw_e(r) / r;
//   a_ipq = tanh(c_ipq Wa0 + ba0), c = rhat_ip . rhat_iq;
//   three layers, each: a <- a + tanh([a, e_ip[:32], e_iq[:32]] Waa + baa);
//     m_ip = sum_q sw_a(r_ip) sw_a(r_iq) / asel tanh([a, e_iq[:32]] Wea + bea);
//     e_ij <- e_ij + tanh([n_i, n_j, e_ij] Wee + bee) + m_ij;
//     n_i <- n_i + tanh([n_i, sum_j sw_e(r_ij) e_ij / sel] Wnn + bnn);
//   E_i = y2 G3 + d3, y2 = tanh(y1 G2 + d2) + y1, y1 = tanh(n_i G1 + d1).
#pragma once
#include "dp_internal.h"

namespace dp {
namespace gnn {

constexpr int NDIM = 64;   // node width
constexpr int EDIM = 64;   // edge width
constexpr int ADIM = 32;   // angle width (and the edge columns angles read)
constexpr int NLAYER = 3;
constexpr int FWID = 128;  // fitting width
constexpr int ASEL = 48;   // largest angle-neighbour count a model may set

// Device weights, float32, row-major [in][out] as in the model file.
struct Weights {
  const float *TN;                // [NTYPES][64]
  const float *We0, *be0;         // [64]
  const float *Wa0, *ba0;         // [32]
  const float *Waa[NLAYER], *baa[NLAYER];  // [96][32], [32]
  const float *Wea[NLAYER], *bea[NLAYER];  // [64][64], [64]
  const float *Wee[NLAYER], *bee[NLAYER];  // [192][64], [64]
  const float *Wnn[NLAYER], *bnn[NLAYER];  // [128][64], [64]
  const float *G1, *d1, *G2, *d2, *G3;     // [64][128], [128], [128][128], [128], [128]
  const double *G3d;              // [128]  last layer in float64 (energy sum)
  double d3;
};

// Per-step device buffers.  Edge rows use the neighbour-list stride SEL; angles of atom
// i start at aoff[i] (p-major: angle (p, q) at aoff[i] + p (nc_i - 1) + q - (q > p)).
struct Buffers {
  int64_t cap = 0, acap = 0;  // atoms, angles
  int64_t *aoff = nullptr;    // [cap + 3]: angle offsets, then the step's edge and angle-list edge counts
  float *nf = nullptr;        // [2][cap][64]       n after layers 1, 2
  float *ef = nullptr;        // [3][cap][SEL][64]  e after layers 1, 2, 3
  float *af = nullptr;        // [3][acap][32]      a after layers 1, 2, 3
  float *da = nullptr;        // [acap][32]         dE/da, updated in place layer by layer
  float *de = nullptr;        // [cap][SEL][64]     dE/de, likewise
  float *dnj = nullptr;       // [2][cap][SEL][64]  edge (i, j)'s part of dE/dn_j, by layer parity
  float *dnl = nullptr;       // [cap][64]          atom i's own part of dE/dn_i
  float *gs = nullptr;        // [cap][SEL][2]      dE/dsw_e, dE/dsw_a per edge over the layers
  int *slot = nullptr;        // [cap][SEL]         position of i in the list of its j-th neighbour, or -1
};

struct Geo {
  float rc, rcs, rca, inv_sel, inv_asel;
  int asel;
};

// aoff[1 .. n]: angle counts of every atom, then their inclusive prefix (aoff[0] = 0);
// aoff[cap + 1]: the number of edges (sum of the list lengths); aoff[cap + 2]: the
// number of angle-list edges of the atoms with angles.
void launch_angle_offsets(const Buffers &b, const Workspace &ws, const double *coords, int n, const Geo &geo,
                          hipStream_t st);
// Layer `layer` (0 .. 2) forward over all n atoms; the last layer also evaluates the
// fitting net (E_i into Ei) and its gradient dE/dn (into dnl).
template <typename T>
void launch_layer_fwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, double *Ei, hipStream_t st);
// Layer `layer` backward (called for 2, 1, 0); layer 0 writes g_ij = dE/dDelta_ij into ws.g.
template <typename T>
void launch_layer_bwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, hipStream_t st);

}  // namespace gnn
}  // namespace dp
