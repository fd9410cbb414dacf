// The repformer-style model (the paper's DPA2 family, Section II: single-atom and pair
// representations updated layer by layer with neighbour-to-neighbour message passing):
// sizes, device weights and buffers, launchers.
//
// Model (the functional form the library implements; the paper gives none):
//   g1_i = TN[t_i] (64);  g2_ij = tanh(s_ij Wp0 + bp0) (32);  R_ij = (s, s rhat);
//   three layers, each:
//     g2_ij <- g2_ij + tanh([g2_ij, g1_j] Wa + ba)
//     Q, K, V = g2 Wq, g2 Wk, g2 Wv;  P_jk = sw_k exp(Q_j.K_k / sqrt 32) / sum_k' (...);
//     g2_ij <- g2_ij + sum_k P_jk (rhat_j . rhat_k) V_k
//     T_i = sum_j g2_ij R_ij^T / sel (32 x 4);  D_i = T_i T_i[:4]^T;
//     c_i = sum_j sw_ij g2_ij * g1_j[:32] / sel;  g1_i <- g1_i + tanh([g1_i, D_i, c_i] W1 + b1)
//   E_i = y2 G3 + d3, y2 = tanh(y1 G2 + d2) + y1, y1 = tanh(g1_i G1 + d1).
#pragma once
#include "dp_internal.h"

namespace dp {
namespace rep {

constexpr int G1D = 64;                 // node width
constexpr int G2D = 32;                 // pair width (and attention width)
constexpr int NAX = 4;                  // axis columns of D
constexpr int NLAYER = 3;
constexpr int XD = G1D + G2D * NAX + G2D;  // node-update input width, 224
constexpr int FWID = 128;
constexpr int GSN = 8;                  // per-edge gradient slots: ds, dsw, drhat (3), pad

struct Weights {  // float32, row-major [in][out] as in the model file
  const float *TN;                      // [NTYPES][64]
  const float *Wp0, *bp0;               // [32]
  const float *Wa[NLAYER], *ba[NLAYER];  // [96][32], [32]
  const float *Wq[NLAYER], *Wk[NLAYER], *Wv[NLAYER];  // [32][32]
  const float *W1[NLAYER], *b1[NLAYER];  // [224][64], [64]
  const float *G1, *d1, *G2, *d2, *G3;   // fitting
  const double *G3d;
  double d3;
};

// Per-step device buffers (edge rows at the neighbour-list stride SEL).
struct Buffers {
  int64_t cap = 0;
  float *g1f = nullptr;  // [2][cap][64]       g1 after layers 1, 2
  float *g2f = nullptr;  // [3][cap][SEL][32]  g2 after layers 1, 2, 3
  float *dg2 = nullptr;  // [cap][SEL][32]     dE/dg2 of the current layer's output, in place
  float *dnj = nullptr;  // [2][cap][SEL][64]  edge (i, j)'s part of dE/dg1_j, by layer parity
  float *dnl = nullptr;  // [cap][64]          atom i's own part of dE/dg1_i
  float *gs = nullptr;   // [cap][SEL][GSN]    dE/ds, dE/dsw, dE/drhat per edge over the layers
  int *slot = nullptr;   // [cap][SEL]         position of i in the list of its j-th neighbour, or -1
  int64_t *etot = nullptr;  // [1] edges of the step
};

struct Geo {
  float rc, rcs, inv_sel;
};

// *b.etot = sum of the list lengths of the n atoms.
void launch_edge_count(const Buffers &b, const Workspace &ws, int n, hipStream_t st);
// Layer `layer` (0 .. 2) forward over all n atoms; the last layer also evaluates the
// fitting net (E_i into Ei) and its gradient dE/dg1 (into dnl).  Layer `layer` backward
// (called for 2, 1, 0); layer 0 writes g_ij = dE/dDelta_ij into ws.g.
void launch_layer_fwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, double *Ei, hipStream_t st);
void launch_layer_bwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, hipStream_t st);

}  // namespace rep
}  // namespace dp
