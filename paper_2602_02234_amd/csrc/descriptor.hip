// Per-atom descriptor kernels on gfx950: environment matrix, type-embedded
// embedding net, two gated self-attention layers over the atom's neighbours,
// and the descriptor contraction (forward), plus the hand-written backward
// that turns dE/dD into g_ij = dE_i/dDelta_ij.
//
// Model (paper, Section II: embedding net over an atom and its neighbours,
// self-attention layers updating that representation residually; sizes of the
// attention model studied here):
//   r = |Delta|, sw = quintic switch (1 below rcs, 0 from rc), s = sw / r,
//   rhat = Delta / r, Rt = (s, s rhat);
//   h1 = tanh(s w1s + B[t_i][t_j]) (type part of the first layer folded into B),
//   h2 = tanh(h1 W2 + b2) + [h1, h1], G = tanh(h2 W3 + b3) + [h2, h2];
//   per layer: S = G (WQ WK^T / sqrt d) G^T, P = sw-weighted row softmax of S,
//   A = P * (rhat_j . rhat_k), Y = A G (WV WO), G <- gamma LN(G + Y) + beta;
//   T = G^T Rt / sel, D = T T_<16^T.
// With one head and no projection biases, Q K^T = G (WQ WK^T) G^T and
// (A V) WO = (A G)(WV WO), so each layer needs the two 100x100 products only;
// they are formed once at model load.
//
// Layout: one workgroup (8 waves) per atom; tokens padded to NP = 16 ceil(n/16)
// (<= 128).  The atom's [NP][100] representation lives in LDS; each attention
// layer is processed in blocks of 16 query rows that all 8 waves share, so the
// NP x NP score matrix never exists as a whole.  All cross-wave sums go through
// per-wave partial arrays added in a fixed order: results do not depend on
// scheduling.
#include "dp_env.h"

namespace dp {
namespace {

// Embedding net for the 16 rows of block jb: writes h1 -> h1b, h2 -> h2b, G rows -> Gout.
template <typename T>
__device__ void embed_block(const Weights<T> &w, const Env &e, int ti, int jb, float *h1b, float *h2b,
                            float *Gout) {
  for (int q = threadIdx.x; q < 16 * E1; q += NTHREADS) {
    const int r = q / E1, c = q % E1, j = jb * 16 + r;
    h1b[r * LDM + c] = tanhf(e.s[j] * w.w1s[c] + w.Bt[(ti * NTYPES + e.tj[j]) * E1 + c]);
  }
  __syncthreads();
  const int wv = wave_id();
  if (wv < 4) {  // 16 x 50 -> four 16-column tiles
    const int c0 = wv * 16;
    f4 acc = {0, 0, 0, 0};
    Mma<T>::tile(acc, [&](int r, int k) { return h1b[r * LDM + k]; },
                 [&](int c, int k) { return (c0 + c < E2) ? ldw(w.W2T, (c0 + c) * E1 + k) : 0.f; }, E1);
    const int col = c0 + acc_col();
    if (col < E2)
      for (int i = 0; i < 4; ++i) {
        const int r = acc_row(i);
        h2b[r * LDM + col] = tanhf(acc[i] + w.b2[col]) + h1b[r * LDM + (col % E1)];
      }
  }
  __syncthreads();
  if (wv < 7) {  // 16 x 100 -> seven tiles
    const int c0 = wv * 16;
    f4 acc = {0, 0, 0, 0};
    Mma<T>::tile(acc, [&](int r, int k) { return h2b[r * LDM + k]; },
                 [&](int c, int k) { return (c0 + c < M) ? ldw(w.W3T, (c0 + c) * E2 + k) : 0.f; }, E2);
    const int col = c0 + acc_col();
    if (col < M)
      for (int i = 0; i < 4; ++i) {
        const int r = acc_row(i);
        Gout[(jb * 16 + r) * LDM + col] = tanhf(acc[i] + w.b3[col]) + h2b[r * LDM + (col % E2)];
      }
  }
  __syncthreads();
}

// Shared part of a layer for one 16-row block: U block, scores, weights E = exp(S - m)/Z
// (into Eb, may be null), attention block A (into Ab) and H = A G (into Hb).
template <typename T>
__device__ void attn_block_front(const Weights<T> &w, int layer, const Env &e, const float *Gin, int jb, int n,
                                 int NP, float *Ub, float *Eb, float *Ab, float *Hb, float *red) {
  const int wv = wave_id();
  const int nb = NP / 16;
  // (a) U block = G_blk Wqk
  if (wv < 7) {
    const int c0 = wv * 16;
    f4 acc = {0, 0, 0, 0};
    const T *WqkT = w.WqkT[layer];
    Mma<T>::tile(acc, [&](int r, int k) { return Gin[(jb * 16 + r) * LDM + k]; },
                 [&](int c, int k) { return (c0 + c < M) ? ldw(WqkT, (c0 + c) * M + k) : 0.f; }, M);
    const int col = c0 + acc_col();
    if (col < M)
      for (int i = 0; i < 4; ++i) Ub[acc_row(i) * LDM + col] = acc[i];
  }
  __syncthreads();
  // (b) scores S = U G^T for this block; wave wv owns column tile wv
  f4 sacc = {0, 0, 0, 0};
  const int k = wv * 16 + acc_col();
  const bool has = wv < nb;
  if (has)
    Mma<T>::tile(sacc, [&](int r, int kk) { return Ub[r * LDM + kk]; },
                 [&](int c, int kk) { return Gin[(wv * 16 + c) * LDM + kk]; }, M);
  const bool kval = has && k < n;
  for (int i = 0; i < 4; ++i) {
    const float m = max16(kval ? sacc[i] : -INFINITY);
    if ((lane_id() & 15) == 0) red[(wv * 16 + acc_row(i)) * 8 + 0] = m;
  }
  __syncthreads();
  float ex[4], esum[4];
  for (int i = 0; i < 4; ++i) {
    const int r = acc_row(i);
    float m = -INFINITY;
    for (int q = 0; q < NW; ++q) m = fmaxf(m, red[(q * 16 + r) * 8 + 0]);
    if (m == -INFINITY) m = 0.f;
    ex[i] = kval ? expf(sacc[i] - m) : 0.f;
    esum[i] = sum16(kval ? e.sw[k] * ex[i] : 0.f);
    if ((lane_id() & 15) == 0) red[(wv * 16 + r) * 8 + 1] = esum[i];
  }
  __syncthreads();
  if (has)
    for (int i = 0; i < 4; ++i) {
      const int r = acc_row(i), j = jb * 16 + r;
      float Z = 0.f;
      for (int q = 0; q < NW; ++q) Z += red[(q * 16 + r) * 8 + 1];
      const float E = Z > 0.f ? ex[i] / Z : 0.f;
      if (Eb) Eb[r * LDN + k] = E;
      const float gate = e.rh[3 * j] * e.rh[3 * k] + e.rh[3 * j + 1] * e.rh[3 * k + 1] + e.rh[3 * j + 2] * e.rh[3 * k + 2];
      Ab[r * LDN + k] = e.sw[k] * E * gate;
    }
  __syncthreads();
  // (c) H = A G
  if (wv < 7) {
    const int c0 = wv * 16;
    f4 acc = {0, 0, 0, 0};
    Mma<T>::tile(acc, [&](int r, int kk) { return Ab[r * LDN + kk]; },
                 [&](int c, int kk) { return (c0 + c < M) ? Gin[kk * LDM + c0 + c] : 0.f; }, NP);
    const int col = c0 + acc_col();
    if (col < M)
      for (int i = 0; i < 4; ++i) Hb[acc_row(i) * LDM + col] = acc[i];
  }
  __syncthreads();
}

// Y = H Wvo for the block held by wave wv (< 7), then the residual X = G_in + Y and its
// per-row LayerNorm statistics.  Returns xh (normalised X) and isig per accumulator row.
template <typename T>
__device__ void attn_block_ln(const Weights<T> &w, int layer, const float *Hb, const float *Gin, int jb, float *red,
                              float ln_eps, f4 &yh, float isig[4]) {
  const int wv = wave_id();
  const int col = wv * 16 + acc_col();
  const bool cval = wv < 7 && col < M;
  f4 y = {0, 0, 0, 0};
  if (wv < 7) {
    const int c0 = wv * 16;
    const T *WvoT = w.WvoT[layer];
    Mma<T>::tile(y, [&](int r, int k) { return Hb[r * LDM + k]; },
                 [&](int c, int k) { return (c0 + c < M) ? ldw(WvoT, (c0 + c) * M + k) : 0.f; }, M);
  }
  if (cval)
    for (int i = 0; i < 4; ++i) y[i] += Gin[(jb * 16 + acc_row(i)) * LDM + col];
  for (int i = 0; i < 4; ++i) {
    const float p = sum16(cval ? y[i] : 0.f);
    if ((lane_id() & 15) == 0) red[(wv * 16 + acc_row(i)) * 8 + 2] = p;
  }
  __syncthreads();
  float mu[4];
  for (int i = 0; i < 4; ++i) {
    const int r = acc_row(i);
    float sacc = 0.f;
    for (int q = 0; q < NW; ++q) sacc += red[(q * 16 + r) * 8 + 2];
    mu[i] = sacc / (float)M;
    const float dv = cval ? y[i] - mu[i] : 0.f;
    const float p = sum16(dv * dv);
    if ((lane_id() & 15) == 0) red[(wv * 16 + r) * 8 + 3] = p;
  }
  __syncthreads();
  for (int i = 0; i < 4; ++i) {
    const int r = acc_row(i);
    float v = 0.f;
    for (int q = 0; q < NW; ++q) v += red[(q * 16 + r) * 8 + 3];
    isig[i] = 1.f / sqrtf(v / (float)M + ln_eps);
    yh[i] = (y[i] - mu[i]) * isig[i];
  }
}

// ======================================================================== forward
struct SmemFwd {
  float G[2][NPMAX * LDM];
  float Ub[16 * LDM];
  float Ab[16 * LDN];
  float Hb[16 * LDM];
  float red[NW * 16 * 8];
  float T[M * 4];
  Env e;
};

template <typename T>
__global__ void __launch_bounds__(NTHREADS)
k_desc_fwd(Weights<T> w, const double *__restrict__ X, const int *__restrict__ types, int natoms, int c0,
           const int *__restrict__ nlist, const int *__restrict__ nnei, const Grid *__restrict__ grids, const int *__restrict__ sys_of,
           float rc, float rcs, float ln_eps, float *__restrict__ Gsave, float *__restrict__ Tsave,
           float *__restrict__ D) {
  __shared__ SmemFwd sm;
  const int i = c0 + blockIdx.x;
  const Grid g = grids[sys_of[i]];
  const int n = min(max(nnei[i], 0), SEL);
  const int NP = n > 0 ? ((n + 15) / 16) * 16 : 16;
  const int nb = NP / 16;
  const int ti = clamp_type(types[i]);
  build_env(sm.e, X, types, nlist, i, n, natoms, g, rc, rcs);
  __syncthreads();
  for (int jb = 0; jb < nb; ++jb) embed_block(w, sm.e, ti, jb, sm.Ub, sm.Hb, sm.G[0]);
  for (int layer = 0; layer < NATTN; ++layer) {
    float *Gin = sm.G[layer & 1];
    float *Gout = sm.G[(layer + 1) & 1];
    float *gs = Gsave + ((size_t)i * NATTN + layer) * GSAVE_LAYER;
    for (int q = threadIdx.x; q < NP * M; q += NTHREADS) gs[q] = Gin[(q / M) * LDM + q % M];
    for (int jb = 0; jb < nb; ++jb) {
      attn_block_front(w, layer, sm.e, Gin, jb, n, NP, sm.Ub, nullptr, sm.Ab, sm.Hb, sm.red);
      f4 yh;
      float isig[4];
      attn_block_ln(w, layer, sm.Hb, Gin, jb, sm.red, ln_eps, yh, isig);
      const int wv = wave_id();
      const int col = wv * 16 + acc_col();
      if (wv < 7 && col < M)
        for (int ii = 0; ii < 4; ++ii) {
          const int j = jb * 16 + acc_row(ii);
          Gout[j * LDM + col] = w.gamma[layer][col] * yh[ii] + w.beta[layer][col];
        }
      __syncthreads();
    }
  }
  const float *Gf = sm.G[NATTN & 1];
  for (int q = threadIdx.x; q < M * 4; q += NTHREADS) {
    const int m = q >> 2, c = q & 3;
    float acc = 0.f;
    for (int j = 0; j < n; ++j) acc += Gf[j * LDM + m] * sm.e.Rt[4 * j + c];
    acc *= 1.f / (float)SEL;
    sm.T[q] = acc;
    Tsave[(size_t)i * M * 4 + q] = acc;
  }
  __syncthreads();
  for (int q = threadIdx.x; q < ND; q += NTHREADS) {
    const int m = q / M2, a = q % M2;
    const float *tm = sm.T + 4 * m, *ta = sm.T + 4 * a;
    D[(size_t)i * ND + q] = tm[0] * ta[0] + tm[1] * ta[1] + tm[2] * ta[2] + tm[3] * ta[3];
  }
}

// ======================================================================== backward
struct SmemBwd {
  float Gin[NPMAX * LDM];
  float dG[NPMAX * LDM];
  float Ub[16 * LDM];
  float Eb[16 * LDN];
  float Ab[16 * LDN];
  float Hb[16 * LDM];
  float dHb[16 * LDM];
  float red[NW * 16 * 8];
  float T[M * 4];
  float dT[M * 4];
  float dswa[NPMAX];
  float drh[NPMAX * 3];
  float dRt[NPMAX * 4];
  Env e;
};

template <typename T>
__global__ void __launch_bounds__(NTHREADS)
k_desc_bwd(Weights<T> w, const double *__restrict__ X, const int *__restrict__ types, int natoms, int c0,
           const int *__restrict__ nlist, const int *__restrict__ nnei, const Grid *__restrict__ grids, const int *__restrict__ sys_of,
           float rc, float rcs, float ln_eps, const float *__restrict__ Gsave, const float *__restrict__ Tsave,
           const float *__restrict__ dD, float4 *__restrict__ gout) {
  __shared__ SmemBwd sm;
  const int i = c0 + blockIdx.x;
  const Grid g = grids[sys_of[i]];
  const int n = min(max(nnei[i], 0), SEL);
  const int NP = n > 0 ? ((n + 15) / 16) * 16 : 16;
  const int nb = NP / 16;
  const int ti = clamp_type(types[i]);
  const int wv = wave_id();
  build_env(sm.e, X, types, nlist, i, n, natoms, g, rc, rcs);
  for (int q = threadIdx.x; q < NPMAX; q += NTHREADS) {
    sm.dswa[q] = 0.f;
    for (int a = 0; a < 3; ++a) sm.drh[3 * q + a] = 0.f;
    for (int a = 0; a < 4; ++a) sm.dRt[4 * q + a] = 0.f;
  }
  for (int q = threadIdx.x; q < M * 4; q += NTHREADS) sm.T[q] = Tsave[(size_t)i * M * 4 + q];
  __syncthreads();
  // dT from dD:  D_ma = T_m . T_a  =>  dT_m += sum_a dD_ma T_a ;  dT_a += sum_m dD_ma T_m (a < 16)
  const float *dDi = dD + (size_t)i * ND;
  for (int q = threadIdx.x; q < M * 4; q += NTHREADS) {
    const int m = q >> 2, c = q & 3;
    float acc = 0.f;
    for (int a = 0; a < M2; ++a) acc += dDi[m * M2 + a] * sm.T[4 * a + c];
    if (m < M2)
      for (int mm = 0; mm < M; ++mm) acc += dDi[mm * M2 + m] * sm.T[4 * mm + c];
    sm.dT[q] = acc;
  }
  __syncthreads();
  const float inv_sel = 1.f / (float)SEL;

  for (int layer = NATTN - 1; layer >= 0; --layer) {
    const float *gs = Gsave + ((size_t)i * NATTN + layer) * GSAVE_LAYER;
    for (int q = threadIdx.x; q < NP * M; q += NTHREADS) sm.Gin[(q / M) * LDM + q % M] = gs[q];
    __syncthreads();
    f4 colacc[7];
    for (int t = 0; t < 7; ++t) colacc[t] = f4{0, 0, 0, 0};
    const bool top = layer == NATTN - 1;
    for (int jb = 0; jb < nb; ++jb) {
      attn_block_front(w, layer, sm.e, sm.Gin, jb, n, NP, sm.Ub, sm.Eb, sm.Ab, sm.Hb, sm.red);
      f4 yh;
      float isig[4];
      attn_block_ln(w, layer, sm.Hb, sm.Gin, jb, sm.red, ln_eps, yh, isig);
      // (d) LayerNorm backward; for the top layer the incoming gradient is
      // dG = Rt dT^T / sel and the layer output also feeds dRt = G_out dT / sel.
      // The residual runs through the LayerNorm: dG_in starts as dX and dY = dX.
      const int col = wv * 16 + acc_col();
      const bool cval = wv < 7 && col < M;
      float dyh[4];
      float prt[4][4];
      for (int ii = 0; ii < 4; ++ii) {
        const int r = acc_row(ii), j = jb * 16 + r;
        float go = 0.f;
        if (cval) {
          if (top) {
            go = (sm.e.Rt[4 * j] * sm.dT[4 * col] + sm.e.Rt[4 * j + 1] * sm.dT[4 * col + 1] +
                  sm.e.Rt[4 * j + 2] * sm.dT[4 * col + 2] + sm.e.Rt[4 * j + 3] * sm.dT[4 * col + 3]) * inv_sel;
            const float gout_v = w.gamma[layer][col] * yh[ii] + w.beta[layer][col];
            for (int c = 0; c < 4; ++c) prt[ii][c] = gout_v * sm.dT[4 * col + c] * inv_sel;
          } else {
            go = sm.dG[j * LDM + col];
            for (int c = 0; c < 4; ++c) prt[ii][c] = 0.f;
          }
        } else {
          for (int c = 0; c < 4; ++c) prt[ii][c] = 0.f;
        }
        dyh[ii] = cval ? go * w.gamma[layer][col] : 0.f;
        const float p0 = sum16(dyh[ii]);
        const float p1 = sum16(dyh[ii] * (cval ? yh[ii] : 0.f));
        if ((lane_id() & 15) == 0) {
          sm.red[(wv * 16 + r) * 8 + 4] = p0;
          sm.red[(wv * 16 + r) * 8 + 5] = p1;
        }
        if (top)
          for (int c = 0; c < 4; ++c) prt[ii][c] = sum16(prt[ii][c]);
      }
      __syncthreads();
      for (int ii = 0; ii < 4; ++ii) {
        const int r = acc_row(ii);
        float s0 = 0.f, s1 = 0.f;
        for (int q = 0; q < NW; ++q) {
          s0 += sm.red[(q * 16 + r) * 8 + 4];
          s1 += sm.red[(q * 16 + r) * 8 + 5];
        }
        const float dX = (dyh[ii] - s0 / (float)M - (cval ? yh[ii] : 0.f) * (s1 / (float)M)) * isig[ii];
        if (cval) {
          sm.Hb[r * LDM + col] = dX;
          sm.dG[(jb * 16 + r) * LDM + col] = dX;
        }
      }
      // dRt row sums for the top layer: 4 values per row, reduced in two rounds of 2
      if (top) {
        for (int half = 0; half < 2; ++half) {
          __syncthreads();
          for (int ii = 0; ii < 4; ++ii)
            if ((lane_id() & 15) == 0) {
              const int r = acc_row(ii);
              sm.red[(wv * 16 + r) * 8 + 6] = prt[ii][2 * half];
              sm.red[(wv * 16 + r) * 8 + 7] = prt[ii][2 * half + 1];
            }
          __syncthreads();
          if ((int)threadIdx.x < 16) {
            const int r = threadIdx.x, j = jb * 16 + r;
            float a0 = 0.f, a1 = 0.f;
            for (int q = 0; q < NW; ++q) {
              a0 += sm.red[(q * 16 + r) * 8 + 6];
              a1 += sm.red[(q * 16 + r) * 8 + 7];
            }
            sm.dRt[4 * j + 2 * half] += a0;
            sm.dRt[4 * j + 2 * half + 1] += a1;
          }
        }
      }
      __syncthreads();
      // (e) dH = dY Wvo^T
      if (wv < 7) {
        const int c0 = wv * 16;
        f4 acc = {0, 0, 0, 0};
        const T *Wvo = w.Wvo[layer];
        Mma<T>::tile(acc, [&](int r, int k) { return sm.Hb[r * LDM + k]; },
                     [&](int c, int k) { return (c0 + c < M) ? ldw(Wvo, (c0 + c) * M + k) : 0.f; }, M);
        const int cc = c0 + acc_col();
        if (cc < M)
          for (int ii = 0; ii < 4; ++ii) sm.dHb[acc_row(ii) * LDM + cc] = acc[ii];
      }
      __syncthreads();
      // (f) dA = dH G^T, then gate, weighted-softmax backward; wave wv owns column tile wv
      {
        const bool has = wv < nb;
        const int k = wv * 16 + acc_col();
        f4 dA = {0, 0, 0, 0};
        if (has)
          Mma<T>::tile(dA, [&](int r, int kk) { return sm.dHb[r * LDM + kk]; },
                       [&](int c, int kk) { return sm.Gin[(wv * 16 + c) * LDM + kk]; }, M);
        const bool kval = has && k < n;
        float dP[4], P[4], dC[4];
        for (int ii = 0; ii < 4; ++ii) {
          const int r = acc_row(ii), j = jb * 16 + r;
          const bool v = kval && j < n;
          const float E = v ? sm.Eb[r * LDN + k] : 0.f;
          const float gate = sm.e.rh[3 * j] * sm.e.rh[3 * k] + sm.e.rh[3 * j + 1] * sm.e.rh[3 * k + 1] +
                             sm.e.rh[3 * j + 2] * sm.e.rh[3 * k + 2];
          P[ii] = v ? sm.e.sw[k] * E : 0.f;
          dP[ii] = v ? dA[ii] * gate : 0.f;
          dC[ii] = v ? dA[ii] * P[ii] : 0.f;
          const float rp = sum16(P[ii] * dP[ii]);
          const float hx = sum16(dC[ii] * sm.e.rh[3 * k]);
          const float hy = sum16(dC[ii] * sm.e.rh[3 * k + 1]);
          const float hz = sum16(dC[ii] * sm.e.rh[3 * k + 2]);
          if ((lane_id() & 15) == 0) {
            sm.red[(wv * 16 + r) * 8 + 0] = rp;
            sm.red[(wv * 16 + r) * 8 + 1] = hx;
            sm.red[(wv * 16 + r) * 8 + 2] = hy;
            sm.red[(wv * 16 + r) * 8 + 3] = hz;
          }
        }
        __syncthreads();
        float wsum = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
        for (int ii = 0; ii < 4; ++ii) {
          const int r = acc_row(ii), j = jb * 16 + r;
          float rho = 0.f;
          for (int q = 0; q < NW; ++q) rho += sm.red[(q * 16 + r) * 8 + 0];
          const bool v = kval && j < n;
          const float E = v ? sm.Eb[r * LDN + k] : 0.f;
          const float W = v ? E * (dP[ii] - rho) : 0.f;
          if (has) sm.Eb[r * LDN + k] = v ? sm.e.sw[k] * W : 0.f;  // dS (the 1/sqrt(d) lives in Wqk)
          wsum += W;
          cx += dC[ii] * sm.e.rh[3 * j];
          cy += dC[ii] * sm.e.rh[3 * j + 1];
          cz += dC[ii] * sm.e.rh[3 * j + 2];
        }
        wsum = sum_cols4(wsum);
        cx = sum_cols4(cx);
        cy = sum_cols4(cy);
        cz = sum_cols4(cz);
        if (has && lane_id() < 16) {
          sm.dswa[k] += wsum;
          sm.drh[3 * k] += cx;
          sm.drh[3 * k + 1] += cy;
          sm.drh[3 * k + 2] += cz;
        }
        __syncthreads();
        if ((int)threadIdx.x < 16) {
          const int r = threadIdx.x, j = jb * 16 + r;
          float hx = 0.f, hy = 0.f, hz = 0.f;
          for (int q = 0; q < NW; ++q) {
            hx += sm.red[(q * 16 + r) * 8 + 1];
            hy += sm.red[(q * 16 + r) * 8 + 2];
            hz += sm.red[(q * 16 + r) * 8 + 3];
          }
          sm.drh[3 * j] += hx;
          sm.drh[3 * j + 1] += hy;
          sm.drh[3 * j + 2] += hz;
        }
      }
      __syncthreads();
      // (g) dU = dS G
      if (wv < 7) {
        const int c0 = wv * 16;
        f4 acc = {0, 0, 0, 0};
        Mma<T>::tile(acc, [&](int r, int kk) { return sm.Eb[r * LDN + kk]; },
                     [&](int c, int kk) { return (c0 + c < M) ? sm.Gin[kk * LDM + c0 + c] : 0.f; }, NP);
        const int cc = c0 + acc_col();
        if (cc < M)
          for (int ii = 0; ii < 4; ++ii) sm.Hb[acc_row(ii) * LDM + cc] = acc[ii];
      }
      __syncthreads();
      // (h) rows of this block: dG += dU Wqk^T ; (i) columns owned by this wave:
      // dG[k] += sum_j A_jk dH_j + dS_jk U_j, accumulated in registers until the layer ends
      if (wv < 7) {
        const int c0 = wv * 16;
        f4 acc = {0, 0, 0, 0};
        const T *Wqk = w.Wqk[layer];
        Mma<T>::tile(acc, [&](int r, int kk) { return sm.Hb[r * LDM + kk]; },
                     [&](int c, int kk) { return (c0 + c < M) ? ldw(Wqk, (c0 + c) * M + kk) : 0.f; }, M);
        const int cc = c0 + acc_col();
        if (cc < M)
          for (int ii = 0; ii < 4; ++ii) sm.dG[(jb * 16 + acc_row(ii)) * LDM + cc] += acc[ii];
      }
      if (wv < nb) {
        const int k0 = wv * 16;
        for (int t = 0; t < 7; ++t) {
          const int m0 = t * 16;
          Mma<T>::tile(colacc[t], [&](int rr, int kk) { return sm.Ab[kk * LDN + k0 + rr]; },
                       [&](int c, int kk) { return (m0 + c < M) ? sm.dHb[kk * LDM + m0 + c] : 0.f; }, 16);
          Mma<T>::tile(colacc[t], [&](int rr, int kk) { return sm.Eb[kk * LDN + k0 + rr]; },
                       [&](int c, int kk) { return (m0 + c < M) ? sm.Ub[kk * LDM + m0 + c] : 0.f; }, 16);
        }
      }
      __syncthreads();
    }
    if (wv < nb) {
      for (int t = 0; t < 7; ++t) {
        const int cc = t * 16 + acc_col();
        if (cc < M)
          for (int ii = 0; ii < 4; ++ii) sm.dG[(wv * 16 + acc_row(ii)) * LDM + cc] += colacc[t][ii];
      }
    }
    __syncthreads();
  }

  // ---- embedding and environment backward, per block of 16 rows
  float *h1b = sm.Ub;   // h1            [16][E1]
  float *t2b = sm.Ab;   // tanh of layer 2, then dpre2
  float *h2b = sm.Hb;   // h2
  float *p3b = sm.dHb;  // dpre3
  float *rsb = sm.Eb;   // dG halves sum, then dh2
  for (int jb = 0; jb < nb; ++jb) {
    for (int q = threadIdx.x; q < 16 * E1; q += NTHREADS) {
      const int r = q / E1, c = q % E1, j = jb * 16 + r;
      h1b[r * LDM + c] = tanhf(sm.e.s[j] * w.w1s[c] + w.Bt[(ti * NTYPES + sm.e.tj[j]) * E1 + c]);
    }
    __syncthreads();
    if (wv < 4) {
      const int c0 = wv * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return h1b[r * LDM + k]; },
                   [&](int c, int k) { return (c0 + c < E2) ? ldw(w.W2T, (c0 + c) * E1 + k) : 0.f; }, E1);
      const int col = c0 + acc_col();
      if (col < E2)
        for (int ii = 0; ii < 4; ++ii) {
          const int r = acc_row(ii), j = jb * 16 + r;
          const float t2 = tanhf(acc[ii] + w.b2[col]);
          t2b[r * LDN + col] = t2;
          h2b[r * LDM + col] = t2 + h1b[r * LDM + (col % E1)];
          rsb[r * LDN + col] = sm.dG[j * LDM + col] + sm.dG[j * LDM + col + E2];
        }
    }
    __syncthreads();
    if (wv < 7) {
      const int c0 = wv * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return h2b[r * LDM + k]; },
                   [&](int c, int k) { return (c0 + c < M) ? ldw(w.W3T, (c0 + c) * E2 + k) : 0.f; }, E2);
      const int col = c0 + acc_col();
      if (col < M)
        for (int ii = 0; ii < 4; ++ii) {
          const int r = acc_row(ii), j = jb * 16 + r;
          const float t3 = tanhf(acc[ii] + w.b3[col]);
          p3b[r * LDM + col] = sm.dG[j * LDM + col] * (1.f - t3 * t3);
        }
    }
    __syncthreads();
    // dh2 = dpre3 W3^T + (dG[:, :50] + dG[:, 50:]);  dpre2 = dh2 (1 - t2^2)
    if (wv < 4) {
      const int c0 = wv * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return p3b[r * LDM + k]; },
                   [&](int c, int k) { return (c0 + c < E2) ? ldw(w.W3, (c0 + c) * M + k) : 0.f; }, M);
      const int col = c0 + acc_col();
      if (col < E2)
        for (int ii = 0; ii < 4; ++ii) {
          const int r = acc_row(ii);
          const float dh2 = acc[ii] + rsb[r * LDN + col];
          rsb[r * LDN + col] = dh2;
          const float t2 = t2b[r * LDN + col];
          t2b[r * LDN + col] = dh2 * (1.f - t2 * t2);
        }
    }
    __syncthreads();
    // dh1 = dpre2 W2^T + (dh2[:, :25] + dh2[:, 25:]);  ds_emb = sum_c dh1 (1 - h1^2) w1s
    if (wv < 2) {
      const int c0 = wv * 16;
      f4 acc = {0, 0, 0, 0};
      Mma<T>::tile(acc, [&](int r, int k) { return t2b[r * LDN + k]; },
                   [&](int c, int k) { return (c0 + c < E1) ? ldw(w.W2, (c0 + c) * E2 + k) : 0.f; }, E2);
      const int col = c0 + acc_col();
      for (int ii = 0; ii < 4; ++ii) {
        const int r = acc_row(ii);
        float v = 0.f;
        if (col < E1) {
          const float dh1 = acc[ii] + rsb[r * LDN + col] + rsb[r * LDN + col + E1];
          const float h1 = h1b[r * LDM + col];
          v = dh1 * (1.f - h1 * h1) * w.w1s[col];
        }
        const float p = sum16(v);
        if ((lane_id() & 15) == 0) sm.red[(wv * 16 + r) * 8 + 0] = p;
      }
    }
    __syncthreads();
    if ((int)threadIdx.x < 16) {
      const int r = threadIdx.x, j = jb * 16 + r;
      float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
      if (j < n) {
        const float ds_emb = sm.red[(0 * 16 + r) * 8] + sm.red[(1 * 16 + r) * 8];
        out = pair_gradient(sm.e, j, ds_emb, sm.dRt + 4 * j, sm.drh + 3 * j, sm.dswa[j]);
      }
      if (j < SEL) gout[(size_t)i * SEL + j] = out;
    }
    __syncthreads();
  }
  for (int j = NP + threadIdx.x; j < SEL; j += NTHREADS) gout[(size_t)i * SEL + j] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

template <typename T>
void launch_descriptor_fwd(const Weights<T> &w, const Workspace &ws, const double *coords, const int *types, int n,
                           int c0, int c1, float rc, float rcs, float ln_eps, hipStream_t st) {
  hipLaunchKernelGGL(k_desc_fwd<T>, dim3(c1 - c0), dim3(NTHREADS), 0, st, w, coords, types, n, c0, ws.nlist, ws.nnei, ws.grids,
                     ws.sys_of, rc, rcs, ln_eps, ws.Gsave, ws.Tsave, ws.D);
}

template <typename T>
void launch_descriptor_bwd(const Weights<T> &w, const Workspace &ws, const double *coords, const int *types, int n,
                           int c0, int c1, float rc, float rcs, float ln_eps, hipStream_t st) {
  hipLaunchKernelGGL(k_desc_bwd<T>, dim3(c1 - c0), dim3(NTHREADS), 0, st, w, coords, types, n, c0, ws.nlist, ws.nnei, ws.grids,
                     ws.sys_of, rc, rcs, ln_eps, ws.Gsave, ws.Tsave, ws.D, ws.g);
}

template void launch_descriptor_fwd<float>(const Weights<float> &, const Workspace &, const double *, const int *,
                                           int, int, int, float, float, float, hipStream_t);
template void launch_descriptor_bwd<float>(const Weights<float> &, const Workspace &, const double *, const int *,
                                           int, int, int, float, float, float, hipStream_t);

}  // namespace dp
