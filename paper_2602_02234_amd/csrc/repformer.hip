// Repformer-style model kernels for gfx950: one workgroup (eight waves) per centre atom
// and one launch per layer, forward and backward (a layer's pair update and convolution
// read the neighbours' g1 of the layer before, so layers meet at launch boundaries).
// The products run on MFMA (16x16x4 f32): the pair update and projections and the
// backward's dE/d[g2, g1_j] over tiles of 16 edges, one tile per wave; the
// neighbour-to-neighbour attention (every ordered pair of an atom's up to 120
// neighbours, width 32) over tiles of 16 queries in the forward and the backward's row
// pass (statistics, dQ, the row terms of the gate), and tiles of 16 keys in the column
// pass (dK, dV, the key terms of the switch and gate, with the scores recomputed).
// The contraction T = sum_j g2_j R_j^T and its gradient also run on MFMA; the node
// update (input 224) and the convolution sums stay float32 VALU work.  Every sum has
// one owner and a fixed order: results are deterministic.
#include <cmath>

#include "dp_env.h"
#include "repformer.h"

namespace dp {
namespace rep {
namespace {

constexpr int NWG = 8;
constexpr int NT = NWG * 64;
constexpr int LQ = G2D + 1;   // row stride of [edge][32] LDS arrays (odd: rows fall in different banks)
constexpr int LQA = G2D + 4;  // row stride of the attention operands Q, K, V, dY (16-byte aligned rows)
constexpr int LG = G1D + 1;   // row stride of [edge][64]

__device__ __forceinline__ bool failed(const unsigned *flags) { return (flags[0] & FLAG_ERRORS) != 0u; }

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// tanh and exp of the hot loops from the hardware exponential and reciprocal
// (absolute error a few 1e-8 for tanh; relative a few 1e-7 for the softmax weights).
__device__ __forceinline__ float ftanh(float x) {
  const float t = __expf(-2.f * fabsf(x));
  return copysignf((1.f - t) * __builtin_amdgcn_rcpf(1.f + t), x);
}

constexpr int SELP = 16 * ((SEL + 15) / 16);  // SEL rounded up to whole tiles of 16

// Environment of atom i.  sw and rh are padded to SELP entries (zero past the list) so
// that four consecutive neighbours of a tile are read with 16-byte loads.
struct EnvR {
  float sw[SELP] __attribute__((aligned(16)));
  float rh[SELP * 3] __attribute__((aligned(16)));
  float r[SEL], dsw[SEL], s[SEL];
  int jn[SEL], tj[SEL];
  int nn;
};

// rh of the neighbours k0 .. k0 + 3 (k0 a multiple of 4): h[3 ii + a] = rhat_{k0 + ii}[a].
__device__ __forceinline__ void rh_quad(const EnvR &e, int k0, float (&h)[12]) {
  const float4 a = *reinterpret_cast<const float4 *>(e.rh + 3 * k0);
  const float4 b = *reinterpret_cast<const float4 *>(e.rh + 3 * k0 + 4);
  const float4 c = *reinterpret_cast<const float4 *>(e.rh + 3 * k0 + 8);
  h[0] = a.x; h[1] = a.y; h[2] = a.z; h[3] = a.w;
  h[4] = b.x; h[5] = b.y; h[6] = b.z; h[7] = b.w;
  h[8] = c.x; h[9] = c.y; h[10] = c.z; h[11] = c.w;
}
__device__ __forceinline__ void quad(const float *p, float (&v)[4]) {
  const float4 a = *reinterpret_cast<const float4 *>(p);
  v[0] = a.x; v[1] = a.y; v[2] = a.z; v[3] = a.w;
}

__device__ void build_env_r(EnvR &e, const double *__restrict__ X, const int *__restrict__ types,
                            const int *__restrict__ nlist, const int *__restrict__ nnei, int i, int n, const Grid &g,
                            const Geo &geo) {
  const int nn = min(max(nnei[i], 0), SEL);
  for (int j = threadIdx.x; j < SELP; j += NT) {
    float r = 1.f, sw = 0.f, dsw = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
    int nj = i, tj = 0;
    if (j < nn) {
      nj = nlist[(size_t)i * SEL + j];
      if (nj < 0 || nj >= n) nj = i;
      tj = clamp_type(types[nj]);
      double d[3];
      for (int a = 0; a < 3; ++a) {
        double v = X[3 * nj + a] - X[3 * i + a];
        if (g.periodic) v -= g.L[a] * rint(v * g.invL[a]);
        d[a] = v;
      }
      const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
      r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float u = (r - geo.rcs) / (geo.rc - geo.rcs);
      if (r < geo.rcs) {
        sw = 1.f;
      } else if (r < geo.rc) {
        sw = u * u * u * (-6.f * u * u + 15.f * u - 10.f) + 1.f;
        dsw = -30.f * u * u * (1.f - u) * (1.f - u) / (geo.rc - geo.rcs);
      }
      hx = dx / r; hy = dy / r; hz = dz / r;
    }
    e.sw[j] = sw;
    e.rh[3 * j] = hx; e.rh[3 * j + 1] = hy; e.rh[3 * j + 2] = hz;
    if (j < SEL) {
      e.r[j] = r; e.dsw[j] = dsw; e.s[j] = sw / r;
      e.jn[j] = nj; e.tj[j] = tj;
    }
  }
  if (threadIdx.x == 0) e.nn = nn;
  __syncthreads();
}

__device__ __forceinline__ float Rcomp(const EnvR &e, int j, int a) { return a == 0 ? e.s[j] : e.s[j] * e.rh[3 * j + a - 1]; }

__device__ __forceinline__ size_t erow2(const Buffers &b, int l, int i, int j) {
  return (((size_t)l * b.cap + i) * SEL + j) * G2D;
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }
__device__ __forceinline__ void st4(float *p, float4 v) {  // LDS rows have odd strides: four scalar stores
  p[0] = v.x; p[1] = v.y; p[2] = v.z; p[3] = v.w;
}

// Rows of WIDTH floats (a multiple of 4) for j < nn, copied from global memory (row j
// at src(j)) into LDS rows of stride ld in two steps, so that the reads of several
// arrays can all be issued before the first write.
template <int WIDTH> struct Rows {
  static constexpr int Q = WIDTH / 4, NI = (SEL * Q + NT - 1) / NT;
  float4 v[NI];
  template <class S> __device__ __forceinline__ void issue(int nn, const S &src) {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = threadIdx.x + NT * it, j = k / Q;
      if (j < nn) v[it] = ld4(src(j) + 4 * (k % Q));
    }
  }
  __device__ __forceinline__ void store(float *dst, int ld, int nn) const {
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = threadIdx.x + NT * it, j = k / Q;
      if (j < nn) st4(dst + j * ld + 4 * (k % Q), v[it]);
    }
  }
};

struct NoRows {
  __device__ void issue() {}
  __device__ void store() {}
};

// Layer input of atom i's features: g1 of the neighbours (G1J), g2 of its edges (G2) and
// its own g1 (g1i); `more` issues its own reads after these and stores after them.
template <class More>
__device__ __forceinline__ void load_inputs(const Weights &w, const Buffers &b, const EnvR &e, const int *types, int i,
                                            int l, float *G1J, float *G2, float *g1i, More &more) {
  const int nn = e.nn;
  Rows<G1D> a;
  Rows<G2D> c;
  if (l == 0) {
    a.issue(nn, [&](int j) { return w.TN + e.tj[j] * G1D; });
  } else {
    a.issue(nn, [&](int j) { return b.g1f + ((size_t)(l - 1) * b.cap + e.jn[j]) * G1D; });
    c.issue(nn, [&](int j) { return b.g2f + erow2(b, l - 1, i, j); });
  }
  float gi = 0.f;
  if (threadIdx.x < G1D)
    gi = l == 0 ? w.TN[clamp_type(types[i]) * G1D + threadIdx.x]
                : b.g1f[((size_t)(l - 1) * b.cap + i) * G1D + threadIdx.x];
  more.issue();
  a.store(G1J, LG, nn);
  if (l == 0) {
    for (int k = threadIdx.x; k < nn * G2D; k += NT) {
      const int j = k >> 5, cc = k & 31;
      G2[j * LQ + cc] = tanhf(e.s[j] * w.Wp0[cc] + w.bp0[cc]);
    }
  } else {
    c.store(G2, LQ, nn);
  }
  if (threadIdx.x < G1D) g1i[threadIdx.x] = gi;
  more.store();
}

// Pair update and projections on MFMA (16x16x4 f32), one tile of 16 edges per wave:
// G2A = G2 + tanh([G2, G1J] Wa + ba) (TA, the tanh term, written over G2 when
// `keep_ta`), then Q, K, V = G2A Wq, Wk, Wv.  The weights are B operands held in
// registers (lane l holds W[4 s + l / 16][16 ct + l % 16] for k step s); a wave reads
// and writes only the rows of its own tiles.  Ends synchronised.
__device__ void pair_and_qkv(const Weights &w, int l, int nn, float *G2, const float *G1J, float *G2A, float *Q,
                             float *K, float *V, bool keep_ta) {
  const int ln = lane_id(), wv = wave_id(), kq = ln >> 4, col = ln & 15;
  const int nkt = (nn + 15) >> 4;
  constexpr int KA = (G2D + G1D) / 4, KP = G2D / 4;  // k steps of the two products
  float wa[KA][2], wq[KP][2], wk[KP][2], wvv[KP][2];
#pragma unroll
  for (int st = 0; st < KA; ++st)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) wa[st][ct] = w.Wa[l][(4 * st + kq) * G2D + 16 * ct + col];
#pragma unroll
  for (int st = 0; st < KP; ++st)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) {
      wq[st][ct] = w.Wq[l][(4 * st + kq) * G2D + 16 * ct + col];
      wk[st][ct] = w.Wk[l][(4 * st + kq) * G2D + 16 * ct + col];
      wvv[st][ct] = w.Wv[l][(4 * st + kq) * G2D + 16 * ct + col];
    }
  const float bias[2] = {w.ba[l][col], w.ba[l][16 + col]};
  for (int et = wv; et < nkt; et += NWG) {
    const int ra = 16 * et + col;  // this lane's A-operand row
    const bool aok = ra < nn;
    f4 z[2] = {};
#pragma unroll
    for (int st = 0; st < KA; ++st) {
      const int k = 4 * st + kq;
      const float x = aok ? (k < G2D ? G2[ra * LQ + k] : G1J[ra * LG + k - G2D]) : 0.f;
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) z[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, wa[st][ct], z[ct], 0, 0, 0);
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 16 * et + 4 * kq + ii, c = 16 * ct + col;
        if (r < nn) {
          const float ta = ftanh(z[ct][ii] + bias[ct]);
          G2A[r * LQ + c] = G2[r * LQ + c] + ta;
          if (keep_ta) G2[r * LQ + c] = ta;
        }
      }
    wave_sync();
    f4 q[2] = {}, k[2] = {}, v[2] = {};
#pragma unroll
    for (int st = 0; st < KP; ++st) {
      const float x = aok ? G2A[ra * LQ + 4 * st + kq] : 0.f;
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        q[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, wq[st][ct], q[ct], 0, 0, 0);
        k[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, wk[st][ct], k[ct], 0, 0, 0);
        v[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(x, wvv[st][ct], v[ct], 0, 0, 0);
      }
    }
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 16 * et + 4 * kq + ii, c = 16 * ct + col;
        if (r < nn) {
          Q[r * LQA + c] = q[ct][ii];
          K[r * LQA + c] = k[ct][ii];
          V[r * LQA + c] = v[ct][ii];
        }
      }
  }
  __syncthreads();
}

// One column of the node update's product z_c = b1_c + xs . W1[:, c], split over the
// waves (wave u sums the XD / NWG consecutive inputs from u XD / NWG, in order) and
// combined in wave order; the result is in zc[c] for c < 64.  Ends synchronised.
__device__ void node_product(const float *W1, const float *b1, const float *xs, float (*part)[G1D], float *zc) {
  const int c = threadIdx.x & 63, u = threadIdx.x >> 6;
  constexpr int QW = XD / NWG;
  float v = 0.f;
#pragma unroll 8
  for (int q = u * QW; q < (u + 1) * QW; ++q) v += xs[q] * W1[q * G1D + c];
  part[u][c] = v;
  __syncthreads();
  if (threadIdx.x < G1D) {
    float z = b1[c];
    for (int uu = 0; uu < NWG; ++uu) z += part[uu][c];
    zc[c] = z;
  }
  __syncthreads();
}

// T = sum_j g2_j R_j^T / sel (into T[32][4]), c = sum_j sw_j g2_j g1_j[:32] / sel, and the
// node-update input xs = [g1i, D, c] with D = T T[:4]^T.  Waves 0 and 1 form T^T = R^T G2B
// on MFMA (16x16x4 f32, four neighbours per step, rows a < 4 of the 16 used) over the
// two halves of j; waves 2 .. 5 split the sums of c into eight ranges of j.  Partials go
// to `part` (at least 512 floats) and are added in order.  Ends synchronised.
__device__ void node_inputs(const EnvR &e, int nn, const float *G2B, const float *G1J, const float *g1i,
                            float inv_sel, float *T, float *xs, float *part) {
  static_assert(NWG >= 6, "node_inputs uses six waves");
  constexpr int NSEG = 8;
  const int t = threadIdx.x, wv = wave_id(), ln = lane_id();
  if (wv < 2) {
    const int kq = ln >> 4, col = ln & 15;
    const int j0 = wv * nn / 2, j1 = (wv + 1) * nn / 2;
    f4 acc[2] = {};
    for (int jb = j0; jb < j1; jb += 4) {
      const int j = jb + kq;
      float ra = 0.f;  // A[a = col][j] = R_j[a]
      if (j < j1 && col < 4) ra = col == 0 ? e.s[j] : e.s[j] * e.rh[3 * j + col - 1];
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        const float g = j < j1 ? G2B[j * LQ + 16 * ct + col] : 0.f;
        acc[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(ra, g, acc[ct], 0, 0, 0);
      }
    }
    if (kq == 0)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) part[wv * 128 + (16 * ct + col) * 4 + ii] = acc[ct][ii];
  } else if (wv < 6) {
    const int u = t - 128, c = u % G2D, sg = u / G2D;
    const int j0 = sg * nn / NSEG, j1 = (sg + 1) * nn / NSEG;
    float v = 0.f;
    for (int j = j0; j < j1; ++j) v += e.sw[j] * G2B[j * LQ + c] * G1J[j * LG + c];
    part[256 + u] = v;
  }
  __syncthreads();
  if (t < G2D * 4) {
    T[t] = (part[t] + part[128 + t]) * inv_sel;
  } else if (t < G2D * 5) {
    const int c = t - G2D * 4;
    float v = part[256 + c];
    for (int sg = 1; sg < NSEG; ++sg) v += part[256 + sg * G2D + c];
    xs[G1D + G2D * NAX + c] = v * inv_sel;
  } else if (t >= 256 && t < 256 + G1D) {
    xs[t - 256] = g1i[t - 256];
  }
  __syncthreads();
  if (t < G2D * NAX) {
    const int c = t >> 2, bb = t & 3;  // D[c][b], flattened c * 4 + b
    float v = 0.f;
    for (int a = 0; a < 4; ++a) v += T[c * 4 + a] * T[bb * 4 + a];
    xs[G1D + t] = v;
  }
  __syncthreads();
}

// The attention on MFMA (16x16x4 f32).  Score tiles are kept transposed, keys x
// queries: lane l holds S^T[key 16 kt + 4 (l / 16) + i][query q0 + l % 16], so the
// weights of a query are reduced over i, over the key tiles and across l / 16, and they
// are already the B operand of Y^T = V^T A^T with the k order permuted as in the
// products below (step s of a key tile takes key 16 kt + 4 (l / 16) + s).
// acc += sum_{c < 32} A[r][c] B[col][c] with lane's A row (r = l % 16) at arow and B row
// (col = l % 16) at brow, 16-byte aligned rows of 32 floats; nullptr reads as zeros.
__device__ __forceinline__ void dot32_tile(f4 &acc, const float *arow, const float *brow) {
  const int kq = lane_id() >> 4;
#pragma unroll
  for (int kb = 0; kb < 2; ++kb) {
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 a = arow ? ld4(arow + 16 * kb + 4 * kq) : z;
    const float4 b = brow ? ld4(brow + 16 * kb + 4 * kq) : z;
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, b.x, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, b.y, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, b.z, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, b.w, acc, 0, 0, 0);
  }
}
constexpr int NKT = (SEL + 15) / 16;  // key (or query) tiles of 16

// A operand of out^T = W dX^T for a row-major [32][32] W (dE/dx = dE/dy W^T for y = x W):
// lane l holds W[16 ot + l % 16][16 ct + 4 (l / 16) + ii], the k order of the rows of an
// accumulator tile, so a dX^T tile from a product above is the B operand as it stands.
__device__ __forceinline__ void load_wt(const float *W, float (&r)[2][2][4]) {
  const int kq = lane_id() >> 4, col = lane_id() & 15;
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) r[ot][ct][ii] = W[(16 * ot + col) * G2D + 16 * ct + 4 * kq + ii];
}
// out[ot] += W dX^T over the 32 features, x[ct][ii] = dX^T[16 ct + 4 (l / 16) + ii][l % 16].
__device__ __forceinline__ void wt_product(f4 (&out)[2], const float (&r)[2][2][4], const f4 (&x)[2]) {
#pragma unroll
  for (int ot = 0; ot < 2; ++ot)
#pragma unroll
    for (int ct = 0; ct < 2; ++ct)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii)
        out[ot] = __builtin_amdgcn_mfma_f32_16x16x4f32(r[ot][ct][ii], x[ct][ii], out[ot], 0, 0, 0);
}

// ------------------------------------------------------------------ forward
struct SmemF {
  EnvR env;
  float G1J[SEL * LG];
  float G2[SEL * LQ];   // layer input, then the layer's output g2
  float G2A[SEL * LQ];
  float Q[SEL * LQA] __attribute__((aligned(16)));
  float K[SEL * LQA] __attribute__((aligned(16)));
  float V[SEL * LQA] __attribute__((aligned(16)));
  float g1i[G1D], T[G2D * 4], xs[XD], part[NWG][G1D], zc[G1D];
  float y1[FWID], t2[FWID], dp[FWID];
};

__global__ void __launch_bounds__(NT) k_rep_fwd(Weights w, Buffers b, const double *__restrict__ X,
                                                const int *__restrict__ types, const int *__restrict__ nlist,
                                                const int *__restrict__ nnei, const Grid *__restrict__ grids, int n,
                                                int l, Geo geo, double *__restrict__ Ei,
                                                const unsigned *__restrict__ flags) {
  __shared__ SmemF sm;
  const int i = blockIdx.x;
  if (i >= n || failed(flags)) return;
  const int tid = threadIdx.x, wv = wave_id(), ln = lane_id();
  build_env_r(sm.env, X, types, nlist, nnei, i, n, grids[0], geo);
  const EnvR &e = sm.env;
  const int nn = e.nn;
  NoRows none;
  load_inputs(w, b, e, types, i, l, sm.G1J, sm.G2, sm.g1i, none);
  __syncthreads();
  pair_and_qkv(w, l, nn, sm.G2, sm.G1J, sm.G2A, sm.Q, sm.K, sm.V, false);

  // attention, one tile of 16 queries per wave
  const float isq = 1.f / sqrtf((float)G2D);
  const int nkt = (nn + 15) >> 4;
  const int kq = ln >> 4, col = ln & 15;
  for (int qt = wv; qt < nkt; qt += NWG) {
    const int qme = 16 * qt + col;  // this lane's query
    const bool qok = qme < nn;
    f4 st[NKT];
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      st[kt] = f4{0.f, 0.f, 0.f, 0.f};
      if (kt < nkt) {
        const int kr = 16 * kt + col;
        dot32_tile(st[kt], kr < nn ? sm.K + kr * LQA : nullptr, qok ? sm.Q + qme * LQA : nullptr);
      }
    }
    // weights of the lane's query over its keys: max, then sw_k exp(S - max) / sum, times the gate
    float m = -INFINITY;
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int k = 16 * kt + 4 * kq + ii;
        if (kt < nkt && k < nn) m = fmaxf(m, st[kt][ii] * isq);
      }
    m = fmaxf(m, __shfl_xor(m, 16));
    m = fmaxf(m, __shfl_xor(m, 32));
    float z = 0.f;
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      float swv[4];
      quad(e.sw + 16 * kt + 4 * kq, swv);
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int k = 16 * kt + 4 * kq + ii;
        const float ex = (kt < nkt && k < nn) ? swv[ii] * __expf(st[kt][ii] * isq - m) : 0.f;
        st[kt][ii] = ex;
        z += ex;
      }
    }
    z += __shfl_xor(z, 16);
    z += __shfl_xor(z, 32);
    const float iz = qok ? 1.f / z : 0.f;
    const float hx = e.rh[3 * (qok ? qme : 0)], hy = e.rh[3 * (qok ? qme : 0) + 1], hz = e.rh[3 * (qok ? qme : 0) + 2];
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      float h[12];
      rh_quad(e, 16 * kt + 4 * kq, h);
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) st[kt][ii] *= iz * (hx * h[3 * ii] + hy * h[3 * ii + 1] + hz * h[3 * ii + 2]);
    }
    // Y^T[c][q] = sum_k V[k][c] A^T[k][q], two tiles of 16 features
    f4 yt[2] = {};
#pragma unroll
    for (int kt = 0; kt < NKT; ++kt) {
      if (kt >= nkt) break;
#pragma unroll
      for (int ss = 0; ss < 4; ++ss) {
        const int k = 16 * kt + 4 * kq + ss;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const float v = k < nn ? sm.V[k * LQA + 16 * ct + col] : 0.f;
          yt[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(v, st[kt][ss], yt[ct], 0, 0, 0);
        }
      }
    }
    if (qok)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int c = 16 * ct + 4 * kq + ii;
          const float g2b = sm.G2A[qme * LQ + c] + yt[ct][ii];
          sm.G2[qme * LQ + c] = g2b;
          b.g2f[erow2(b, l, i, qme) + c] = g2b;
        }
  }
  __syncthreads();

  node_inputs(e, nn, sm.G2, sm.G1J, sm.g1i, geo.inv_sel, sm.T, sm.xs, &sm.part[0][0]);
  node_product(w.W1[l], w.b1[l], sm.xs, sm.part, sm.zc);
  float g1n = 0.f;
  if (tid < G1D) {
    g1n = sm.g1i[tid] + tanhf(sm.zc[tid]);
    if (l < NLAYER - 1) b.g1f[((size_t)l * b.cap + i) * G1D + tid] = g1n;
  }
  if (l < NLAYER - 1) return;

  // fitting net, E_i and dE/dg1_i
  __syncthreads();
  if (tid < G1D) sm.g1i[tid] = g1n;
  __syncthreads();
  if (tid < FWID) {
    float z = w.d1[tid];
    for (int k = 0; k < G1D; ++k) z += sm.g1i[k] * w.G1[k * FWID + tid];
    sm.y1[tid] = tanhf(z);
  }
  __syncthreads();
  if (tid < FWID) {
    float z = w.d2[tid];
    for (int k = 0; k < FWID; ++k) z += sm.y1[k] * w.G2[k * FWID + tid];
    const float t2 = tanhf(z);
    sm.t2[tid] = t2;
    sm.dp[tid] = w.G3[tid] * (1.f - t2 * t2);
  }
  __syncthreads();
  if (tid == 0) {
    double E = w.d3;
    for (int k = 0; k < FWID; ++k) E += (double)(sm.t2[k] + sm.y1[k]) * w.G3d[k];
    Ei[i] = E;
  }
  float dp1 = 0.f;
  if (tid < FWID) {
    float dy1 = w.G3[tid];
    for (int k = 0; k < FWID; ++k) dy1 += sm.dp[k] * w.G2[tid * FWID + k];
    dp1 = dy1 * (1.f - sm.y1[tid] * sm.y1[tid]);
  }
  __syncthreads();
  if (tid < FWID) sm.dp[tid] = dp1;
  __syncthreads();
  if (tid < G1D) {
    float dn = 0.f;
    for (int k = 0; k < FWID; ++k) dn += sm.dp[k] * w.G1[tid * FWID + k];
    b.dnl[(size_t)i * G1D + tid] = dn;
  }
}

// ------------------------------------------------------------------ backward
struct SmemB {
  EnvR env;
  float G1J[SEL * LG];
  float G2[SEL * LQ];    // layer input g2, then the pair update's tanh term
  float G2A[SEL * LQ];   // after the pair update; later dE/dg2a
  float Q[SEL * LQA] __attribute__((aligned(16)));
  float K[SEL * LQA] __attribute__((aligned(16)));
  float V[SEL * LQA] __attribute__((aligned(16)));
  float G2B[SEL * LQ];   // the layer's output g2
  float DY[SEL * LQA] __attribute__((aligned(16)));  // dE/dg2 of the output; later the pair update's dz
  float EG[SEL * GSN];   // per-edge dE/ds, dE/dsw, dE/drhat
  float stat[3][SELP] __attribute__((aligned(16)));  // per query row: max score, 1 / normaliser, rho
  float g1i[G1D], T[G2D * 4], xs[XD], dg1[G1D], dxn[XD], dT[G2D * 4], part[NWG][G1D], zc[G1D];
  int slot[SEL];
};

__global__ void __launch_bounds__(NT) k_rep_bwd(Weights w, Buffers b, const double *__restrict__ X,
                                                const int *__restrict__ types, const int *__restrict__ nlist,
                                                const int *__restrict__ nnei, const Grid *__restrict__ grids, int n,
                                                int l, Geo geo, float4 *__restrict__ gout,
                                                const unsigned *__restrict__ flags) {
  __shared__ SmemB sm;
  const int i = blockIdx.x;
  if (i >= n || failed(flags)) return;
  const int tid = threadIdx.x, wv = wave_id(), ln = lane_id();
  const bool top = l == NLAYER - 1;
  build_env_r(sm.env, X, types, nlist, nnei, i, n, grids[0], geo);
  const EnvR &e = sm.env;
  const int nn = e.nn;
  // the layer's output g2, the output gradient and edge terms from the layer above and
  // the reverse slots, read together with the layer input
  struct More {
    const Buffers &b;
    SmemB &sm;
    int i, l, nn;
    bool top;
    Rows<G2D> g2b, dy;
    Rows<GSN> eg;
    int sl;
    __device__ void issue() {
      g2b.issue(nn, [&](int j) { return b.g2f + erow2(b, l, i, j); });
      if (!top) {
        dy.issue(nn, [&](int j) { return b.dg2 + ((size_t)i * SEL + j) * G2D; });
        eg.issue(nn, [&](int j) { return b.gs + ((size_t)i * SEL + j) * GSN; });
        if ((int)threadIdx.x < nn) sl = b.slot[(size_t)i * SEL + threadIdx.x];
      }
    }
    __device__ void store() {
      g2b.store(sm.G2B, LQ, nn);
      if (top) {
        for (int k = threadIdx.x; k < nn * G2D; k += NT) sm.DY[(k >> 5) * LQA + (k & 31)] = 0.f;
        for (int k = threadIdx.x; k < nn * GSN; k += NT) sm.EG[k] = 0.f;
      } else {
        dy.store(sm.DY, LQA, nn);
        eg.store(sm.EG, GSN, nn);
        if ((int)threadIdx.x < nn) sm.slot[threadIdx.x] = sl;
      }
    }
  } more{b, sm, i, l, nn, top, {}, {}, {}, -1};
  load_inputs(w, b, e, types, i, l, sm.G1J, sm.G2, sm.g1i, more);
  __syncthreads();
  {  // dE/dg1_i after this layer: own part + the neighbours' edge parts, rows by wave, waves in order
    float v = 0.f;
    if (!top) {
      const float *src = b.dnj + (size_t)((l + 1) & 1) * b.cap * SEL * G1D;
#pragma unroll 8
      for (int j = wv; j < nn; j += NWG) {  // branch-free (a missing slot reads row 0 and adds 0), so the loads overlap
        const int sj = sm.slot[j];
        const float x = src[((size_t)e.jn[j] * SEL + max(sj, 0)) * G1D + ln];
        v += sj >= 0 ? x : 0.f;
      }
    }
    sm.part[wv][ln] = v;
  }
  __syncthreads();
  if (tid < G1D) {
    float v = b.dnl[(size_t)i * G1D + tid];
    for (int u = 0; u < NWG; ++u) v += sm.part[u][tid];
    sm.dg1[tid] = v;
  }
  // recompute the layer's forward: pair update (tanh term kept in G2), projections, node input
  pair_and_qkv(w, l, nn, sm.G2, sm.G1J, sm.G2A, sm.Q, sm.K, sm.V, true);
  node_inputs(e, nn, sm.G2B, sm.G1J, sm.g1i, geo.inv_sel, sm.T, sm.xs, &sm.part[0][0]);
  // node backward: dz = dg1 (1 - t^2), dxn = W1 dz
  node_product(w.W1[l], w.b1[l], sm.xs, sm.part, sm.zc);
  if (tid < G1D) {
    const float t = tanhf(sm.zc[tid]);
    sm.zc[tid] = sm.dg1[tid] * (1.f - t * t);
  }
  __syncthreads();
  if (tid < XD) {
    float v = 0.f;
#pragma unroll 16
    for (int k = 0; k < G1D; ++k) v += sm.zc[k] * w.W1[l][tid * G1D + k];
    sm.dxn[tid] = v;
  }
  __syncthreads();
  // dT from dD = dxn[64:192] (D[c][b] = sum_a T[c][a] T[b][a], b < 4), then / sel
  if (tid < G2D * 4) {
    const int c = tid >> 2, a = tid & 3;
    float v = 0.f;
    for (int bb = 0; bb < 4; ++bb) v += sm.dxn[G1D + c * 4 + bb] * sm.T[bb * 4 + a];
    if (c < 4)
      for (int m = 0; m < G2D; ++m) v += sm.dxn[G1D + m * 4 + c] * sm.T[m * 4 + a];
    sm.dT[tid] = v * geo.inv_sel;
  }
  __syncthreads();
  const float *dc = sm.dxn + G1D + G2D * NAX;  // dE/dc (times sel: divided where used)
  // dE/dg2 of the output from the contraction and the convolution; edge terms of R and sw.
  // dR = G2B dT runs on MFMA, one tile of 16 edges per wave (B operand dT[c][a], columns
  // a < 4 of the 16 used), into part[4 j + a].
  {
    const int kq = ln >> 4, col = ln & 15, net = (nn + 15) >> 4;
    float bv[G2D / 4];
#pragma unroll
    for (int st = 0; st < G2D / 4; ++st) bv[st] = col < 4 ? sm.dT[(4 * st + kq) * 4 + col] : 0.f;
    float *dRs = &sm.part[0][0];
    for (int et = wv; et < net; et += NWG) {
      const int ra = 16 * et + col;
      f4 acc = {};
#pragma unroll
      for (int st = 0; st < G2D / 4; ++st) {
        const float x = ra < nn ? sm.G2B[ra * LQ + 4 * st + kq] : 0.f;
        acc = __builtin_amdgcn_mfma_f32_16x16x4f32(x, bv[st], acc, 0, 0, 0);
      }
      if (col < 4)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int j = 16 * et + 4 * kq + ii;
          if (j < nn) dRs[4 * j + col] = acc[ii];
        }
    }
  }
  for (int o = tid; o < nn * G2D; o += NT) {
    const int j = o >> 5, c = o & 31;
    float v = sm.DY[j * LQA + c] + e.sw[j] * dc[c] * geo.inv_sel * sm.G1J[j * LG + c];
    for (int a = 0; a < 4; ++a) v += sm.dT[c * 4 + a] * Rcomp(e, j, a);
    sm.DY[j * LQA + c] = v;
  }
  __syncthreads();
  for (int j = tid; j < nn; j += NT) {
    const float *dR = &sm.part[0][0] + 4 * j;
    float dswc = 0.f;
#pragma unroll 8
    for (int c = 0; c < G2D; ++c) dswc += dc[c] * geo.inv_sel * sm.G2B[j * LQ + c] * sm.G1J[j * LG + c];
    float *eg = sm.EG + j * GSN;
    eg[0] += dR[0] + dR[1] * e.rh[3 * j] + dR[2] * e.rh[3 * j + 1] + dR[3] * e.rh[3 * j + 2];
    eg[1] += dswc;
    for (int a = 0; a < 3; ++a) eg[2 + a] += e.s[j] * dR[1 + a];
  }
  __syncthreads();

  // attention backward on MFMA.  Row pass: one tile of 16 queries per wave with the
  // score tiles transposed as in the forward; the query's statistics (max, 1 / normaliser,
  // rho), its terms of the gate gradient, dQ^T = K^T dS^T and the query rows of
  // dE/dg2a = dY + dQ Wq^T.
  const float isq = 1.f / sqrtf((float)G2D);
  const int nkt = (nn + 15) >> 4;
  const int kq = ln >> 4, col = ln & 15;
  {
    for (int qt = wv; qt < nkt; qt += NWG) {
      const int qme = 16 * qt + col;
      const bool qok = qme < nn;
      float wq[2][2][4];  // issued first: their latency overlaps the score tiles
      load_wt(w.Wq[l], wq);
      f4 st[NKT], da[NKT];  // S^T and dA^T = V dY^T: [key 16 kt + 4 kq + ii][query qme]
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        st[kt] = f4{0.f, 0.f, 0.f, 0.f};
        da[kt] = f4{0.f, 0.f, 0.f, 0.f};
        if (kt < nkt) {
          const int kr = 16 * kt + col;
          dot32_tile(st[kt], kr < nn ? sm.K + kr * LQA : nullptr, qok ? sm.Q + qme * LQA : nullptr);
          dot32_tile(da[kt], kr < nn ? sm.V + kr * LQA : nullptr, qok ? sm.DY + qme * LQA : nullptr);
        }
      }
      float m = -INFINITY;
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int k = 16 * kt + 4 * kq + ii;
          if (kt < nkt && k < nn) m = fmaxf(m, st[kt][ii] * isq);
        }
      m = fmaxf(m, __shfl_xor(m, 16));
      m = fmaxf(m, __shfl_xor(m, 32));
      float z = 0.f;
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        float swv[4];
        quad(e.sw + 16 * kt + 4 * kq, swv);
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int k = 16 * kt + 4 * kq + ii;
          const float ex = (kt < nkt && k < nn) ? swv[ii] * __expf(st[kt][ii] * isq - m) : 0.f;
          st[kt][ii] = ex;
          z += ex;
        }
      }
      z += __shfl_xor(z, 16);
      z += __shfl_xor(z, 32);
      const float iz = qok ? 1.f / z : 0.f;
      const int qq = qok ? qme : 0;
      const float hx = e.rh[3 * qq], hy = e.rh[3 * qq + 1], hz = e.rh[3 * qq + 2];
      // P, dP = dA gate, rho = sum_k dP P and the row terms sum_k dA P rhat_k of the gate
      float rho = 0.f, h0 = 0.f, h1 = 0.f, h2 = 0.f;
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        float h[12];
        rh_quad(e, 16 * kt + 4 * kq, h);
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const float rx = h[3 * ii], ry = h[3 * ii + 1], rz = h[3 * ii + 2];
          const float P = st[kt][ii] * iz, dA = da[kt][ii];
          const float dP = dA * (hx * rx + hy * ry + hz * rz), dG = dA * P;
          rho += dP * P;
          h0 += dG * rx;
          h1 += dG * ry;
          h2 += dG * rz;
          st[kt][ii] = P;
          da[kt][ii] = dP;
        }
      }
#pragma unroll
      for (int o = 16; o < 64; o <<= 1) {
        rho += __shfl_xor(rho, o);
        h0 += __shfl_xor(h0, o);
        h1 += __shfl_xor(h1, o);
        h2 += __shfl_xor(h2, o);
      }
      if (qok && kq == 0) {
        sm.stat[0][qme] = m;
        sm.stat[1][qme] = iz;
        sm.stat[2][qme] = rho;
        sm.EG[qme * GSN + 2] += h0;
        sm.EG[qme * GSN + 3] += h1;
        sm.EG[qme * GSN + 4] += h2;
      }
      // dS^T = P (dP - rho) / sqrt(32); dQ^T[c][q] = sum_k K[k][c] dS^T[k][q]
      f4 dq[2] = {};
#pragma unroll
      for (int kt = 0; kt < NKT; ++kt) {
        if (kt >= nkt) break;
#pragma unroll
        for (int ss = 0; ss < 4; ++ss) {
          const int k = 16 * kt + 4 * kq + ss;
          const float ds = st[kt][ss] * (da[kt][ss] - rho) * isq;
#pragma unroll
          for (int ct = 0; ct < 2; ++ct) {
            const float kv = k < nn ? sm.K[k * LQA + 16 * ct + col] : 0.f;
            dq[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(kv, ds, dq[ct], 0, 0, 0);
          }
        }
      }
      f4 o[2] = {};
      wt_product(o, wq, dq);
      if (qok)
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            const int c = 16 * ot + 4 * kq + ii;
            sm.G2A[qme * LQ + c] = sm.DY[qme * LQA + c] + o[ot][ii];  // dE/dg2a, row terms
          }
    }
  }
  __syncthreads();
  // column pass: one tile of 16 keys per wave, streaming over the query tiles with the
  // scores S[query][key] recomputed; the key terms of the switch and gate,
  // dV^T = dY^T A, dK^T = Q^T dS and the key rows of dE/dg2a += dV Wv^T + dK Wk^T.
  for (int kt = wv; kt < nkt; kt += NWG) {
    const int kme = 16 * kt + col;
    const bool kok = kme < nn;
    const int kk = kok ? kme : 0;
    float wk[2][2][4], wvv[2][2][4];  // issued first: their latency overlaps the query tiles
    load_wt(w.Wk[l], wk);
    load_wt(w.Wv[l], wvv);
    const float kx = e.rh[3 * kk], ky = e.rh[3 * kk + 1], kz = e.rh[3 * kk + 2], swk = e.sw[kk];
    float dsk = 0.f, h0 = 0.f, h1 = 0.f, h2 = 0.f;
    f4 dv[2] = {}, dk[2] = {};
    for (int jt = 0; jt < nkt; ++jt) {
      f4 sc = {}, da = {};  // S and dA = dY V^T: [query 16 jt + 4 kq + ii][key kme]
      const int jr = 16 * jt + col;
      dot32_tile(sc, jr < nn ? sm.Q + jr * LQA : nullptr, kok ? sm.K + kme * LQA : nullptr);
      dot32_tile(da, jr < nn ? sm.DY + jr * LQA : nullptr, kok ? sm.V + kme * LQA : nullptr);
      float h[12], mx[4], iz[4], rh4[4];
      rh_quad(e, 16 * jt + 4 * kq, h);
      quad(sm.stat[0] + 16 * jt + 4 * kq, mx);
      quad(sm.stat[1] + 16 * jt + 4 * kq, iz);
      quad(sm.stat[2] + 16 * jt + 4 * kq, rh4);
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int j = 16 * jt + 4 * kq + ii;
        float A = 0.f, ds = 0.f;
        if (kok && j < nn) {
          const float exz = __expf(sc[ii] * isq - mx[ii]) * iz[ii];
          const float rx = h[3 * ii], ry = h[3 * ii + 1], rz = h[3 * ii + 2];
          const float P = swk * exz, g = rx * kx + ry * ky + rz * kz, dA = da[ii];
          const float dP = dA * g, dG = dA * P, rho = rh4[ii];
          A = P * g;
          ds = P * (dP - rho) * isq;
          dsk += exz * (dP - rho);
          h0 += dG * rx;
          h1 += dG * ry;
          h2 += dG * rz;
        }
        sc[ii] = A;
        da[ii] = ds;
      }
#pragma unroll
      for (int ss = 0; ss < 4; ++ss) {
        const int j = 16 * jt + 4 * kq + ss;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const float dy = j < nn ? sm.DY[j * LQA + 16 * ct + col] : 0.f;
          const float qv = j < nn ? sm.Q[j * LQA + 16 * ct + col] : 0.f;
          dv[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(dy, sc[ss], dv[ct], 0, 0, 0);
          dk[ct] = __builtin_amdgcn_mfma_f32_16x16x4f32(qv, da[ss], dk[ct], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int o = 16; o < 64; o <<= 1) {
      dsk += __shfl_xor(dsk, o);
      h0 += __shfl_xor(h0, o);
      h1 += __shfl_xor(h1, o);
      h2 += __shfl_xor(h2, o);
    }
    if (kok && kq == 0) {
      sm.EG[kme * GSN + 1] += dsk;
      sm.EG[kme * GSN + 2] += h0;
      sm.EG[kme * GSN + 3] += h1;
      sm.EG[kme * GSN + 4] += h2;
    }
    f4 o[2] = {};
    wt_product(o, wvv, dv);
    wt_product(o, wk, dk);
    if (kok)
#pragma unroll
      for (int ot = 0; ot < 2; ++ot)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int c = 16 * ot + 4 * kq + ii;
          sm.G2A[kme * LQ + c] += o[ot][ii];  // dE/dg2a, complete
        }
  }
  __syncthreads();
  // pair update backward: dz = dE/dg2a (1 - ta^2) into DY
  for (int o = tid; o < nn * G2D; o += NT) {
    const int j = o >> 5, c = o & 31;
    const float ta = sm.G2[j * LQ + c];
    sm.DY[j * LQA + c] = sm.G2A[j * LQ + c] * (1.f - ta * ta);
  }
  __syncthreads();
  // dxa = dz Wa^T on MFMA, one tile of 16 edges per wave; k step s of block kb takes
  // k = 16 kb + 4 (l / 16) + s, so a lane's four B values (Wa[16 qt + l % 16][k]) and A
  // values (dz[row][k]) are each one 16-byte load.  Its first 32 columns go to dE/dg2 of
  // the layer input, the other 64 (with the convolution's term) to the edge's part of
  // dE/dg1_j
  float *dnj = b.dnj + (size_t)(l & 1) * b.cap * SEL * G1D;
  {
    constexpr int QT = (G2D + G1D) / 16;
    float4 wt[2][QT];
#pragma unroll
    for (int kb = 0; kb < 2; ++kb)
#pragma unroll
      for (int qt = 0; qt < QT; ++qt) wt[kb][qt] = ld4(w.Wa[l] + (16 * qt + col) * G2D + 16 * kb + 4 * kq);
    for (int et = wv; et < nkt; et += NWG) {
      const int ra = 16 * et + col;
      const bool aok = ra < nn;
      f4 acc[QT] = {};
#pragma unroll
      for (int kb = 0; kb < 2; ++kb) {
        const float4 x = aok ? ld4(sm.DY + ra * LQA + 16 * kb + 4 * kq) : make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
        for (int qt = 0; qt < QT; ++qt) {
          acc[qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.x, wt[kb][qt].x, acc[qt], 0, 0, 0);
          acc[qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.y, wt[kb][qt].y, acc[qt], 0, 0, 0);
          acc[qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.z, wt[kb][qt].z, acc[qt], 0, 0, 0);
          acc[qt] = __builtin_amdgcn_mfma_f32_16x16x4f32(x.w, wt[kb][qt].w, acc[qt], 0, 0, 0);
        }
      }
#pragma unroll
      for (int qt = 0; qt < QT; ++qt)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int j = 16 * et + 4 * kq + ii, q = 16 * qt + col;
          if (j >= nn) continue;
          float v = acc[qt][ii];
          if (q < G2D) {
            const float dg2in = sm.G2A[j * LQ + q] + v;
            if (l > 0) b.dg2[((size_t)i * SEL + j) * G2D + q] = dg2in;
            else sm.V[j * LQA + q] = dg2in;  // kept for the initial-feature gradient below
          } else if (l > 0) {
            const int c1 = q - G2D;
            if (c1 < G2D) v += e.sw[j] * dc[c1] * geo.inv_sel * sm.G2B[j * LQ + c1];
            dnj[((size_t)i * SEL + j) * G1D + c1] = v;
          }
        }
    }
  }
  if (l > 0) {
    if (tid < G1D) {
      float v = sm.dg1[tid] + sm.dxn[tid];
      b.dnl[(size_t)i * G1D + tid] = v;
    }
    for (int k = tid; k < nn * GSN; k += NT) b.gs[(size_t)i * SEL * GSN + k] = sm.EG[k];
    return;
  }
  __syncthreads();
  // layer 0: g2 = tanh(s Wp0 + bp0) adds to dE/ds; then g_ij = dE/dDelta_ij
  for (int j = tid; j < nn; j += NT) {
    float ds = sm.EG[j * GSN];
    for (int c = 0; c < G2D; ++c) {
      const float g0 = tanhf(e.s[j] * w.Wp0[c] + w.bp0[c]);
      ds += sm.V[j * LQA + c] * (1.f - g0 * g0) * w.Wp0[c];
    }
    const float rr = e.r[j], sw = e.sw[j];
    const float dr = ds * (e.dsw[j] / rr - sw / (rr * rr)) + sm.EG[j * GSN + 1] * e.dsw[j];
    const float hx = e.rh[3 * j], hy = e.rh[3 * j + 1], hz = e.rh[3 * j + 2];
    const float gx = sm.EG[j * GSN + 2], gy = sm.EG[j * GSN + 3], gz = sm.EG[j * GSN + 4];
    const float proj = gx * hx + gy * hy + gz * hz;
    gout[(size_t)i * SEL + j] = make_float4((gx - proj * hx) / rr + dr * hx, (gy - proj * hy) / rr + dr * hy,
                                            (gz - proj * hz) / rr + dr * hz, 0.f);
  }
}

__global__ void __launch_bounds__(1024) k_edge_count(const int *__restrict__ nnei, int n, int64_t *__restrict__ etot) {
  __shared__ int64_t part[1024];
  int64_t s = 0;
  for (int k = threadIdx.x; k < n; k += 1024) s += min(max(nnei[k], 0), SEL);
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int k = 0; k < 1024; ++k) t += part[k];
    *etot = t;
  }
}

}  // namespace

void launch_edge_count(const Buffers &b, const Workspace &ws, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_edge_count, dim3(1), dim3(1024), 0, st, ws.nnei, n, b.etot);
}

void launch_layer_fwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, double *Ei, hipStream_t st) {
  hipLaunchKernelGGL(k_rep_fwd, dim3(n), dim3(NT), 0, st, w, b, coords, types, ws.nlist, ws.nnei, ws.grids, n, layer,
                     geo, Ei, ws.flags);
}

void launch_layer_bwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, hipStream_t st) {
  hipLaunchKernelGGL(k_rep_bwd, dim3(n), dim3(NT), 0, st, w, b, coords, types, ws.nlist, ws.nnei, ws.grids, n, layer,
                     geo, ws.g, ws.flags);
}

}  // namespace rep
}  // namespace dp
