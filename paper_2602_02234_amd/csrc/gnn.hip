// GNN-variant descriptor kernels for gfx950: one workgroup (four waves) per centre atom
// and one launch per message-passing layer, forward and backward (a layer's edge update
// reads the neighbours' node features of the layer before, so layers meet at launch
// boundaries).  Every product of a feature tile with a weight matrix runs on MFMA
// (16 angles or 16 edges per tile, f32 or bf16 operands, f32 accumulation); feature
// tiles are staged in per-wave LDS slabs and the angle weights of a layer stay in each
// wave's registers for all its tiles.  Features are stored in float32.
//
// Forward, layer l, centre i:
//   angles  each wave owns angle rows p (p = wave, wave + 4, ...) and walks q in tiles
//           of 16: a' = a + tanh([a, e_ip, e_iq] Waa + b), then the message tile
//           tanh([a', e_iq] Wea + b) weighted by sw_a(r_ip) sw_a(r_iq) / asel and summed
//           over q in a fixed order into m_ip;
//   edges   tiles of 16 edges: e' = e + tanh([n_i, n_j, e] Wee + b) + m;
//   node    n' = n + tanh([n, sum_j sw_e e' / sel] Wnn + b); after the last layer the
//           fitting net, E_i in float64, and dE/dn_i.
// Backward, layer l (reverse of the above, activations recomputed from the stored layer
// inputs): dE/dn_i is gathered from the edges (j, i) of the neighbours in list order
// (binary search of i in N(j)); per-angle terms that belong to edge (i, q) are summed
// per wave in LDS and the wave sums added in wave order, so every sum has a fixed order
// and the result is deterministic.  Layer 0 turns the accumulated gradients of s, sw_e,
// sw_a and rhat into g_ij = dE/dDelta_ij for the shared force gather.
#include "dp_env.h"
#include "gnn.h"

namespace dp {
namespace gnn {
namespace {

constexpr int NWG = 4;          // waves per workgroup
constexpr int NT = NWG * 64;
constexpr int LDE = 68;         // row stride of [edge][64] LDS arrays
constexpr int LDF = 196;        // forward slab row stride (192 columns used)
constexpr int LDB = 164;        // backward slab row stride (160 columns used)
constexpr int QLD = 36;         // per-edge angle accumulators: 32 features, sw_a, rhat

__device__ __forceinline__ bool failed(const unsigned *flags) { return (flags[0] & FLAG_ERRORS) != 0u; }

// Ordering of LDS traffic between the lanes of one wave (per-wave slabs).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Sum over all 64 lanes, the same in every lane.
__device__ __forceinline__ float wave_sum64(float v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Weight fragments held in registers for one 16-column tile of a product X W (X: 16
// rows in an LDS slab, W: K x 16).  The k order inside each MFMA step is permuted
// (the sum does not depend on it) so that a lane's A operands for consecutive steps
// are adjacent in LDS and come in 128-bit reads: f32, steps s = 0..3 of block kb use
// k = 16 kb + 4 (lane / 16) + s; bf16, block kb uses k = 32 kb + 8 (lane / 16) + e.
// y(c, k) gives W[k][c]; col(k0) maps the first k of a block to its slab column
// (operands may come from several column ranges, each a multiple of 32 wide).
template <typename T, int K> struct Frag;

template <int K> struct Frag<float, K> {
  float v[K / 4];
  template <class Y> __device__ __forceinline__ void load(const Y &y) {
    const int c = lane_id() & 15, kq = lane_id() >> 4;
#pragma unroll
    for (int kb = 0; kb < K / 16; ++kb)
#pragma unroll
      for (int s = 0; s < 4; ++s) v[kb * 4 + s] = y(c, kb * 16 + 4 * kq + s);
  }
  template <class C> __device__ __forceinline__ void mma(f4 &acc, const float *row, const C &col) const {
    const int kq = lane_id() >> 4;
#pragma unroll
    for (int kb = 0; kb < K / 16; ++kb) {
      const float4 a = *reinterpret_cast<const float4 *>(row + col(kb * 16) + 4 * kq);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.x, v[kb * 4 + 0], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.y, v[kb * 4 + 1], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.z, v[kb * 4 + 2], acc, 0, 0, 0);
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.w, v[kb * 4 + 3], acc, 0, 0, 0);
    }
  }
};

template <int K> struct Frag<bf16_t, K> {
  bf8 v[K / 32];
  template <class Y> __device__ __forceinline__ void load(const Y &y) {
    const int c = lane_id() & 15, kq = lane_id() >> 4;
#pragma unroll
    for (int kb = 0; kb < K / 32; ++kb)
#pragma unroll
      for (int e = 0; e < 8; ++e) v[kb][e] = (__bf16)y(c, kb * 32 + 8 * kq + e);
  }
  template <class C> __device__ __forceinline__ void mma(f4 &acc, const float *row, const C &col) const {
    const int kq = lane_id() >> 4;
#pragma unroll
    for (int kb = 0; kb < K / 32; ++kb) {
      const float *q = row + col(kb * 32) + 8 * kq;
      const float4 a0 = *reinterpret_cast<const float4 *>(q);
      const float4 a1 = *reinterpret_cast<const float4 *>(q + 4);
      bf8 a;
      a[0] = (__bf16)a0.x; a[1] = (__bf16)a0.y; a[2] = (__bf16)a0.z; a[3] = (__bf16)a0.w;
      a[4] = (__bf16)a1.x; a[5] = (__bf16)a1.y; a[6] = (__bf16)a1.z; a[7] = (__bf16)a1.w;
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, v[kb], acc, 0, 0, 0);
    }
  }
};

// tanh of the layers' hot loops, from the hardware exponential and reciprocal:
// tanh|x| = (1 - t) / (1 + t), t = exp(-2|x|); absolute error a few 1e-8, below the
// float32 rounding of the products it follows (measured forces unchanged against tanhf).
template <typename T> __device__ __forceinline__ float act(float x) {
  const float t = __expf(-2.f * fabsf(x));
  return copysignf((1.f - t) * __builtin_amdgcn_rcpf(1.f + t), x);
}

// Compiler barrier: weight fragments loaded after it are not hoisted out of the loop
// around it (they would then all be live at once).
__device__ __forceinline__ void opaque() { asm volatile("" ::: "memory"); }

struct Ident {
  __device__ __forceinline__ int operator()(int k) const { return k; }
};
struct Shift {  // operands at slab columns from `s` on
  int s;
  __device__ __forceinline__ int operator()(int k) const { return s + k; }
};

struct GEnv {
  float r[SEL], swe[SEL], dswe[SEL], swa[SEL], dswa[SEL], s[SEL];
  float rh[SEL * 3];
  int jn[SEL], tj[SEL], cpos[SEL];  // neighbour, its type, its angle-list position (-1: none)
  int cl[ASEL];                      // edge slot of each angle-list position
  int nn, nc;
};

__device__ __forceinline__ float quintic(float r, float rc, float rcs, float &dsw) {
  const float u = (r - rcs) / (rc - rcs);
  dsw = 0.f;
  if (r < rcs) return 1.f;
  if (r >= rc) return 0.f;
  dsw = -30.f * u * u * (1.f - u) * (1.f - u) / (rc - rcs);
  return u * u * u * (-6.f * u * u + 15.f * u - 10.f) + 1.f;
}

// Geometry of centre i's edges and its angle list (the first asel neighbours, in list
// order, closer than rca; the test is made in float64 on the minimum-image vector).
__device__ void build_genv(GEnv &e, const double *__restrict__ X, const int *__restrict__ types,
                           const int *__restrict__ nlist, const int *__restrict__ nnei, int i, int n,
                           const Grid &g, const Geo &geo) {
  const int nn = min(max(nnei[i], 0), SEL);
  for (int j = threadIdx.x; j < SEL; j += NT) {
    float r = 1.f, sw = 0.f, dsw = 0.f, sa = 0.f, dsa = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
    int nj = i, tj = 0, close = 0;
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
      close = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < (double)geo.rca;
      const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
      r = sqrtf(dx * dx + dy * dy + dz * dz);
      sw = quintic(r, geo.rc, geo.rcs, dsw);
      sa = quintic(r, geo.rca, geo.rcs, dsa);
      hx = dx / r; hy = dy / r; hz = dz / r;
    }
    e.r[j] = r; e.swe[j] = sw; e.dswe[j] = dsw; e.swa[j] = sa; e.dswa[j] = dsa; e.s[j] = sw / r;
    e.rh[3 * j] = hx; e.rh[3 * j + 1] = hy; e.rh[3 * j + 2] = hz;
    e.jn[j] = nj; e.tj[j] = tj; e.cpos[j] = close;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int base = 0;
    for (int j0 = 0; j0 < nn; j0 += 64) {
      const int j = j0 + lane;
      const bool flag = j < nn && e.cpos[j] != 0;
      const unsigned long long mask = __ballot(flag);
      const int rank = base + __popcll(mask & ((1ull << lane) - 1ull));
      const bool in = flag && rank < geo.asel;
      if (j < nn) e.cpos[j] = in ? rank : -1;
      if (in) e.cl[rank] = j;
      base += __popcll(mask);
    }
    if (lane == 0) {
      e.nn = nn;
      e.nc = min(base, geo.asel);
    }
  }
  __syncthreads();
}

__device__ __forceinline__ float cosang(const GEnv &e, int jp, int jq) {
  return e.rh[3 * jp] * e.rh[3 * jq] + e.rh[3 * jp + 1] * e.rh[3 * jq + 1] + e.rh[3 * jp + 2] * e.rh[3 * jq + 2];
}

__device__ __forceinline__ size_t erow(const Buffers &b, int l, int i, int j) {
  return (((size_t)l * b.cap + i) * SEL + j) * EDIM;
}

// ------------------------------------------------------------------ angle offsets
__global__ void __launch_bounds__(256) k_angle_count(const double *__restrict__ X, const int *__restrict__ nlist,
                                                     const int *__restrict__ nnei, const Grid *__restrict__ grids,
                                                     int n, Geo geo, int64_t *__restrict__ aoff) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const Grid g = grids[0];
  const int nn = min(max(nnei[i], 0), SEL);
  int nc = 0;
  for (int j = 0; j < nn && nc < geo.asel; ++j) {
    int nj = nlist[(size_t)i * SEL + j];
    if (nj < 0 || nj >= n) continue;
    double d[3];
    for (int a = 0; a < 3; ++a) {
      double v = X[3 * nj + a] - X[3 * i + a];
      if (g.periodic) v -= g.L[a] * rint(v * g.invL[a]);
      d[a] = v;
    }
    nc += sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) < (double)geo.rca;
  }
  aoff[i + 1] = (int64_t)nc * (nc - 1);
  if (i == 0) aoff[0] = 0;
}

// Inclusive prefix of aoff[1 .. n] in one workgroup: each thread sums a contiguous run,
// the 1024 run totals are scanned, then each run is rewritten.
// The same workgroup also writes the total edge count (sum of nnei) to etot[0] and the
// number of angle-list edges of the atoms that have angles (sum of nc, from nc (nc - 1))
// to etot[1].
__global__ void __launch_bounds__(1024) k_angle_scan(int64_t *__restrict__ aoff, const int *__restrict__ nnei, int n,
                                                     int64_t *__restrict__ etot) {
  __shared__ int64_t part[1024];
  __shared__ int64_t epart[1024], cpart[1024];
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int b0 = 1 + t * per, b1 = min(n + 1, b0 + per);
  int64_t s = 0, se = 0, sc = 0;
  for (int k = b0; k < b1; ++k) {
    const int64_t cnt = aoff[k];
    s += cnt;
    se += min(max(nnei[k - 1], 0), SEL);
    int nc = 0;
    while ((int64_t)nc * (nc - 1) < cnt) ++nc;  // cnt = nc (nc - 1), nc <= 48 (atoms with angles)
    sc += nc;
  }
  part[t] = s;
  epart[t] = se;
  cpart[t] = sc;
  __syncthreads();
  if (t == 0) {
    int64_t tot = 0, totc = 0;
    for (int k = 0; k < 1024; ++k) {
      tot += epart[k];
      totc += cpart[k];
    }
    etot[0] = tot;
    etot[1] = totc;
  }
  for (int off = 1; off < 1024; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = t > 0 ? part[t - 1] : 0;
  for (int k = b0; k < b1; ++k) {
    run += aoff[k];
    aoff[k] = run;
  }
}

// The terms an angle's products take from its two edges depend on the edge alone:
// PQ[x] = [e_x[:32] Waa[32:64], e_x[:32] Waa[64:96], e_x[:32] Wea[32:64]] for every
// angle-list edge x (rows of E at stride lde, first 32 columns), computed once per
// layer instead of once per angle.  Each thread owns one of the 128 columns and holds
// its 32 weights in registers.  Ends synchronised.
constexpr int PQW = 2 * ADIM + EDIM;  // 128
__device__ void edge_terms(const float *__restrict__ Waa, const float *__restrict__ Wea, const float *E, int lde,
                           const int *cl, int nc, float *PQ) {
  const int c = threadIdx.x & (PQW - 1);
  float wc[ADIM];
#pragma unroll
  for (int k = 0; k < ADIM; ++k)
    wc[k] = c < ADIM ? Waa[(ADIM + k) * ADIM + c]
                     : (c < 2 * ADIM ? Waa[(2 * ADIM + k) * ADIM + c - ADIM] : Wea[(ADIM + k) * EDIM + c - 2 * ADIM]);
  for (int x = threadIdx.x >> 7; x < nc; x += NT / PQW) {
    const float *ex = E + (lde > 0 ? cl[x] * lde : x * ADIM);
    float v = 0.f;
#pragma unroll
    for (int k = 0; k < ADIM; ++k) v += ex[k] * wc[k];
    PQ[x * PQW + c] = v;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ forward
struct SmemF {
  GEnv env;
  float El[SEL * LDE] __attribute__((aligned(16)));  // e of the layer's input
  float Msg[ASEL * EDIM];                            // m_ip
  float PQ[ASEL * PQW];                              // per-edge terms of the angle products
  float slab[NWG][16 * LDF] __attribute__((aligned(16)));  // per-wave operand tiles
  float ni[NDIM] __attribute__((aligned(16))), xs[2 * NDIM], aggw[NWG][NDIM], nbias[EDIM];
  float y1[FWID], t2[FWID], dp[FWID];
};

// Stages 16 rows x 32 S floats into a slab: segment s (columns 32 s .. 32 s + 31) of
// row r is src(s, r, c4), c4 = 0..7 the float4 within the segment (zero for rows past
// the end).  Each lane moves two rows of one float4 column per segment; the reads of G
// segments are issued before their writes, so their latencies overlap.  s is a
// compile-time constant in every call of src (the loops are unrolled).
template <int S, int G, class Src>
__device__ __forceinline__ void stage(float *sl, int ld, const Src &src) {
  const int c4 = lane_id() & 7, r0 = lane_id() >> 3;
#pragma unroll
  for (int g0 = 0; g0 < S; g0 += G) {
    float4 v[G][2];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (g0 + g < S) v[g][h] = src(g0 + g, r0 + 8 * h, c4);
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (g0 + g < S) *reinterpret_cast<float4 *>(sl + (r0 + 8 * h) * ld + 32 * (g0 + g) + 4 * c4) = v[g][h];
  }
}

__device__ __forceinline__ float4 ld4(const float *p) { return *reinterpret_cast<const float4 *>(p); }

template <typename T>
__global__ void __launch_bounds__(NT) k_layer_fwd(Weights w, Buffers b, const double *__restrict__ X,
                                                  const int *__restrict__ types, const int *__restrict__ nlist,
                                                  const int *__restrict__ nnei, const Grid *__restrict__ grids,
                                                  int n, int layer, Geo geo, double *__restrict__ Ei,
                                                  const unsigned *__restrict__ flags) {
  __shared__ SmemF sm;
  const int i = blockIdx.x;
  if (i >= n || failed(flags)) return;
  const int tid = threadIdx.x, wv = wave_id(), ln = lane_id();
  const int l = layer;
  const float *Waa = w.Waa[l], *baa = w.baa[l], *Wea = w.Wea[l], *bea = w.bea[l];
  const float *Wee = w.Wee[l], *bee = w.bee[l], *Wnn = w.Wnn[l], *bnn = w.bnn[l];
  // the angle rows' parts of this layer's angle weights (the first 32 inputs), held by
  // every wave for all its tiles
  Frag<T, ADIM> fa[2];
  Frag<T, ADIM> fm[4];
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) fa[ct].load([&](int c, int k) { return Waa[k * ADIM + ct * 16 + c]; });
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) fm[ct].load([&](int c, int k) { return Wea[k * EDIM + ct * 16 + c]; });
  build_genv(sm.env, X, types, nlist, nnei, i, n, grids[0], geo);
  const GEnv &e = sm.env;
  const int nn = e.nn, nc = e.nc;

  if (l == 0) {
    for (int k = tid; k < nn * EDIM; k += NT) {
      const int j = k >> 6, c = k & 63;
      sm.El[j * LDE + c] = tanhf(e.s[j] * w.We0[c] + w.be0[c]);
    }
  } else {  // the input edges, all reads issued before the writes
    constexpr int NI = (SEL * EDIM / 4 + NT - 1) / NT;
    float4 v[NI];
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = tid + NT * it, j = k >> 4;
      if (j < nn) v[it] = ld4(b.ef + erow(b, l - 1, i, j) + 4 * (k & 15));
    }
#pragma unroll
    for (int it = 0; it < NI; ++it) {
      const int k = tid + NT * it, j = k >> 4;
      if (j < nn) *reinterpret_cast<float4 *>(sm.El + j * LDE + 4 * (k & 15)) = v[it];
    }
  }
  if (tid < NDIM)
    sm.ni[tid] = l == 0 ? w.TN[clamp_type(types[i]) * NDIM + tid] : b.nf[((size_t)(l - 1) * b.cap + i) * NDIM + tid];
  __syncthreads();
  if (tid < EDIM) {  // the centre's part of every edge update: bee + n_i Wee[0:64]
    float v = bee[tid];
    for (int k = 0; k < NDIM; ++k) v += sm.ni[k] * Wee[k * EDIM + tid];
    sm.nbias[tid] = v;
  }
  edge_terms(Waa, Wea, sm.El, LDE, e.cl, nc, sm.PQ);

  float *sl = sm.slab[wv];
  const float *rowA = sl + (ln & 15) * LDF;
  const int na = nc - 1;  // angles per row p
  const int64_t abase = b.aoff[i];
  // ---------------- angles and messages
  // A wave takes rows p = wv, wv + NWG, ... and the angles of each in pairs of tiles of
  // 16 (t0 .. t0 + 15 at slab columns 0 .. 31, t0 + 16 .. t0 + 31 at columns 32 .. 63),
  // whose product chains are independent and interleave; for l > 0 the input a of its
  // next pair is read while the current pair is processed.
  const int sc4 = ln & 7, sr0 = ln >> 3;  // the lane's float4 column and first row in a staged tile
  auto pair_in = [&](int p, int t0, float4 (&v)[4]) {
    const float *ap = b.af + ((size_t)(l - 1) * b.acap + abase + (int64_t)p * na) * ADIM;
#pragma unroll
    for (int h = 0; h < 4; ++h) {
      const int t = t0 + 16 * (h >> 1) + sr0 + 8 * (h & 1);
      v[h] = t < na ? ld4(ap + (size_t)t * ADIM + 4 * sc4) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  const Shift second{ADIM};
  float4 nxt[4];
  if (l > 0 && wv < nc && na > 0) pair_in(wv, 0, nxt);
  for (int p = wv; p < nc; p += NWG) {
    float mr[4] = {0.f, 0.f, 0.f, 0.f};
    const int jp = e.cl[p];
    for (int t0 = 0; t0 < na; t0 += 32) {
      // a of the pair's 32 angles; the edge terms come from PQ
      if (l > 0) {
        const float4 cur[4] = {nxt[0], nxt[1], nxt[2], nxt[3]};
        const int pn = t0 + 32 < na ? p : p + NWG, tn = t0 + 32 < na ? t0 + 32 : 0;
        if (pn < nc) pair_in(pn, tn, nxt);
#pragma unroll
        for (int h = 0; h < 4; ++h)
          *reinterpret_cast<float4 *>(sl + (sr0 + 8 * (h & 1)) * LDF + ADIM * (h >> 1) + 4 * sc4) = cur[h];
      } else stage<2, 2>(sl, LDF, [&](int sg, int r, int c4) -> float4 {
        const int t = t0 + 16 * sg + r;
        if (t >= na) return make_float4(0.f, 0.f, 0.f, 0.f);
        const float cs = cosang(e, jp, e.cl[t + (t >= p)]);
        float4 v;
        v.x = tanhf(cs * w.Wa0[4 * c4] + w.ba0[4 * c4]);
        v.y = tanhf(cs * w.Wa0[4 * c4 + 1] + w.ba0[4 * c4 + 1]);
        v.z = tanhf(cs * w.Wa0[4 * c4 + 2] + w.ba0[4 * c4 + 2]);
        v.w = tanhf(cs * w.Wa0[4 * c4 + 3] + w.ba0[4 * c4 + 3]);
        return v;
      });
      wave_sync();
      int qrow[2][4];
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int t = t0 + 16 * h + acc_row(ii);
          qrow[h][ii] = t < na ? t + (t >= p) : p;  // rows past the end read a valid row, and are not used
        }
      f4 aa[2][2] = {};
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        fa[ct].mma(aa[0][ct], rowA, Ident());
        fa[ct].mma(aa[1][ct], rowA, second);
      }
      wave_sync();
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            const int r = acc_row(ii), c = ct * 16 + acc_col(), t = t0 + 16 * h + r;
            const float z = aa[h][ct][ii] + baa[c] + sm.PQ[p * PQW + c] + sm.PQ[qrow[h][ii] * PQW + ADIM + c];
            const float a1 = sl[r * LDF + ADIM * h + c] + act<T>(z);
            sl[r * LDF + ADIM * h + c] = a1;
            if (t < na) b.af[((size_t)l * b.acap + abase + (int64_t)p * na + t) * ADIM + c] = a1;
          }
      wave_sync();
      f4 am[2][4] = {};
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        fm[ct].mma(am[0][ct], rowA, Ident());
        fm[ct].mma(am[1][ct], rowA, second);
      }
#pragma unroll
      for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int t = t0 + 16 * h + acc_row(ii);
          const float wr = t < na ? e.swa[jp] * e.swa[e.cl[qrow[h][ii]]] * geo.inv_asel : 0.f;
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) {
            const int c = ct * 16 + acc_col();
            mr[ct] += wr * act<T>(am[h][ct][ii] + bea[c] + sm.PQ[qrow[h][ii] * PQW + 2 * ADIM + c]);
          }
        }
      wave_sync();
    }
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      const float v = sum_cols4(mr[ct]);
      if (ln < 16) sm.Msg[p * EDIM + ct * 16 + ln] = v;
    }
  }
  __syncthreads();

  // ---------------- edges
  float aw[4] = {0.f, 0.f, 0.f, 0.f};
  for (int j0 = wv * 16; j0 < nn; j0 += NWG * 16) {
    // [n_i, n_j, e_ij]
    stage<4, 2>(sl, LDF, [&](int sg, int r, int c4) -> float4 {  // [n_j, e_ij]; n_i enters through nbias
      const int j = j0 + r;
      if (j >= nn) return make_float4(0.f, 0.f, 0.f, 0.f);
      const int c = 32 * (sg & 1) + 4 * c4;
      if (sg < 2)
        return l == 0 ? ld4(w.TN + e.tj[j] * NDIM + c) : ld4(b.nf + ((size_t)(l - 1) * b.cap + e.jn[j]) * NDIM + c);
      return ld4(sm.El + j * LDE + c);
    });
    wave_sync();
    f4 ae[4] = {};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      opaque();  // load each column tile's weights here, not once for all tiles
      Frag<T, 128> f;
      f.load([&](int c, int k) { return Wee[(NDIM + k) * EDIM + ct * 16 + c]; });
      f.mma(ae[ct], rowA, Ident());
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = j0 + acc_row(ii);
      if (j < nn) {
        const int cp = e.cpos[j];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int c = ct * 16 + acc_col();
          const float e1 =
              sm.El[j * LDE + c] + act<T>(ae[ct][ii] + sm.nbias[c]) + (cp >= 0 ? sm.Msg[cp * EDIM + c] : 0.f);
          b.ef[erow(b, l, i, j) + c] = e1;
          aw[ct] += e.swe[j] * e1;
        }
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const float v = sum_cols4(aw[ct]);
    if (ln < 16) sm.aggw[wv][ct * 16 + ln] = v;
  }
  __syncthreads();

  // ---------------- node
  if (tid < NDIM) {
    sm.xs[tid] = sm.ni[tid];
    sm.xs[NDIM + tid] = (sm.aggw[0][tid] + sm.aggw[1][tid] + sm.aggw[2][tid] + sm.aggw[3][tid]) * geo.inv_sel;
  }
  __syncthreads();
  float n1 = 0.f;
  if (tid < NDIM) {
    float z = bnn[tid];
    for (int k = 0; k < 2 * NDIM; ++k) z += sm.xs[k] * Wnn[k * NDIM + tid];
    n1 = sm.ni[tid] + tanhf(z);
    if (l < NLAYER - 1) b.nf[((size_t)l * b.cap + i) * NDIM + tid] = n1;
  }
  if (l < NLAYER - 1) return;

  // ---------------- fitting net, E_i and dE/dn_i
  __syncthreads();
  if (tid < NDIM) sm.ni[tid] = n1;
  __syncthreads();
  if (tid < FWID) {
    float z = w.d1[tid];
    for (int k = 0; k < NDIM; ++k) z += sm.ni[k] * w.G1[k * FWID + tid];
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
  if (tid < NDIM) {
    float dn = 0.f;
    for (int k = 0; k < FWID; ++k) dn += sm.dp[k] * w.G1[tid * FWID + k];
    b.dnl[(size_t)i * NDIM + tid] = dn;
  }
}

// ------------------------------------------------------------------ backward
struct SmemB {
  GEnv env;
  float DEl[SEL * EDIM];      // dE/de of this layer's input edges
  float DM[ASEL * EDIM];      // dE/dm_ip
  float Ec[ASEL * ADIM] __attribute__((aligned(16)));  // e[:32] of the angle-list edges
  float slab[NWG][16 * LDB] __attribute__((aligned(16)));
  float Qacc[NWG][ASEL * QLD];  // per-wave sums of the terms of edge q
  float Pacc[ASEL * QLD];       // terms of edge p from its own angle row
  float PQ[ASEL * PQW];         // per-edge terms of the angle products
  float dn[NDIM], ni[NDIM] __attribute__((aligned(16))), xs[2 * NDIM], dagg[NDIM], dnsum[NWG][NDIM], zz[NDIM],
      nbias[EDIM];
  int slot[SEL];
};

template <typename T>
__global__ void __launch_bounds__(NT) k_layer_bwd(Weights w, Buffers b, const double *__restrict__ X,
                                                  const int *__restrict__ types, const int *__restrict__ nlist,
                                                  const int *__restrict__ nnei, const Grid *__restrict__ grids,
                                                  int n, int layer, Geo geo, float4 *__restrict__ gout,
                                                  const unsigned *__restrict__ flags) {
  __shared__ SmemB sm;
  const int i = blockIdx.x;
  if (i >= n || failed(flags)) return;
  const int tid = threadIdx.x, wv = wave_id(), ln = lane_id();
  build_genv(sm.env, X, types, nlist, nnei, i, n, grids[0], geo);
  const GEnv &e = sm.env;
  const int nn = e.nn, nc = e.nc, l = layer;
  const float *Waa = w.Waa[l], *baa = w.baa[l], *Wea = w.Wea[l], *bea = w.bea[l];
  const float *Wee = w.Wee[l], *bee = w.bee[l], *Wnn = w.Wnn[l], *bnn = w.bnn[l];
  const bool top = l == NLAYER - 1;

  // ---------------- dE/dn_i after this layer: own part + the neighbours' edge parts
  if (!top)
    for (int j = tid; j < nn; j += NT) sm.slot[j] = b.slot[(size_t)i * SEL + j];
  for (int k = tid; k < nc * ADIM; k += NT) {
    const int p = k >> 5, c = k & 31, j = e.cl[p];
    sm.Ec[k] = l == 0 ? tanhf(e.s[j] * w.We0[c] + w.be0[c]) : b.ef[erow(b, l - 1, i, j) + c];
  }
  if (tid < NDIM)
    sm.ni[tid] = l == 0 ? w.TN[clamp_type(types[i]) * NDIM + tid] : b.nf[((size_t)(l - 1) * b.cap + i) * NDIM + tid];
  __syncthreads();
  {
    // each wave sums the rows j = wave, wave + 4, ... in list order (the neighbours' edge
    // parts of dE/dn_i, and agg from the stored output edges); waves combine in order
    float dn = 0.f, agg = 0.f;
    const float *src = b.dnj + (size_t)((l + 1) & 1) * b.cap * SEL * EDIM;
#pragma unroll 8
    for (int j = wv; j < nn; j += NWG) {
      if (!top) {  // branch-free in j (a missing slot reads row 0 and adds 0), so the loads overlap
        const int sj = sm.slot[j];
        const float x = src[((size_t)e.jn[j] * SEL + max(sj, 0)) * EDIM + ln];
        dn += sj >= 0 ? x : 0.f;
      }
      agg += e.swe[j] * b.ef[erow(b, l, i, j) + ln];
    }
    sm.dnsum[wv][ln] = dn;
    sm.Pacc[wv * EDIM + ln] = agg;
  }
  __syncthreads();
  if (tid < NDIM) {
    float dn = b.dnl[(size_t)i * NDIM + tid], agg = 0.f;
    for (int u = 0; u < NWG; ++u) {
      dn += sm.dnsum[u][tid];
      agg += sm.Pacc[u * EDIM + tid];
    }
    sm.dn[tid] = dn;
    sm.xs[tid] = sm.ni[tid];
    sm.xs[NDIM + tid] = agg * geo.inv_sel;
  }
  __syncthreads();
  // ---------------- node backward (and the centre's part of every edge update)
  if (tid < EDIM) {
    float v = bee[tid];
    for (int k = 0; k < NDIM; ++k) v += sm.ni[k] * Wee[k * EDIM + tid];
    sm.nbias[tid] = v;
  }
  if (tid < NDIM) {
    float z = bnn[tid];
    for (int k = 0; k < 2 * NDIM; ++k) z += sm.xs[k] * Wnn[k * NDIM + tid];
    const float t = tanhf(z);
    sm.zz[tid] = sm.dn[tid] * (1.f - t * t);
  }
  __syncthreads();
  if (tid < NDIM) {
    float dni = sm.dn[tid], dg = 0.f;
    for (int k = 0; k < NDIM; ++k) {
      dni += sm.zz[k] * Wnn[tid * NDIM + k];
      dg += sm.zz[k] * Wnn[(NDIM + tid) * NDIM + k];
    }
    sm.dn[tid] = dni;  // now dE/dn_i of this layer's input, without the edge terms
    sm.dagg[tid] = dg * geo.inv_sel;
  }
  __syncthreads();

  float *sl = sm.slab[wv];
  const float *rowA = sl + (ln & 15) * LDB;
  // ---------------- edges
  float dns[4] = {0.f, 0.f, 0.f, 0.f};
  for (int j0 = wv * 16; j0 < nn; j0 += NWG * 16) {
    stage<4, 2>(sl, LDB, [&](int sg, int r, int c4) -> float4 {  // [n_j, e_ij]; n_i enters through nbias
      const int j = j0 + r;
      if (j >= nn) return make_float4(0.f, 0.f, 0.f, 0.f);
      const int c = 32 * (sg & 1) + 4 * c4;
      if (sg < 2)
        return l == 0 ? ld4(w.TN + e.tj[j] * NDIM + c) : ld4(b.nf + ((size_t)(l - 1) * b.cap + e.jn[j]) * NDIM + c);
      if (l > 0) return ld4(b.ef + erow(b, l - 1, i, j) + c);
      float4 v;
      v.x = tanhf(e.s[j] * w.We0[c] + w.be0[c]);
      v.y = tanhf(e.s[j] * w.We0[c + 1] + w.be0[c + 1]);
      v.z = tanhf(e.s[j] * w.We0[c + 2] + w.be0[c + 2]);
      v.w = tanhf(e.s[j] * w.We0[c + 3] + w.be0[c + 3]);
      return v;
    });
    float pde[4][4], pef[4][4];  // dE/de and e of the layer's output, read ahead of their use
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = j0 + acc_row(ii);
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int c = ct * 16 + acc_col();
        pde[ct][ii] = (!top && j < nn) ? b.de[((size_t)i * SEL + j) * EDIM + c] : 0.f;
        pef[ct][ii] = j < nn ? b.ef[erow(b, l, i, j) + c] : 0.f;
      }
    }
    wave_sync();
    f4 ae[4] = {};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      if constexpr (sizeof(T) == 2) {
        opaque();  // load each column tile's weights here, not once for all tiles
        Frag<T, 128> f;
        f.load([&](int c, int k) { return Wee[(NDIM + k) * EDIM + ct * 16 + c]; });
        f.mma(ae[ct], rowA, Ident());
      } else {  // float32 operands: 32 more registers per lane would spill; read W as it goes
        Mma<T>::tile(ae[ct], [&](int r, int k) { return sl[r * LDB + k]; },
                     [&](int c, int k) { return Wee[(NDIM + k) * EDIM + ct * 16 + c]; }, 128);
      }
    }
    wave_sync();
    float de1[4][4], rs[4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int r = acc_row(ii), j = j0 + r;
      const bool ok = j < nn;
      rs[ii] = 0.f;
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) {
        const int c = ct * 16 + acc_col();
        float d = 0.f, dz = 0.f;
        if (ok) {
          d = pde[ct][ii] + e.swe[j] * sm.dagg[c];
          rs[ii] += pef[ct][ii] * sm.dagg[c];
          const float t = act<T>(ae[ct][ii] + sm.nbias[c]);
          dz = d * (1.f - t * t);
        }
        de1[ct][ii] = d;
        sl[r * LDB + c] = dz;  // dz_e over the n_j columns (the products that read them are done)
        dns[ct] += dz;
      }
      rs[ii] = sum16(rs[ii]);
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = j0 + acc_row(ii);
      if (j < nn && acc_col() == 0) {
        float *g = b.gs + ((size_t)i * SEL + j) * 2;
        g[0] = top ? rs[ii] : g[0] + rs[ii];
      }
    }
    wave_sync();
    if (l > 0) {  // edge (i, j)'s part of dE/dn_j
      float *dst = b.dnj + (size_t)(l & 1) * b.cap * SEL * EDIM;
      f4 an[4] = {};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
        opaque();
        Frag<T, 64> f;
        f.load([&](int c, int k) { return Wee[(NDIM + ct * 16 + c) * EDIM + k]; });
        f.mma(an[ct], rowA, Ident());
      }
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int j = j0 + acc_row(ii);
        if (j < nn)
#pragma unroll
          for (int ct = 0; ct < 4; ++ct) dst[((size_t)i * SEL + j) * EDIM + ct * 16 + acc_col()] = an[ct][ii];
      }
    }
    f4 ad[4] = {};
#pragma unroll
    for (int ct = 0; ct < 4; ++ct) {
      opaque();
      Frag<T, 64> f;
      f.load([&](int c, int k) { return Wee[(2 * NDIM + ct * 16 + c) * EDIM + k]; });
      f.mma(ad[ct], rowA, Ident());
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = j0 + acc_row(ii);
      if (j < nn) {
        const int cp = e.cpos[j];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int c = ct * 16 + acc_col();
          sm.DEl[j * EDIM + c] = de1[ct][ii] + ad[ct][ii];
          if (cp >= 0) sm.DM[cp * EDIM + c] = de1[ct][ii];
        }
      }
    }
    wave_sync();
  }
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) {
    const float v = sum_cols4(dns[ct]);
    if (ln < 16) sm.dnsum[wv][ct * 16 + ln] = v;
  }
  float *Q = sm.Qacc[wv];
  for (int k = ln; k < ASEL * QLD; k += 64) Q[k] = 0.f;
  __syncthreads();

  // ---------------- angles
  // this layer's angle weights in registers: forward recomputation (Wea, Waa) and the
  // transposed products (Wea^T, Waa^T, and [Wea; Waa]^T for the terms of edge q)
  // ([Wea; Waa]^T stays in registers only for bf16 operands: as float32 it would not fit
  // beside the rest and is reloaded for each tile)
  constexpr bool FV_RESIDENT = sizeof(T) == 2;
  auto wv_q = [&](int ct) {
    return [=](int c, int k) {
      return k < 64 ? Wea[(32 + ct * 16 + c) * EDIM + k] : Waa[(64 + ct * 16 + c) * ADIM + k - 64];
    };
  };
  Frag<T, ADIM> fm[4], fa[2];  // the angle rows' parts (first 32 inputs) of Wea, Waa
  Frag<T, 64> fx[2];
  Frag<T, 96> fv[FV_RESIDENT ? 2 : 1];
  Frag<T, 32> fy[2];
#pragma unroll
  for (int ct = 0; ct < 4; ++ct) fm[ct].load([&](int c, int k) { return Wea[k * EDIM + ct * 16 + c]; });
#pragma unroll
  for (int ct = 0; ct < 2; ++ct) {
    fa[ct].load([&](int c, int k) { return Waa[k * ADIM + ct * 16 + c]; });
    fx[ct].load([&](int c, int k) { return Wea[(ct * 16 + c) * EDIM + k]; });
    fy[ct].load([&](int c, int k) { return Waa[(ct * 16 + c) * ADIM + k]; });
    if constexpr (FV_RESIDENT) fv[ct].load(wv_q(ct));
  }
  edge_terms(Waa, Wea, sm.Ec, 0, e.cl, nc, sm.PQ);
  const int na = nc - 1;
  const int64_t abase = b.aoff[i];
  for (int p = wv; p < nc; p += NWG) {
    const int jp = e.cl[p];
    float S[2] = {0.f, 0.f};      // column sums of dz_a
    float sp = 0.f, hp[3] = {0.f, 0.f, 0.f};  // dE/dsw_a(r_ip), dE/drhat_ip from this row
    const float *a1p = b.af + ((size_t)l * b.acap + abase + (int64_t)p * na) * ADIM;
    const float *a0p = b.af + ((size_t)(l > 0 ? l - 1 : 0) * b.acap + abase + (int64_t)p * na) * ADIM;
    for (int t0 = 0; t0 < na; t0 += 16) {
      // [a', a] of the tile's 16 angles; the edge terms come from PQ
      stage<2, 2>(sl, LDB, [&](int sg, int r, int c4) -> float4 {
        const int t = t0 + r;
        if (t >= na) return make_float4(0.f, 0.f, 0.f, 0.f);
        if (sg == 0) return ld4(a1p + (size_t)t * ADIM + 4 * c4);
        if (l > 0) return ld4(a0p + (size_t)t * ADIM + 4 * c4);
        const float cs = cosang(e, jp, e.cl[t + (t >= p)]);
        const int c = 4 * c4;
        float4 v;
        v.x = tanhf(cs * w.Wa0[c] + w.ba0[c]);
        v.y = tanhf(cs * w.Wa0[c + 1] + w.ba0[c + 1]);
        v.z = tanhf(cs * w.Wa0[c + 2] + w.ba0[c + 2]);
        v.w = tanhf(cs * w.Wa0[c + 3] + w.ba0[c + 3]);
        return v;
      });
      float dap[2][4];  // dE/da of the layer's output, read ahead of its use
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int t = t0 + acc_row(ii);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
          dap[ct][ii] = (!top && t < na) ? b.da[(size_t)(abase + (int64_t)p * na + t) * ADIM + ct * 16 + acc_col()] : 0.f;
      }
      wave_sync();
      f4 am[4] = {}, aa[2] = {};
#pragma unroll
      for (int ct = 0; ct < 4; ++ct) fm[ct].mma(am[ct], rowA, Ident());  // a' (columns 0..31)
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) fa[ct].mma(aa[ct], rowA, [](int k) { return ADIM + k; });  // a (32..63)
      float dwa[4], ta[2][4];
      int qv[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = acc_row(ii), t = t0 + r;
        qv[ii] = t < na ? t + (t >= p) : -1;
        const int qr = qv[ii] >= 0 ? qv[ii] : p;  // rows past the end read a valid row, unused
        const float wr = qv[ii] >= 0 ? e.swa[jp] * e.swa[e.cl[qv[ii]]] * geo.inv_asel : 0.f;
        float d = 0.f;
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
          const int c = ct * 16 + acc_col();
          const float tm = act<T>(am[ct][ii] + bea[c] + sm.PQ[qr * PQW + 2 * ADIM + c]);
          const float dm = qv[ii] >= 0 ? sm.DM[p * EDIM + c] : 0.f;
          d += dm * tm;
          sl[r * LDB + 64 + c] = wr * dm * (1.f - tm * tm);  // dz_m
        }
        dwa[ii] = sum16(d);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const int c = ct * 16 + acc_col();
          ta[ct][ii] = act<T>(aa[ct][ii] + baa[c] + sm.PQ[p * PQW + c] + sm.PQ[qr * PQW + ADIM + c]);
        }
      }
      wave_sync();
      f4 ax[2] = {};
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) fx[ct].mma(ax[ct], rowA, [](int k) { return 64 + k; });
      float da1[2][4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = acc_row(ii);
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const int c = ct * 16 + acc_col();
          float d = 0.f;
          if (qv[ii] >= 0) d = dap[ct][ii] + ax[ct][ii];
          da1[ct][ii] = d;
          const float dz = d * (1.f - ta[ct][ii] * ta[ct][ii]);
          sl[r * LDB + 128 + c] = dz;  // dz_a
          S[ct] += dz;
        }
      }
      wave_sync();
      f4 ay[2] = {}, av[2] = {};
#pragma unroll
      for (int ct = 0; ct < 2; ++ct) {
        fy[ct].mma(ay[ct], rowA, [](int k) { return 128 + k; });
        if constexpr (FV_RESIDENT) {
          fv[ct].mma(av[ct], rowA, [](int k) { return 64 + k; });
        } else {
          opaque();
          Frag<T, 96> f;
          f.load(wv_q(ct));
          f.mma(av[ct], rowA, [](int k) { return 64 + k; });
        }
      }
      float dc[4];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = acc_row(ii);
        float d = 0.f;
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
          const int c = ct * 16 + acc_col();
          const float dal = da1[ct][ii] + ay[ct][ii];
          if (qv[ii] >= 0) {
            if (l > 0) b.da[(size_t)(abase + (int64_t)p * na + t0 + r) * ADIM + c] = dal;
            Q[qv[ii] * QLD + c] += av[ct][ii];
          }
          if (l == 0) {
            const float a0 = sl[r * LDB + ADIM + c];
            d += dal * (1.f - a0 * a0) * w.Wa0[c];
          }
        }
        dc[ii] = l == 0 ? sum16(d) : 0.f;
      }
      if (acc_col() == 0)
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int q = qv[ii];
          if (q < 0) continue;
          const int jq = e.cl[q];
          Q[q * QLD + 32] += dwa[ii] * e.swa[jp] * geo.inv_asel;
          sp += dwa[ii] * e.swa[jq] * geo.inv_asel;
          if (l == 0)
            for (int a = 0; a < 3; ++a) {
              Q[q * QLD + 33 + a] += dc[ii] * e.rh[3 * jp + a];
              hp[a] += dc[ii] * e.rh[3 * jq + a];
            }
        }
      wave_sync();
    }
    // row p: its own edge's terms
    S[0] = sum_cols4(S[0]);
    S[1] = sum_cols4(S[1]);
    sp = wave_sum64(sp);
    for (int a = 0; a < 3; ++a) hp[a] = wave_sum64(hp[a]);
    if (ln < 16) {
      sl[ln] = S[0];
      sl[16 + ln] = S[1];
    }
    wave_sync();
    if (ln < ADIM) {
      float v = 0.f;
      for (int k = 0; k < ADIM; ++k) v += sl[k] * Waa[(ADIM + ln) * ADIM + k];
      sm.Pacc[p * QLD + ln] = v;
    }
    if (ln == 0) {
      sm.Pacc[p * QLD + 32] = sp;
      for (int a = 0; a < 3; ++a) sm.Pacc[p * QLD + 33 + a] = hp[a];
    }
    wave_sync();
  }
  __syncthreads();

  // ---------------- the angle terms of each angle-list edge, in wave order
  for (int k = tid; k < nc * QLD; k += NT) {
    const int q = k / QLD, c = k % QLD;
    float v = sm.Pacc[k];
    for (int u = 0; u < NWG; ++u) v += sm.Qacc[u][k];
    if (c < ADIM) sm.DEl[e.cl[q] * EDIM + c] += v;
    else sm.Pacc[k] = v;  // sw_a and rhat terms, complete
  }
  if (tid < NDIM) {
    float s = 0.f;
    for (int u = 0; u < NWG; ++u) s += sm.dnsum[u][tid];
    sm.zz[tid] = s;
  }
  __syncthreads();
  for (int j = tid; j < nn; j += NT) {
    const int cp = e.cpos[j];
    float *g = b.gs + ((size_t)i * SEL + j) * 2;
    const float dsa = cp >= 0 ? sm.Pacc[cp * QLD + 32] : 0.f;
    g[1] = top ? dsa : g[1] + dsa;
  }
  if (l > 0) {
    for (int k = tid; k < nn * EDIM; k += NT) b.de[(size_t)i * SEL * EDIM + k] = sm.DEl[k];
    if (tid < NDIM) {
      float v = sm.dn[tid];
      for (int k = 0; k < NDIM; ++k) v += sm.zz[k] * Wee[tid * EDIM + k];
      b.dnl[(size_t)i * NDIM + tid] = v;
    }
    return;
  }
  __syncthreads();
  // ---------------- layer 0: g_ij = dE/dDelta_ij
  for (int j = tid; j < nn; j += NT) {
    float ds = 0.f;
    for (int c = 0; c < EDIM; ++c) {
      const float e0 = tanhf(e.s[j] * w.We0[c] + w.be0[c]);
      ds += sm.DEl[j * EDIM + c] * (1.f - e0 * e0) * w.We0[c];
    }
    const float *g2 = b.gs + ((size_t)i * SEL + j) * 2;
    const int cp = e.cpos[j];
    const float rr = e.r[j], sw = e.swe[j];
    const float dr = ds * (e.dswe[j] / rr - sw / (rr * rr)) + g2[0] * e.dswe[j] + g2[1] * e.dswa[j];
    const float hx = e.rh[3 * j], hy = e.rh[3 * j + 1], hz = e.rh[3 * j + 2];
    float gx = 0.f, gy = 0.f, gz = 0.f;
    if (cp >= 0) {
      gx = sm.Pacc[cp * QLD + 33];
      gy = sm.Pacc[cp * QLD + 34];
      gz = sm.Pacc[cp * QLD + 35];
    }
    const float proj = gx * hx + gy * hy + gz * hz;
    gout[(size_t)i * SEL + j] = make_float4((gx - proj * hx) / rr + dr * hx, (gy - proj * hy) / rr + dr * hy,
                                            (gz - proj * hz) / rr + dr * hz, 0.f);
  }
}

}  // namespace

void launch_angle_offsets(const Buffers &b, const Workspace &ws, const double *coords, int n, const Geo &geo,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_angle_count, dim3((n + 255) / 256), dim3(256), 0, st, coords, ws.nlist, ws.nnei, ws.grids, n,
                     geo, b.aoff);
  hipLaunchKernelGGL(k_angle_scan, dim3(1), dim3(1024), 0, st, b.aoff, ws.nnei, n, b.aoff + b.cap + 1);
}

template <typename T>
void launch_layer_fwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, double *Ei, hipStream_t st) {
  hipLaunchKernelGGL(k_layer_fwd<T>, dim3(n), dim3(NT), 0, st, w, b, coords, types, ws.nlist, ws.nnei, ws.grids, n,
                     layer, geo, Ei, ws.flags);
}

template <typename T>
void launch_layer_bwd(const Weights &w, const Buffers &b, const Workspace &ws, const double *coords,
                      const int *types, int n, int layer, const Geo &geo, hipStream_t st) {
  hipLaunchKernelGGL(k_layer_bwd<T>, dim3(n), dim3(NT), 0, st, w, b, coords, types, ws.nlist, ws.nnei, ws.grids, n,
                     layer, geo, ws.g, ws.flags);
}

template void launch_layer_fwd<float>(const Weights &, const Buffers &, const Workspace &, const double *,
                                      const int *, int, int, const Geo &, double *, hipStream_t);
template void launch_layer_fwd<bf16_t>(const Weights &, const Buffers &, const Workspace &, const double *,
                                       const int *, int, int, const Geo &, double *, hipStream_t);
template void launch_layer_bwd<float>(const Weights &, const Buffers &, const Workspace &, const double *,
                                      const int *, int, int, const Geo &, hipStream_t);
template void launch_layer_bwd<bf16_t>(const Weights &, const Buffers &, const Workspace &, const double *,
                                       const int *, int, int, const Geo &, hipStream_t);

}  // namespace gnn
}  // namespace dp
