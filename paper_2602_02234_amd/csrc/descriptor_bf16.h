// Shared parts of the bfloat16 descriptor kernels (gfx950 MFMA, fp32 accumulation):
// the trimmed per-atom environment, the MFMA tile products, and one attention layer
// for a wave's row blocks.  Included by descriptor_bf16.hip (forward) and
// descriptor_bf16_bwd.hip (backward); everything here has internal linkage.
//
// Same model as descriptor.hip (environment, type-embedded embedding net, two
// switch-weighted gated self-attention layers with a residual LayerNorm update,
// descriptor T = G^T Rt / sel, D = T T_<16^T), organised for throughput:
//
//  * every wave owns whole 16-token row blocks and carries them through a layer
//    (U = G Wqk, S = U G^T, softmax, H = A G, Y = H Wvo, LayerNorm) in registers,
//    so a layer needs two workgroup barriers instead of one per product;
//  * the representation G lives in LDS twice as bf16, token-major (Gb) and
//    feature-major (GbT), so that every MFMA fragment -- whichever index is the
//    reduction index -- is one 16-byte load; the fp32 master copy of the wave's
//    own rows stays in registers (residual and LayerNorm in fp32);
//  * the attention weights are read from global memory (L2-resident), pre-padded and
//    in MFMA fragment order, so a wave's fragment load is 1 KB of whole cache lines;
//    the small embedding weights are staged in LDS;
//  * feature width 100 is padded to 112 and contracted as 3 x 32 + 16 along k.
//
// lane() is the lane index.  A translation unit that defines DP_BF16_OPAQUE_LANE
// before including this header gets it through an empty asm statement, so that the
// compiler recomputes lane-derived addresses at each use instead of keeping them
// live (and spilling them) across the whole kernel.
#pragma once
#include "dp_env.h"

namespace dp {
namespace {

// Per-atom environment of the bfloat16 kernels (as Env, trimmed to what they read, so
// that a 7-wave backward workgroup fits in LDS): s = sw/r, sw, r, rhat; the neighbour's
// type as a byte.  Padded tokens (j >= n) have s = sw = 0, r = 1, rhat = 0.
struct EnvB {
  float s[NPMAX], sw[NPMAX], r[NPMAX];
  float rh[NPMAX * 3];
  unsigned char tj[NPMAX];
};

__device__ inline void build_envb(EnvB &e, const double *__restrict__ X, const int *__restrict__ types,
                                  const int *__restrict__ nlist, int i, int n, int natoms, const Grid &g, float rc,
                                  float rcs) {
  for (int j = threadIdx.x; j < NPMAX; j += blockDim.x) {
    float s = 0.f, sw = 0.f, r = 1.f, hx = 0.f, hy = 0.f, hz = 0.f;
    int tj = 0;
    if (j < n) {
      int nj = nlist[(size_t)i * SEL + j];
      if (nj < 0 || nj >= natoms) nj = i;  // never read outside the coordinate array
      tj = clamp_type(types[nj]);
      double d[3];
      for (int a = 0; a < 3; ++a) {
        double v = X[3 * nj + a] - X[3 * i + a];
        if (g.periodic) v -= g.L[a] * rint(v * g.invL[a]);
        d[a] = v;
      }
      const float dx = (float)d[0], dy = (float)d[1], dz = (float)d[2];
      r = sqrtf(dx * dx + dy * dy + dz * dz);
      const float u = (r - rcs) / (rc - rcs);
      if (r < rcs) sw = 1.f;
      else if (r < rc) sw = u * u * u * (-6.f * u * u + 15.f * u - 10.f) + 1.f;
      s = sw / r;
      hx = dx / r; hy = dy / r; hz = dz / r;
    }
    e.s[j] = s; e.sw[j] = sw; e.r[j] = r;
    e.rh[3 * j] = hx; e.rh[3 * j + 1] = hy; e.rh[3 * j + 2] = hz;
    e.tj[j] = (unsigned char)tj;
  }
}

// g = dE_i/dDelta_ij of token j from the gradients reaching s (ds_emb, through Rt),
// rhat (drh, through Rt and the gate) and sw (dswa, through the softmax weights); the
// switch derivative is formed here from r.
__device__ __forceinline__ float4 pair_gradient_b(const EnvB &e, int j, float ds_emb, const float *dRt,
                                                  const float *drh, float dswa, float rc, float rcs) {
  const float s = e.s[j], sw = e.sw[j], rr = e.r[j];
  const float hx = e.rh[3 * j], hy = e.rh[3 * j + 1], hz = e.rh[3 * j + 2];
  const float u = (rr - rcs) / (rc - rcs);
  const float dsw = (rr >= rcs && rr < rc) ? -30.f * u * u * (1.f - u) * (1.f - u) / (rc - rcs) : 0.f;
  const float ds = ds_emb + dRt[0] + dRt[1] * hx + dRt[2] * hy + dRt[3] * hz;
  const float gx = drh[0] + s * dRt[1];
  const float gy = drh[1] + s * dRt[2];
  const float gz = drh[2] + s * dRt[3];
  const float dswt = dswa + ds / rr;
  const float dr = -ds * sw / (rr * rr) + dswt * dsw;
  const float proj = gx * hx + gy * hy + gz * hz;
  return make_float4((gx - proj * hx) / rr + dr * hx, (gy - proj * hy) / rr + dr * hy, (gz - proj * hz) / rr + dr * hz,
                     0.f);
}

#ifdef DP_BF16_OPAQUE_LANE
__device__ __forceinline__ int lane() {
  int l = lane_id();
  asm volatile("" : "+v"(l));
  return l;
}
#else
__device__ __forceinline__ int lane() { return lane_id(); }
#endif

constexpr int KM = 112;   // padded feature width
constexpr int LDK = 120;  // stride (elements) of [token][feature] bf16 arrays
constexpr int LDT = 136;  // stride of [feature or row][token] bf16 arrays (tokens padded to 128)
constexpr int NWF = 8;    // waves per workgroup, forward
constexpr int SPLIT_NB = 7;  // atoms with up to this many row blocks go to the 7-wave backward instance
typedef short s4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf8 ld8(const bf16_t *p) { return *(const bf8 *)p; }
__device__ __forceinline__ s4 ld4(const bf16_t *p) { return *(const s4 *)p; }
__device__ __forceinline__ short bfbits(float x) {
  const bf16_t b = (bf16_t)x;
  return *(const short *)&b;
}
// Exponential and tanh from the hardware base-2 exponential (v_exp_f32) and reciprocal:
// relative error a few 1e-7, far below the bfloat16 rounding of the products they feed.
__device__ __forceinline__ float fexp(float x) { return __expf(x); }
__device__ __forceinline__ float ftanh(float x) {
  const float t = __expf(-2.f * fabsf(x));
  return copysignf((1.f - t) * __builtin_amdgcn_rcpf(1.f + t), x);
}

// Orders this wave's LDS accesses across a point (the wave reuses its staging buffer):
// the wave's outstanding LDS operations are drained and no instruction is moved across
// the point; global loads may stay in flight (their users wait for them as usual).
__device__ __forceinline__ void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): LDS done; global loads may stay in flight
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

// A 16x16x16 product (4 k per lane) through the 16x16x32 instruction.  Lane group q
// holds k = 4q + i (i < 4) of the short form; both operands place it at k' = 8q + i of
// the long form with k' = 8q + 4..7 zero, so the sum over k' equals the sum over k.
// The 16x16x16 bf16 instruction itself is not used: in this kernel its results varied
// from run to run (up to 1e-1 in pair gradients, depending on the surrounding
// instruction timing), while this form reproduces the CPU emulation of the kernel and is
// bitwise stable.
__device__ __forceinline__ f4 mma16(s4 a, s4 b, f4 c) {
  bf8 x, y;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const short av = a[i], bv = b[i];
    x[i] = *(const __bf16 *)&av;
    y[i] = *(const __bf16 *)&bv;
    x[i + 4] = (__bf16)0.f;
    y[i + 4] = (__bf16)0.f;
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

// Two 16x16x16 products summed into one accumulator, c + a0 b0 + a1 b1, through one
// 16x16x32 instruction: lane group q places k = 4q + i of the first product at
// k' = 8q + i and of the second at k' = 8q + 4 + i, so no half of either operand is zero.
__device__ __forceinline__ f4 mma16x2(s4 a0, s4 b0, s4 a1, s4 b1, f4 c) {
  bf8 x, y;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const short u0 = a0[i], v0 = b0[i], u1 = a1[i], v1 = b1[i];
    x[i] = *(const __bf16 *)&u0;
    y[i] = *(const __bf16 *)&v0;
    x[i + 4] = *(const __bf16 *)&u1;
    y[i + 4] = *(const __bf16 *)&v1;
  }
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, c, 0, 0, 0);
}

// acc[t] += A(16 x K) . B_t(16 x K)^T for t < nt; A rows at a (stride lda); B_t rows
// at b + 16 t ldb (stride ldb); K a multiple of 16; operands bf16, k contiguous.
template <int NT>
__device__ __forceinline__ void mm(f4 (&acc)[NT], const bf16_t *a, int lda, const bf16_t *b, int ldb, int K, int nt) {
  const int l = lane(), r = l & 15, q = l >> 4;
  int k0 = 0;
  for (; k0 + 32 <= K; k0 += 32) {
    const bf8 x = ld8(a + r * lda + k0 + 8 * q);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (t < nt) {
        const bf8 y = ld8(b + (16 * t + r) * ldb + k0 + 8 * q);
        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[t], 0, 0, 0);
      }
  }
  if (k0 < K) {
    const s4 x = ld4(a + r * lda + k0 + 4 * q);
#pragma unroll
    for (int t = 0; t < NT; ++t)
      if (t < nt) {
        const s4 y = ld4(b + (16 * t + r) * ldb + k0 + 4 * q);
        acc[t] = mma16(x, y, acc[t]);
      }
  }
}

// acc[t] += A(16 x 112) . B_t(16 x 112)^T for t < NT with B in global memory (weights, L2
// resident).  The fragments of the next k step are loaded before the products of the
// current one are issued, so a product waits for one L2 round trip, not for one per tile.
template <int NT>
__device__ __forceinline__ void mm_g(f4 (&acc)[NT], const bf16_t *a, int lda, const bf16_t *__restrict__ bf) {
  const int l = lane(), r = l & 15, q = l >> 4;
  // B in fragment order: tile t at bf + 1792 t, its k fragments s < 3 at + 512 s + 8 l,
  // the k = 96..111 tail at + 1536 + 4 l
  bf8 y[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) y[t] = *(const bf8 *)(bf + 1792 * t + 8 * l);
#pragma unroll
  for (int st = 0; st < 3; ++st) {
    const bf8 x = ld8(a + r * lda + 32 * st + 8 * q);
    bf8 yn[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      if (st < 2) {
        yn[t] = *(const bf8 *)(bf + 1792 * t + 512 * (st + 1) + 8 * l);
      } else {  // the k = 96..111 tail, four per lane, placed as in mma16
        const s4 v = *(const s4 *)(bf + 1792 * t + 1536 + 4 * l);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const short e = v[i];
          yn[t][i] = *(const __bf16 *)&e;
          yn[t][i + 4] = (__bf16)0.f;
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y[t], acc[t], 0, 0, 0);
#pragma unroll
    for (int t = 0; t < NT; ++t) y[t] = yn[t];
  }
  const s4 xt = ld4(a + r * lda + 96 + 4 * q);
  bf8 x;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const short e = xt[i];
    x[i] = *(const __bf16 *)&e;
    x[i + 4] = (__bf16)0.f;
  }
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y[t], acc[t], 0, 0, 0);
}

// Same with the A operand held as fp32 in LDS (rounded to bf16 when loaded); K multiple of 32.
template <int NT>
__device__ __forceinline__ void mm_a32(f4 (&acc)[NT], const float *a, int lda, const bf16_t *b, int ldb, int K) {
  const int l = lane(), r = l & 15, q = l >> 4;
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf8 x;
    const float *ap = a + r * lda + k0 + 8 * q;
#pragma unroll
    for (int e = 0; e < 8; ++e) x[e] = (__bf16)ap[e];
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const bf8 y = ld8(b + (16 * t + r) * ldb + k0 + 8 * q);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(x, y, acc[t], 0, 0, 0);
    }
  }
}

template <int NT> __device__ __forceinline__ void zero(f4 (&a)[NT]) {
#pragma unroll
  for (int t = 0; t < NT; ++t) a[t] = f4{0.f, 0.f, 0.f, 0.f};
}

// Writes the wave's 16 rows (block jb; fp32 tiles gv, columns 16 t + lane%16) into
// Gb (token-major) and GbT (feature-major) as bf16; columns >= M are written as zero.
__device__ __forceinline__ void put_rows(bf16_t *Gb, bf16_t *GbT, const f4 (&gv)[7], int jb) {
  const int l = lane(), q = l >> 4, cl = l & 15;
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const int m = 16 * t + cl;
    s4 col;  // the lane's four rows of feature m, consecutive in GbT: one 8-byte store
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const bf16_t v = (bf16_t)(m < M ? gv[t][ii] : 0.f);
      Gb[(jb * 16 + 4 * q + ii) * LDK + m] = v;
      col[ii] = __builtin_bit_cast(short, v);
    }
    *(s4 *)(GbT + m * LDT + jb * 16 + 4 * q) = col;
  }
}

// Embedding net for the wave's rows (block jb) -> G (fp32 tiles).  h1 is staged (fp32) in
// scr1 (>= 512 floats), h2 in scr2 (>= 1024 floats); both wave-private.
__device__ void embed_rows(const Tables &w, const bf16_t *w2T, int ld2, const bf16_t *w3T, int ld3,
                           const EnvB &e, int ti, int jb, float *scr1, float *scr2, f4 (&gv)[7]) {
  const int l = lane(), q = l >> 4, cl = l & 15;
  // per-lane weights: first layer column c1 = lane % 32 (type part for every neighbour
  // type), second-layer bias columns 16 t + lane%16, third-layer bias columns
  const int c1 = l & 31;
  const bool c1v = c1 < E1;
  const float w1c = c1v ? w.w1s[c1] : 0.f;
  float bt[NTYPES];
#pragma unroll
  for (int u = 0; u < NTYPES; ++u) bt[u] = c1v ? w.Bt[(ti * NTYPES + u) * E1 + c1] : 0.f;
  float b2v[4], b3v[7];
#pragma unroll
  for (int t = 0; t < 4; ++t) b2v[t] = (16 * t + cl < E2) ? w.b2[16 * t + cl] : 0.f;
#pragma unroll
  for (int t = 0; t < 7; ++t) b3v[t] = (16 * t + cl < M) ? w.b3[16 * t + cl] : 0.f;
#pragma unroll
  for (int x = 0; x < 8; ++x) {
    const int r = (l >> 5) + 2 * x, j = jb * 16 + r;
    const int tj = e.tj[j];
    float b = bt[0];
#pragma unroll
    for (int u = 1; u < NTYPES; ++u) b = (tj == u) ? bt[u] : b;
    scr1[r * 32 + c1] = c1v ? ftanh(e.s[j] * w1c + b) : 0.f;
  }
  wave_fence();
  f4 a2[4];
  zero(a2);
  mm_a32<4>(a2, scr1, 32, w2T, ld2, 32);
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int c = 16 * t + cl;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int r = 4 * q + ii;
      scr2[r * 64 + c] = c < E2 ? ftanh(a2[t][ii] + b2v[t]) + scr1[r * 32 + (c % E1)] : 0.f;
    }
  }
  wave_fence();
  f4 a3[7];
  zero(a3);
  mm_a32<7>(a3, scr2, 64, w3T, ld3, 64);
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    const int m = 16 * t + cl;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int r = 4 * q + ii;
      gv[t][ii] = m < M ? ftanh(a3[t][ii] + b3v[t]) + scr2[r * 64 + (m % E2)] : 0.f;
    }
  }
  wave_fence();
}

// Scores of the wave's rows (block jb) against every token -> row softmax weights.
// sv holds S on entry and E = exp(S - m)/Z on exit (0 for invalid tokens); the
// attention weights A = sw_k E gate_jk are written (bf16) to stg [16][LDT].
// Optionally records the row max and 1/Z (rmax, rz) for a later recomputation.
__device__ __forceinline__ void softmax_rows(f4 (&sv)[8], const EnvB &e, int jb, int n, int nb, bf16_t *stg,
                                             float *rmax, float *rz) {
  const int l = lane(), q = l >> 4, cl = l & 15;
  float mx[4], z[4], iz[4], hj[4][3];
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    const int j = jb * 16 + 4 * q + ii;
    hj[ii][0] = e.rh[3 * j];
    hj[ii][1] = e.rh[3 * j + 1];
    hj[ii][2] = e.rh[3 * j + 2];
    mx[ii] = -INFINITY;
    z[ii] = 0.f;
  }
#pragma unroll
  for (int ct = 0; ct < 8; ++ct)
    if (ct < nb && 16 * ct + cl < n)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) mx[ii] = fmaxf(mx[ii], sv[ct][ii]);
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    mx[ii] = max16(mx[ii]);
    if (mx[ii] == -INFINITY) mx[ii] = 0.f;
  }
#pragma unroll
  for (int ct = 0; ct < 8; ++ct) {
    const int k = 16 * ct + cl;
    const bool kv = ct < nb && k < n;
    const float swk = ct < nb ? e.sw[k] : 0.f;
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const float ex = kv ? fexp(sv[ct][ii] - mx[ii]) : 0.f;
      sv[ct][ii] = ex;
      z[ii] += swk * ex;
    }
  }
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    z[ii] = sum16(z[ii]);
    iz[ii] = z[ii] > 0.f ? 1.f / z[ii] : 0.f;
  }
#pragma unroll
  for (int ct = 0; ct < 8; ++ct)
    if (ct < nb) {
      const int k = 16 * ct + cl;
      const float swk = e.sw[k], hx = e.rh[3 * k], hy = e.rh[3 * k + 1], hz = e.rh[3 * k + 2];
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const float E = sv[ct][ii] * iz[ii];
        sv[ct][ii] = E;
        const float gt = hj[ii][0] * hx + hj[ii][1] * hy + hj[ii][2] * hz;
        stg[(4 * q + ii) * LDT + k] = (bf16_t)(swk * E * gt);
      }
    }
  if (rmax && cl == 0)
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = jb * 16 + 4 * q + ii;
      rmax[j] = mx[ii];
      rz[j] = iz[ii];
    }
}

// Stages fp32 tiles (columns 16 t + lane%16, t < 7) into stg [16][LDT] as bf16.
__device__ __forceinline__ void stage7(bf16_t *stg, const f4 (&v)[7]) {
  const int l = lane(), q = l >> 4, cl = l & 15;
#pragma unroll
  for (int t = 0; t < 7; ++t)
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) stg[(4 * q + ii) * LDT + 16 * t + cl] = (bf16_t)v[t][ii];
}

// One attention layer forward for the wave's rows: gv (G_in, fp32) -> gv (G_out).
// Also returns xh (normalised residual) and isig (1/sigma per accumulator row).
// If Uall is given, U rows are written there (and read from there for S).  The weight
// operands wqkT and wvoT are read from global memory in MFMA fragment order.
__device__ void layer_rows(const Tables &w, const bf16_t *wqkT, const bf16_t *wvoT, int layer,
                           const EnvB &e, const bf16_t *Gb,
                           const bf16_t *GbT, bf16_t *stg, bf16_t *Uall, int jb, int n, int nb, int NP, float ln_eps,
                           f4 (&gv)[7], f4 (&sv)[8], f4 (&xh)[7], float (&isig)[4], float *rmax, float *rz) {
  const int l = lane(), q = l >> 4, cl = l & 15;
  f4 acc[7];
  zero(acc);
  mm_g<7>(acc, Gb + jb * 16 * LDK, LDK, wqkT);  // U = G Wqk
  const bf16_t *ua;
  int lda;
  if (Uall) {
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) Uall[(jb * 16 + 4 * q + ii) * LDK + 16 * t + cl] = (bf16_t)acc[t][ii];
    ua = Uall + jb * 16 * LDK;
    lda = LDK;
  } else {
    stage7(stg, acc);
    ua = stg;
    lda = LDT;
  }
  wave_fence();
  zero(sv);
  mm<8>(sv, ua, lda, Gb, LDK, KM, nb);  // S = U G^T
  wave_fence();
  softmax_rows(sv, e, jb, n, nb, stg, rmax, rz);
  wave_fence();
  zero(acc);
  mm<7>(acc, stg, LDT, GbT, LDT, NP, 7);  // H = A G
  wave_fence();
  stage7(stg, acc);
  wave_fence();
  zero(acc);
  mm_g<7>(acc, stg, LDT, wvoT);  // Y = H Wvo
  wave_fence();
  // X = G + Y;  G <- gamma (X - mu) / sigma + beta
#pragma unroll
  for (int ii = 0; ii < 4; ++ii) {
    float s1 = 0.f;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      const float x = (16 * t + cl < M) ? gv[t][ii] + acc[t][ii] : 0.f;
      xh[t][ii] = x;
      s1 += x;
    }
    const float mu = sum16(s1) * (1.f / M);
    float s2 = 0.f;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      const float d = (16 * t + cl < M) ? xh[t][ii] - mu : 0.f;
      s2 += d * d;
    }
    isig[ii] = 1.f / sqrtf(sum16(s2) * (1.f / M) + ln_eps);
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      const int m = 16 * t + cl;
      const float xn = (m < M) ? (xh[t][ii] - mu) * isig[ii] : 0.f;
      xh[t][ii] = xn;
      gv[t][ii] = (m < M) ? w.gamma[layer][m] * xn + w.beta[layer][m] : 0.f;
    }
  }
}

// One layer input, saved for the backward in the accumulator layout of the row blocks:
// block jb at dst + 1600 jb, its tiles t < 6 at + 256 t with lane l's four values at
// + 4 l, and the four real features of tile 6 (lanes with l % 16 < 4) at
// + 1536 + 4 (4 (l / 16) + l % 16); each tile is one contiguous access per wave.  Rows
// j >= n of the block are stored as they are and masked on reading.
__device__ __forceinline__ void save_rows(float *__restrict__ dst, const f4 (&gv)[7], int jb) {
  const int l = lane(), q = l >> 4, cl = l & 15;
  float *p = dst + 1600 * jb;
#pragma unroll
  for (int t = 0; t < 6; ++t) *(f4 *)(p + 256 * t + 4 * l) = gv[t];
  if (cl < M - 96) *(f4 *)(p + 1536 + 4 * (4 * q + cl)) = gv[6];
}

// Reads those rows back (rows j >= n, which never reach a valid token, and features
// m >= M as zero).
__device__ __forceinline__ void load_rows(const float *__restrict__ src, f4 (&gv)[7], int jb, int n) {
  const int l = lane(), q = l >> 4, cl = l & 15;
  const int j0 = jb * 16 + 4 * q;
  const float *p = src + 1600 * jb;
#pragma unroll
  for (int t = 0; t < 7; ++t) {
    f4 v = f4{0.f, 0.f, 0.f, 0.f};
    if (t < 6) v = *(const f4 *)(p + 256 * t + 4 * l);
    else if (cl < M - 96) v = *(const f4 *)(p + 1536 + 4 * (4 * q + cl));
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) gv[t][ii] = j0 + ii < n ? v[ii] : 0.f;
  }
}

constexpr int LD2 = 40;   // ... of the staged W2^T [64][32]
constexpr int LD3 = 72;   // ... of the staged W3^T [112][64]

// Workgroup copy of two bf16 matrices, [R0][C0] and [R1][C1] (columns multiples of 8,
// row strides g0, g1 in global memory), into LDS with row strides l0, l1, by NTHR
// threads in 16-byte pieces.  Every load of a thread is issued before its first store,
// so the copy costs one L2 round trip.
template <int R0, int C0, int R1, int C1, int NTHR>
__device__ __forceinline__ void stage_weights2(bf16_t *d0, int l0, const bf16_t *__restrict__ s0, int g0, bf16_t *d1,
                                               int l1, const bf16_t *__restrict__ s1, int g1) {
  constexpr int P0 = C0 / 8, T0 = R0 * P0, N0 = (T0 + NTHR - 1) / NTHR;
  constexpr int P1 = C1 / 8, T1 = R1 * P1, N1 = (T1 + NTHR - 1) / NTHR;
  bf8 v0[N0], v1[N1];
#pragma unroll
  for (int c = 0; c < N0; ++c) {
    const int x = threadIdx.x + c * NTHR;
    if (x < T0) v0[c] = *(const bf8 *)(s0 + (size_t)(x / P0) * g0 + 8 * (x % P0));
  }
#pragma unroll
  for (int c = 0; c < N1; ++c) {
    const int x = threadIdx.x + c * NTHR;
    if (x < T1) v1[c] = *(const bf8 *)(s1 + (size_t)(x / P1) * g1 + 8 * (x % P1));
  }
#pragma unroll
  for (int c = 0; c < N0; ++c) {
    const int x = threadIdx.x + c * NTHR;
    if (x < T0) *(bf8 *)(d0 + (x / P0) * l0 + 8 * (x % P0)) = v0[c];
  }
#pragma unroll
  for (int c = 0; c < N1; ++c) {
    const int x = threadIdx.x + c * NTHR;
    if (x < T1) *(bf8 *)(d1 + (x / P1) * l1 + 8 * (x % P1)) = v1[c];
  }
}

}  // namespace
}  // namespace dp
