// Backward descriptor kernels of the bfloat16 path: g_ij = dE_i / dDelta_ij from
// dE/dD, one workgroup per atom.  Each layer's forward is recomputed from its saved
// fp32 input rows; the terms of dG that couple a token to every query row (A^T dH and
// dS^T U) are gathered in a second, column pass in which wave w recomputes the score
// and score-gradient tiles of its own token blocks against every query block from U
// and dH kept in LDS.  Atoms with up to 7 row blocks of 16 neighbours run on a 7-wave
// instance (one block per wave), the others on a 4-wave instance (two blocks per wave).
#define DP_BF16_OPAQUE_LANE 1
#include "descriptor_bf16.h"

namespace dp {
namespace {

template <int NW> struct __align__(16) SmemB16 {
  bf16_t Gb[NPMAX * LDK];
  bf16_t GbT[KM * LDT];
  bf16_t Uall[NPMAX * LDK];
  bf16_t dHall[NPMAX * LDK];
  bf16_t stg[NW][16 * LDT];
  EnvB e;
  float rmax[NPMAX], rz[NPMAX], rrho[NPMAX];
  float drh[NPMAX * 3];
  float dswa[NPMAX];
  float dRt[NPMAX * 4];
  float dT[M * 4];
};

// Backward of one layer for the wave's blocks, from the layer input saved by the forward
// kernel (gin: the wave's fp32 rows, j >= n zero).  If gs_next is given, the next
// layer's saved input rows are loaded into gin before the column pass, so that their
// latency overlaps it.  dg: on entry the gradient w.r.t. the layer output
// (ignored for the top layer, whose output gradient is Rt dT^T / sel), on exit w.r.t.
// the layer input.  The column pass also adds, for the wave's own token columns k, the
// column sums over every query row of the softmax-weight gradient W_jk (to dswa[k]) and
// of the gate gradient dC_jk rhat_j (to drh[k]).
template <int NW, int BPW>
__device__ __forceinline__ void layer_bwd(const Tables &w, const WeightsB16 &wp, int layer, bool top,
                                       SmemB16<NW> &sm, f4 (&gin)[BPW][7], const float *__restrict__ gs_next, int n,
                                       int nb, int NP, float ln_eps, f4 (&dg)[BPW][7]) {
  const int wv = wave_id(), l = lane(), q = l >> 4, cl = l & 15;
  bf16_t *stg = sm.stg[wv];
  const float inv_sel = 1.f / (float)SEL;
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    const int jb = wv + NW * b;
    if (jb >= nb) continue;
    f4 gcur[7], sv[8], xh[7];
    float isig[4];
#pragma unroll
    for (int t = 0; t < 7; ++t) gcur[t] = gin[b][t];
    layer_rows(w, wp.WqkT[layer], wp.WvoT[layer], layer, sm.e, sm.Gb, sm.GbT, stg, sm.Uall, jb, n, nb, NP,
               ln_eps, gcur, sv, xh, isig, sm.rmax, sm.rz);
    // incoming gradient of the layer output: for the top layer go = Rt dT^T / sel (and
    // dRt = G_out dT / sel), otherwise the gradient the layer above passed down
    f4 go[7];
    if (top) {
      float4 dTv[7];
#pragma unroll
      for (int t = 0; t < 7; ++t)
        dTv[t] = (16 * t + cl < M) ? *(const float4 *)(sm.dT + 4 * (16 * t + cl)) : make_float4(0.f, 0.f, 0.f, 0.f);
      float pr[16];  // the lane's partial G_out dT over its feature columns, [row ii][c]
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int j = jb * 16 + 4 * q + ii;
        const float sj = sm.e.s[j], hx = sm.e.rh[3 * j], hy = sm.e.rh[3 * j + 1], hz = sm.e.rh[3 * j + 2];
        float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
#pragma unroll
        for (int t = 0; t < 7; ++t) {
          const float4 d = dTv[t];
          go[t][ii] = sj * (d.x + hx * d.y + hy * d.z + hz * d.w) * inv_sel;  // zero for padded features
          const float gvv = gcur[t][ii];
          p0 += gvv * d.x; p1 += gvv * d.y; p2 += gvv * d.z; p3 += gvv * d.w;
        }
        pr[4 * ii] = p0; pr[4 * ii + 1] = p1; pr[4 * ii + 2] = p2; pr[4 * ii + 3] = p3;
      }
      // reduce-scatter over the 16 lanes of the row group: at the step of bit h each lane
      // keeps the half of its entries selected by that bit of its lane index and adds the
      // partner's copy of it (partners differ in bit h and agree in the bits above);
      // afterwards lane cl holds the total of entry cl = 4 ii + c
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const bool up = (cl & 8) != 0;
        const float lo = pr[k], hi = pr[k + 8];
        pr[k] = (up ? hi : lo) + dpp<0x128>(up ? lo : hi);
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool up = (cl & 4) != 0;
        const float lo = pr[k], hi = pr[k + 4];
        pr[k] = (up ? hi : lo) + dpp<0x141>(up ? lo : hi);
      }
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const bool up = (cl & 2) != 0;
        const float lo = pr[k], hi = pr[k + 2];
        pr[k] = (up ? hi : lo) + dpp<0x4E>(up ? lo : hi);
      }
      {
        const bool up = (cl & 1) != 0;
        pr[0] = (up ? pr[1] : pr[0]) + dpp<0xB1>(up ? pr[0] : pr[1]);
      }
      sm.dRt[4 * (jb * 16 + 4 * q) + cl] = pr[0] * inv_sel;
    } else {
#pragma unroll
      for (int t = 0; t < 7; ++t) go[t] = (16 * t + cl < M) ? dg[b][t] : f4{0.f, 0.f, 0.f, 0.f};
    }
    // LayerNorm backward: dX = (dxh - mean(dxh) - xh mean(dxh xh)) / sigma, dxh = gamma dG_out
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const int m = 16 * t + cl;
        const float d = (m < M) ? w.gamma[layer][m] * go[t][ii] : 0.f;
        go[t][ii] = d;
        s0 += d;
        s1 += d * xh[t][ii];
      }
      s0 = sum16(s0) * (1.f / M);
      s1 = sum16(s1) * (1.f / M);
#pragma unroll
      for (int t = 0; t < 7; ++t) {
        const int m = 16 * t + cl;
        dg[b][t][ii] = (m < M) ? (go[t][ii] - s0 - xh[t][ii] * s1) * isig[ii] : 0.f;  // dG_in starts as dX
      }
    }
    wave_fence();
    stage7(stg, dg[b]);  // dY = dX
    wave_fence();
    f4 acc[7];
    zero(acc);
    mm_g<7>(acc, stg, LDT, wp.Wvo[layer]);  // dH = dY Wvo^T
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) sm.dHall[(jb * 16 + 4 * q + ii) * LDK + 16 * t + cl] = (bf16_t)acc[t][ii];
    wave_fence();
    f4 da[8];
    zero(da);
    mm<8>(da, sm.dHall + jb * 16 * LDK, LDK, sm.Gb, LDK, KM, nb);  // dA = dH G^T
    wave_fence();
    // weighted-softmax and gate backward
    float hj[4][3], rho[4], hxa[4], hya[4], hza[4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = jb * 16 + 4 * q + ii;
      hj[ii][0] = sm.e.rh[3 * j];
      hj[ii][1] = sm.e.rh[3 * j + 1];
      hj[ii][2] = sm.e.rh[3 * j + 2];
      rho[ii] = hxa[ii] = hya[ii] = hza[ii] = 0.f;
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct) {
      const int k = 16 * ct + cl;
      const bool kv = ct < nb && k < n;
      float swk = 0.f, hx = 0.f, hy = 0.f, hz = 0.f;
      if (ct < nb) {
        swk = sm.e.sw[k];
        hx = sm.e.rh[3 * k];
        hy = sm.e.rh[3 * k + 1];
        hz = sm.e.rh[3 * k + 2];
      }
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        if (kv && jb * 16 + 4 * q + ii < n) {
          const float P = swk * sv[ct][ii];
          const float gt = hj[ii][0] * hx + hj[ii][1] * hy + hj[ii][2] * hz;
          const float dP = da[ct][ii] * gt;
          const float dC = da[ct][ii] * P;
          rho[ii] += P * dP;
          hxa[ii] += dC * hx;
          hya[ii] += dC * hy;
          hza[ii] += dC * hz;
          da[ct][ii] = dP;
        } else {
          da[ct][ii] = 0.f;
        }
      }
    }
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = jb * 16 + 4 * q + ii;
      rho[ii] = sum16(rho[ii]);
      const float hx = sum16(hxa[ii]), hy = sum16(hya[ii]), hz = sum16(hza[ii]);
      if (cl == 0) {
        sm.rrho[j] = rho[ii];
        sm.drh[3 * j] += hx;
        sm.drh[3 * j + 1] += hy;
        sm.drh[3 * j + 2] += hz;
      }
    }
#pragma unroll
    for (int ct = 0; ct < 8; ++ct)
      if (ct < nb) {
        const int k = 16 * ct + cl;
        const float swk = sm.e.sw[k];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const bool v = k < n && jb * 16 + 4 * q + ii < n;
          const float W = v ? sv[ct][ii] * (da[ct][ii] - rho[ii]) : 0.f;
          stg[(4 * q + ii) * LDT + k] = (bf16_t)(swk * W);  // dS
        }
      }
    wave_fence();
    zero(acc);
    mm<7>(acc, stg, LDT, sm.GbT, LDT, NP, 7);  // dU = dS G
    wave_fence();
    stage7(stg, acc);
    wave_fence();
    zero(acc);
    mm_g<7>(acc, stg, LDT, wp.Wqk[layer]);  // dG += dU Wqk^T
#pragma unroll
    for (int t = 0; t < 7; ++t) dg[b][t] += acc[t];
    wave_fence();
  }
  if (gs_next) {
#pragma unroll
    for (int b = 0; b < BPW; ++b)
      if (wv + NW * b < nb) load_rows(gs_next, gin[b], wv + NW * b, n);
  }
  __syncthreads();
  // Token-major copies for the column pass, whose products contract over tokens: U^T into
  // GbT (free until the next layer's input is put there) and, where the staging area
  // holds it (seven waves), dH^T there; each wave transposes its own blocks.
  constexpr bool HT = NW * 16 * LDT >= KM * LDT;
  bf16_t *UT = sm.GbT, *HTs = &sm.stg[0][0];
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    const int jb = wv + NW * b;
    if (jb >= nb) continue;
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      s4 u, h;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int j = jb * 16 + 4 * q + ii;
        const bf16_t vu = sm.Uall[j * LDK + 16 * t + cl], vh = sm.dHall[j * LDK + 16 * t + cl];
        u[ii] = *(const short *)&vu;
        h[ii] = *(const short *)&vh;
      }
      *(s4 *)(UT + (16 * t + cl) * LDT + jb * 16 + 4 * q) = u;
      if constexpr (HT) *(s4 *)(HTs + (16 * t + cl) * LDT + jb * 16 + 4 * q) = h;
    }
  }
  __syncthreads();
  // column pass: dG[k] += sum_j A_jk dH_j + dS_jk U_j for the wave's own token blocks
  // (kb = wave and wave + NW); the U / dH columns of each block jb are read once for both
  {
    bool has[BPW];
    float swk[BPW], hk[BPW][3];
    float cw[BPW][4];  // per-lane partial column sums: W, dC rhat_j (x, y, z)
    f4 cacc[BPW][7];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      const int kb = wv + NW * b;
      has[b] = kb < nb;
      const int k = min(kb, 7) * 16 + cl;
      swk[b] = sm.e.sw[k];
      hk[b][0] = sm.e.rh[3 * k];
      hk[b][1] = sm.e.rh[3 * k + 1];
      hk[b][2] = sm.e.rh[3 * k + 2];
      cw[b][0] = cw[b][1] = cw[b][2] = cw[b][3] = 0.f;
      zero(cacc[b]);
    }
    // the key-side fragments (Gb rows of the wave's column blocks) are the same for every jb
    bf8 gk[BPW][3];
    s4 gkt[BPW];
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      const bf16_t *gr = sm.Gb + (min(wv + NW * b, 7) * 16 + (l & 15)) * LDK;
#pragma unroll
      for (int st = 0; st < 3; ++st) gk[b][st] = ld8(gr + 32 * st + 8 * q);
      gkt[b] = ld4(gr + 96 + 4 * q);
    }
    if (has[0]) {
      for (int jb = 0; jb < nb; ++jb) {
        float rmx[4], rzz[4], rro[4], hj[4][3];
        bool jv[4];
#pragma unroll
        for (int ii = 0; ii < 4; ++ii) {
          const int j = jb * 16 + 4 * q + ii;
          jv[ii] = j < n;
          rmx[ii] = sm.rmax[j];
          rzz[ii] = sm.rz[j];
          rro[ii] = sm.rrho[j];
          hj[ii][0] = sm.e.rh[3 * j];
          hj[ii][1] = sm.e.rh[3 * j + 1];
          hj[ii][2] = sm.e.rh[3 * j + 2];
        }
        s4 yh[7], yu[7];
#pragma unroll
        for (int t = 0; t < 7; ++t) {
          const int m = 16 * t + cl;
          yu[t] = ld4(UT + m * LDT + jb * 16 + 4 * q);
          if constexpr (HT) {
            yh[t] = ld4(HTs + m * LDT + jb * 16 + 4 * q);
          } else {
#pragma unroll
            for (int ii = 0; ii < 4; ++ii) {
              const bf16_t vh = sm.dHall[(jb * 16 + 4 * q + ii) * LDK + m];
              yh[t][ii] = *(const short *)&vh;
            }
          }
        }
#pragma unroll
        for (int b = 0; b < BPW; ++b) {
          if (!has[b]) continue;
          const int kb = wv + NW * b;
          const bool kv = kb * 16 + cl < n;
          f4 st[1], dt[1];
          zero(st);
          zero(dt);
          {
            const bf16_t *ur = sm.Uall + (jb * 16 + (l & 15)) * LDK, *hr = sm.dHall + (jb * 16 + (l & 15)) * LDK;
#pragma unroll
            for (int s3 = 0; s3 < 3; ++s3) {
              st[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(ur + 32 * s3 + 8 * q), gk[b][s3], st[0], 0, 0, 0);
              dt[0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ld8(hr + 32 * s3 + 8 * q), gk[b][s3], dt[0], 0, 0, 0);
            }
            st[0] = mma16(ld4(ur + 96 + 4 * q), gkt[b], st[0]);
            dt[0] = mma16(ld4(hr + 96 + 4 * q), gkt[b], dt[0]);
          }
          s4 xa, xs;
#pragma unroll
          for (int ii = 0; ii < 4; ++ii) {
            float A = 0.f, dS = 0.f;
            if (kv && jv[ii]) {
              const float E = fexp(st[0][ii] - rmx[ii]) * rzz[ii];
              const float P = swk[b] * E;
              const float gt = hj[ii][0] * hk[b][0] + hj[ii][1] * hk[b][1] + hj[ii][2] * hk[b][2];
              const float W = E * (dt[0][ii] * gt - rro[ii]);  // softmax-weight gradient
              const float dC = dt[0][ii] * P;                   // gate gradient
              A = P * gt;
              dS = swk[b] * W;
              cw[b][0] += W;
              cw[b][1] += dC * hj[ii][0];
              cw[b][2] += dC * hj[ii][1];
              cw[b][3] += dC * hj[ii][2];
            }
            xa[ii] = bfbits(A);
            xs[ii] = bfbits(dS);
          }
#pragma unroll
          for (int t = 0; t < 7; ++t) {
            cacc[b][t] = mma16x2(xa, yh[t], xs, yu[t], cacc[b][t]);  // A^T dH + dS^T U
          }
        }
      }
    }
#pragma unroll
    for (int b = 0; b < BPW; ++b) {
      // column sums over the 4 row groups; column k is owned by this wave alone
#pragma unroll
      for (int c = 0; c < 4; ++c) cw[b][c] = sum_cols4(cw[b][c]);
      if (has[b]) {
#pragma unroll
        for (int t = 0; t < 7; ++t) dg[b][t] += cacc[b][t];
        if (q == 0) {
          const int k = (wv + NW * b) * 16 + cl;
          sm.dswa[k] += cw[b][0];
          sm.drh[3 * k] += cw[b][1];
          sm.drh[3 * k + 1] += cw[b][2];
          sm.drh[3 * k + 2] += cw[b][3];
        }
      }
    }
  }
  __syncthreads();
}

// Puts the saved layer input rows (fp32 -> bf16) of the wave's blocks into Gb / GbT.
// The wave's layer input rows (bf16) into Gb and GbT.
template <int NW, int BPW>
__device__ __forceinline__ void put_layer_input(SmemB16<NW> &sm, const f4 (&gin)[BPW][7], int nb) {
  const int wv = wave_id();
#pragma unroll
  for (int b = 0; b < BPW; ++b)
    if (wv + NW * b < nb) put_rows(sm.Gb, sm.GbT, gin[b], wv + NW * b);
}

// NW waves per workgroup, each owning BPW row blocks (wave w owns blocks w, w + NW, ...);
// the workgroup takes atom idx[blockIdx.x] for blockIdx.x < *count, so atoms can be sent
// to the instance whose block count fits their neighbour count.
template <int NW, int BPW>
__global__ void __launch_bounds__(NW * 64)
k_desc_bwd_b16(Tables w, WeightsB16 wp, const double *__restrict__ X, const int *__restrict__ types, int natoms,
               const int *__restrict__ nlist, const int *__restrict__ nnei, const Grid *__restrict__ grids,
               const int *__restrict__ sys_of, float rc, float rcs, float ln_eps, const float *__restrict__ Gsave,
               const float *__restrict__ Tsave, const float *__restrict__ dD, float4 *__restrict__ gout,
               const int *__restrict__ idx, const int *__restrict__ count) {
  __shared__ SmemB16<NW> sm;
  if ((int)blockIdx.x >= *count) return;
  const int i = idx[blockIdx.x];
  const Grid g = grids[sys_of[i]];
  const int n = min(max(nnei[i], 0), SEL);
  const int NP = n > 0 ? ((n + 15) / 16) * 16 : 16;
  const int nb = NP / 16;
  const int ti = clamp_type(types[i]);
  const int wv = wave_id(), l = lane(), q = l >> 4, cl = l & 15;
  // the top layer's saved input rows of the wave's blocks, loaded first so that their
  // latency overlaps the environment and dT work
  const float *gs0 = Gsave + (size_t)i * NATTN * GSAVE_LAYER;
  const float *gs1 = gs0 + GSAVE_LAYER;
  f4 gin[BPW][7];
#pragma unroll
  for (int b = 0; b < BPW; ++b)
    if (wv + NW * b < nb) load_rows(gs1, gin[b], wv + NW * b, n);
  // dT = dE/dT from dE/dD (D = T T<^T): dT[m] = sum_a dD[m][a] T[a] + [m < M2] sum_m' dD[m'][m] T[m'];
  // staging is free until the first layer: T [100][4], dE/dD [1600], partial sums [NW * 64]
  float *T = (float *)sm.stg[0];
  float *dDi = T + M * 4;
  float *part = dDi + ND;
  static_assert((M * 4 + ND + NW * 64) * sizeof(float) <= sizeof(sm.stg), "dT staging must fit in stg");
  for (int x = threadIdx.x; x < M; x += NW * 64)
    *(float4 *)(T + 4 * x) = *(const float4 *)(Tsave + ((size_t)i * M + x) * 4);
  for (int x = threadIdx.x; x < ND / 4; x += NW * 64)
    *(float4 *)(dDi + 4 * x) = *(const float4 *)(dD + (size_t)i * ND + 4 * x);
  build_envb(sm.e, X, types, nlist, i, n, natoms, g, rc, rcs);
  for (int x = threadIdx.x; x < NPMAX; x += NW * 64) {
    sm.dswa[x] = 0.f;
    for (int a = 0; a < 3; ++a) sm.drh[3 * x + a] = 0.f;
    for (int a = 0; a < 4; ++a) sm.dRt[4 * x + a] = 0.f;
  }
  __syncthreads();
  for (int x = threadIdx.x; x < M * 4; x += NW * 64) {
    const int m = x >> 2, c = x & 3;
    float acc = 0.f;
    for (int a = 0; a < M2; ++a) acc += dDi[m * M2 + a] * T[4 * a + c];
    sm.dT[x] = acc;
  }
  {
    // the second sum of the 64 entries m < M2 in NW chunks of m', one (chunk, entry) per thread
    constexpr int CH = (M + NW - 1) / NW;
    const int e = threadIdx.x & 63, ch = threadIdx.x >> 6, m = e >> 2, c = e & 3;
    float acc = 0.f;
    for (int mm2 = ch * CH; mm2 < min(M, (ch + 1) * CH); ++mm2) acc += dDi[mm2 * M2 + m] * T[4 * mm2 + c];
    part[threadIdx.x] = acc;
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    float acc = sm.dT[threadIdx.x];
    for (int ch = 0; ch < NW; ++ch) acc += part[64 * ch + threadIdx.x];
    sm.dT[threadIdx.x] = acc;
  }
  put_layer_input<NW, BPW>(sm, gin, nb);
  __syncthreads();
  f4 dg[BPW][7];
#pragma unroll
  for (int b = 0; b < BPW; ++b)
#pragma unroll
    for (int t = 0; t < 7; ++t) dg[b][t] = f4{0.f, 0.f, 0.f, 0.f};
  layer_bwd<NW, BPW>(w, wp, 1, true, sm, gin, gs0, n, nb, NP, ln_eps, dg);
  put_layer_input<NW, BPW>(sm, gin, nb);
  __syncthreads();
  layer_bwd<NW, BPW>(w, wp, 0, false, sm, gin, nullptr, n, nb, NP, ln_eps, dg);
  // the embedding weights of the larger products into LDS (Uall is free now)
  bf16_t *w3Ts = sm.Uall, *w3s = sm.Uall + KM * LD3;
  stage_weights2<KM, 64, 64, KM, NW * 64>(w3Ts, LD3, wp.W3T, 64, w3s, KM, wp.W3, KM);
  bf16_t *w2Ts = sm.Gb, *w2s = sm.Gb + 64 * LD2;  // Gb is free as well
  static_assert(NW <= 7 && 4 * 16 * 104 * 4 <= KM * LDT * 2 &&
                    (64 * LD2 + 32 * LD3) * 2 + (NW > 4 ? NW - 4 : 0) * 16 * 104 * 4 <= NPMAX * LDK * 2,
                "per-wave fp32 scratch of the embedding backward must fit in GbT and the rest of Gb");
  stage_weights2<64, 32, 32, 64, NW * 64>(w2Ts, LD2, wp.W2T, 32, w2s, LD3, wp.W2, 64);
  __syncthreads();
  // embedding backward and the pair gradients of the wave's rows
#pragma unroll
  for (int b = 0; b < BPW; ++b) {
    const int jb = wv + NW * b;
    if (jb >= nb) continue;
    float *h1 = (float *)(sm.dHall + jb * 16 * LDK);  // [16][32]
    float *h2 = (float *)sm.stg[wv];                  // [16][64]
    // [16][104] fp32: dG0 rows, then dh2; waves 0-3 in GbT, waves 4-6 in Gb after the W2 copies
    float *sc = wv < 4 ? (float *)sm.GbT + wv * 16 * 104 : (float *)(w2s + 32 * LD3) + (wv - 4) * 16 * 104;
    // recompute h1, t2, h2 (fp32) for these rows, as the forward kernel made them
    {
      const int c1 = l & 31;
      const bool c1v = c1 < E1;
      const float w1c = c1v ? w.w1s[c1] : 0.f;
#pragma unroll
      for (int x = 0; x < 8; ++x) {
        const int r = (l >> 5) + 2 * x, j = jb * 16 + r;
        const float bt = c1v ? w.Bt[(ti * NTYPES + sm.e.tj[j]) * E1 + c1] : 0.f;
        h1[r * 32 + c1] = c1v ? ftanh(sm.e.s[j] * w1c + bt) : 0.f;
      }
    }
    wave_fence();
    f4 a2[4];
    zero(a2);
    mm_a32<4>(a2, h1, 32, w2Ts, LD2, 32);
    float t2v[4][4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 16 * t + cl;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii;
        const float tt = c < E2 ? ftanh(a2[t][ii] + w.b2[c]) : 0.f;
        t2v[t][ii] = tt;
        h2[r * 64 + c] = c < E2 ? tt + h1[r * 32 + (c % E1)] : 0.f;
      }
    }
    wave_fence();
    f4 a3[7];
    zero(a3);
    mm_a32<7>(a3, h2, 64, w3Ts, LD3, 64);
    // dpre3 = dG0 (1 - t3^2) staged as bf16; dG0 half sums (cols c and c + 50) into sc
    wave_fence();
    bf16_t *stg = sm.stg[wv];  // aliases h2, which is no longer needed
#pragma unroll
    for (int t = 0; t < 7; ++t) {
      const int m = 16 * t + cl;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii;
        const float t3 = m < M ? ftanh(a3[t][ii] + w.b3[m]) : 0.f;
        a3[t][ii] = m < M ? dg[b][t][ii] * (1.f - t3 * t3) : 0.f;
        if (m < M) sc[r * 104 + m] = dg[b][t][ii];
      }
    }
    wave_fence();
    stage7(stg, a3);  // dpre3 (bf16) over h2 (no longer needed)
    wave_fence();
    // dh2 = dpre3 W3^T + (dG0[:, :50] + dG0[:, 50:]);  dpre2 = dh2 (1 - t2^2)
    f4 d2[4];
    zero(d2);
    mm<4>(d2, stg, LDT, w3s, KM, KM, 4);
    wave_fence();
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 16 * t + cl;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii;
        const float v = c < E2 ? d2[t][ii] + sc[r * 104 + c] + sc[r * 104 + c + E2] : 0.f;
        d2[t][ii] = v;  // dh2
      }
    }
    wave_fence();
    // stage dpre2 (bf16, [16][64]) and dh2 halves sum (fp32, for dh1) in sc
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int c = 16 * t + cl;
#pragma unroll
      for (int ii = 0; ii < 4; ++ii) {
        const int r = 4 * q + ii;
        stg[r * LDT + c] = (bf16_t)(c < E2 ? d2[t][ii] * (1.f - t2v[t][ii] * t2v[t][ii]) : 0.f);
        if (c < E2) sc[r * 104 + c] = d2[t][ii];
      }
    }
    wave_fence();
    // dh1 = dpre2 W2^T + (dh2[:, :25] + dh2[:, 25:]);  ds_emb = sum_c dh1 (1 - h1^2) w1s
    f4 d1[2];
    zero(d1);
    mm<2>(d1, stg, LDT, w2s, LD3, 64, 2);
    float dse[4];
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int r = 4 * q + ii;
      float p = 0.f;
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int c = 16 * t + cl;
        if (c < E1) {
          const float dh1 = d1[t][ii] + sc[r * 104 + c] + sc[r * 104 + c + E1];
          const float hv = h1[r * 32 + c];
          p += dh1 * (1.f - hv * hv) * w.w1s[c];
        }
      }
      dse[ii] = sum16(p);
    }
    // pair gradients (lane cl == ii handles row 4q + ii)
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = jb * 16 + 4 * q + ii;
      if (cl == ii && j < SEL) {
        float4 out = make_float4(0.f, 0.f, 0.f, 0.f);
        if (j < n) out = pair_gradient_b(sm.e, j, dse[ii], sm.dRt + 4 * j, sm.drh + 3 * j, sm.dswa[j], rc, rcs);
        gout[(size_t)i * SEL + j] = out;
      }
    }
    wave_fence();
  }
  for (int j = NP + threadIdx.x; j < SEL; j += NW * 64) gout[(size_t)i * SEL + j] = make_float4(0.f, 0.f, 0.f, 0.f);
}

}  // namespace

void launch_descriptor_bwd_b16(const Tables &w, const WeightsB16 &wp, const Workspace &ws,
                               const double *coords, const int *types, int n, int c0, int c1,
                               float rc, float rcs, float ln_eps, hipStream_t st) {
  const int ncen = c1 - c0;  // the forward listed these atoms in ws.bidx
  // atoms with up to 7 row blocks: 7 waves, one block each (on st); the rest: 4 waves,
  // two blocks each, on the side stream, so that a few dense atoms overlap the bulk.  The
  // forward pass listed the atoms of each instance (bidx, bcnt).
  (void)hipEventRecord(ws.fork_ev, st);
  (void)hipStreamWaitEvent(ws.side, ws.fork_ev, 0);
  hipLaunchKernelGGL((k_desc_bwd_b16<4, 2>), dim3(ncen), dim3(4 * 64), 0, ws.side, w, wp, coords, types, n, ws.nlist,
                     ws.nnei, ws.grids, ws.sys_of, rc, rcs, ln_eps, ws.Gsave, ws.Tsave, ws.D, ws.g, ws.bidx + ws.cap,
                     ws.bcnt + 1);
  hipLaunchKernelGGL((k_desc_bwd_b16<7, 1>), dim3(ncen), dim3(7 * 64), 0, st, w, wp, coords, types, n, ws.nlist, ws.nnei,
                     ws.grids, ws.sys_of, rc, rcs, ln_eps, ws.Gsave, ws.Tsave, ws.D, ws.g, ws.bidx, ws.bcnt);
  (void)hipEventRecord(ws.join_ev, ws.side);
  (void)hipStreamWaitEvent(st, ws.join_ev, 0);
}

}  // namespace dp
