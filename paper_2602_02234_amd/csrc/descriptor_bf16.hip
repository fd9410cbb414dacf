// Forward descriptor kernel of the bfloat16 path: one workgroup (8 waves) per atom.
// Environment, type-embedded embedding net (its weights staged in LDS), two attention
// layers (their weights read from L2 in MFMA fragment order), T = G^T Rt / sel and
// D = T T_<16^T; the input rows of each attention layer are saved for the backward.
#include "descriptor_bf16.h"

namespace dp {
namespace {

struct __align__(16) SmemF16 {
  bf16_t Gb[NPMAX * LDK];
  bf16_t GbT[KM * LDT];
  bf16_t stg[NWF][16 * LDT];
  bf16_t Wemb[64 * LD2 + KM * LD3];  // the embedding's W2^T and W3^T
  EnvB e;
};

__global__ void __launch_bounds__(NWF * 64)
k_desc_fwd_b16(Tables w, WeightsB16 wp, const double *__restrict__ X, const int *__restrict__ types, int natoms, int c0,
               const int *__restrict__ nlist, const int *__restrict__ nnei, const Grid *__restrict__ grids, const int *__restrict__ sys_of,
               float rc, float rcs, float ln_eps, float *__restrict__ Gsave, float *__restrict__ Tsave,
               float *__restrict__ D, int *__restrict__ bidx, int *__restrict__ bcnt, int cap) {
  __shared__ SmemF16 sm;
  const int i = c0 + blockIdx.x;
  const Grid g = grids[sys_of[i]];
  const int n = min(max(nnei[i], 0), SEL);
  const int NP = n > 0 ? ((n + 15) / 16) * 16 : 16;
  const int nb = NP / 16;
  if (threadIdx.x == 0) {  // list the atom for the backward instance that fits its block count
    const int cls = nb <= SPLIT_NB ? 0 : 1;
    bidx[cls * cap + atomicAdd(&bcnt[cls], 1)] = i;
  }
  const int ti = clamp_type(types[i]);
  const int wv = wave_id(), l = lane(), q = l >> 4, cl = l & 15;
  build_envb(sm.e, X, types, nlist, i, n, natoms, g, rc, rcs);
  bf16_t *w2s = sm.Wemb, *w3s = sm.Wemb + 64 * LD2;
  stage_weights2<64, 32, KM, 64, NWF * 64>(w2s, LD2, wp.W2T, 32, w3s, LD3, wp.W3T, 64);
  __syncthreads();
  const bool act = wv < nb;
  const int jb = wv;
  bf16_t *stg = sm.stg[wv];
  f4 gv[7];
  if (act) {
    // h1 scratch in this wave's own (not yet written) rows of Gb, h2 in its staging buffer
    embed_rows(w, w2s, LD2, w3s, LD3, sm.e, ti, jb, (float *)(sm.Gb + jb * 16 * LDK), (float *)stg, gv);
    put_rows(sm.Gb, sm.GbT, gv, jb);
  }
  for (int layer = 0; layer < NATTN; ++layer) {
    __syncthreads();  // Gb and GbT hold the layer input
    f4 sv[8], xh[7];
    float isig[4];
    if (act) {
      save_rows(Gsave + ((size_t)i * NATTN + layer) * GSAVE_LAYER, gv, jb);
      layer_rows(w, wp.WqkT[layer], wp.WvoT[layer], layer, sm.e, sm.Gb, sm.GbT, stg, nullptr, jb, n, nb, NP, ln_eps, gv,
                 sv, xh, isig, nullptr, nullptr);
    }
    __syncthreads();  // every wave is done reading them
    if (act) put_rows(sm.Gb, sm.GbT, gv, jb);
  }
  __syncthreads();
  // T = G^T Rt / sel: per-wave partial over its rows, then a fixed-order sum over waves.
  // The partial is four fp32 MFMAs per feature tile: A = the wave's G rows 4q + ii
  // straight from the accumulator registers (lane (q, c) holds G[4q + ii][16t + c], i.e.
  // A[c][q]), B[q][c] = Rt[4q + ii][c] for c < 4; lane (q, c) ends with T[16t + 4q + r][c].
  float *tp = (float *)sm.stg[wv];
  if (act) {
    f4 tacc[7];
    zero(tacc);
#pragma unroll
    for (int ii = 0; ii < 4; ++ii) {
      const int j = jb * 16 + 4 * q + ii;
      const float sj = (j < n) ? sm.e.s[j] : 0.f;
      const float rt = cl == 0 ? sj : (cl < 4 ? sj * sm.e.rh[3 * j + cl - 1] : 0.f);
#pragma unroll
      for (int t = 0; t < 7; ++t) tacc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(gv[t][ii], rt, tacc[t], 0, 0, 0);
    }
#pragma unroll
    for (int t = 0; t < 7; ++t)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 16 * t + 4 * q + r;
        if (cl < 4 && m < M) tp[m * 4 + cl] = tacc[t][r];
      }
  }
  __syncthreads();
  float *T = (float *)sm.GbT;
  for (int x = threadIdx.x; x < M * 4; x += NWF * 64) {
    float acc = 0.f;
    for (int v = 0; v < nb; ++v) acc += ((float *)sm.stg[v])[x];
    acc *= 1.f / (float)SEL;
    T[x] = acc;
    Tsave[(size_t)i * M * 4 + x] = acc;
  }
  __syncthreads();
  for (int x = threadIdx.x; x < ND; x += NWF * 64) {
    const int m = x / M2, a = x % M2;
    const float *tm = T + 4 * m, *ta = T + 4 * a;
    D[(size_t)i * ND + x] = tm[0] * ta[0] + tm[1] * ta[1] + tm[2] * ta[2] + tm[3] * ta[3];
  }
}

}  // namespace

void launch_descriptor_fwd_b16(const Tables &w, const WeightsB16 &wp, const Workspace &ws,
                               const double *coords, const int *types, int n, int c0, int c1,
                               float rc, float rcs, float ln_eps, hipStream_t st) {
  hipLaunchKernelGGL(k_desc_fwd_b16, dim3(c1 - c0), dim3(NWF * 64), 0, st, w, wp, coords, types, n, c0, ws.nlist, ws.nnei, ws.grids,
                     ws.sys_of, rc, rcs, ln_eps, ws.Gsave, ws.Tsave, ws.D, ws.bidx, ws.bcnt, (int)ws.cap);
}

}  // namespace dp
