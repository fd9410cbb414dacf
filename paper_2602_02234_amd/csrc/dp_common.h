// Device-side building blocks shared by the gfx950 kernels: sizes, the
// wave-level MFMA tile product, cross-lane row reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dp {

// ---------------------------------------------------------------- model sizes
constexpr int NTYPES = 5;
constexpr int TEBD = 8;
constexpr int E1 = 25;       // embedding widths 17 -> 25 -> 50 -> 100
constexpr int E2 = 50;
constexpr int M = 100;       // neighbour representation width
constexpr int NATTN = 2;     // attention layers
constexpr int DATTN = 128;   // attention width (enters through the fused 100x100 products)
constexpr int M2 = 16;       // axis neurons
constexpr int ND = M * M2;   // descriptor length 1600
constexpr int FH = 240;      // fitting width
constexpr int SEL = 120;     // neighbour capacity
constexpr int NPMAX = 128;   // tokens per atom after padding to a multiple of 16
constexpr int GSAVE_LAYER = NPMAX * M;  // floats per atom and layer of the saved layer inputs

// ---------------------------------------------------------------- LDS strides
constexpr int LDM = 104;     // row stride (floats) of [token][M] arrays
constexpr int LDN = 132;     // row stride of [16][token] blocks
constexpr int NW = 8;        // waves per workgroup of the per-atom kernels
constexpr int NTHREADS = NW * 64;

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16_t;

__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }
__device__ __forceinline__ int wave_id() { return threadIdx.x >> 6; }

// ------------------------------------------------------------ MFMA 16x16 tile
// acc[i] += sum_k X(r, k) * Y(c, k) for the 16x16 tile held by one wave, with
// r = 4*(lane/16) + i and c = lane%16 (the gfx9 16x16 accumulator layout).  X and
// Y are functors returning float for (row-in-tile, k); k >= K reads as zero.
// Operand type T selects the instruction: float -> v_mfma_f32_16x16x4_f32,
// bf16 -> v_mfma_f32_16x16x32_bf16 (operands rounded to nearest even).
template <typename T> struct Mma;

template <> struct Mma<float> {
  static constexpr int KS = 4;
  template <class FX, class FY>
  __device__ __forceinline__ static void tile(f4 &acc, const FX &X, const FY &Y, int K) {
    const int l = lane_id();
    const int r = l & 15, kq = l >> 4;
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int k = k0 + kq;
      const float a = (k < K) ? X(r, k) : 0.f;
      const float b = (k < K) ? Y(r, k) : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
  }
};

template <> struct Mma<bf16_t> {
  static constexpr int KS = 32;
  template <class FX, class FY>
  __device__ __forceinline__ static void tile(f4 &acc, const FX &X, const FY &Y, int K) {
    const int l = lane_id();
    const int r = l & 15, kq = (l >> 4) * 8;
    for (int k0 = 0; k0 < K; k0 += 32) {
      bf8 a, b;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + kq + e;
        a[e] = (__bf16)((k < K) ? X(r, k) : 0.f);
        b[e] = (__bf16)((k < K) ? Y(r, k) : 0.f);
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
  }
};

// Row index (within a 16x16 tile) of accumulator element i in this lane.
__device__ __forceinline__ int acc_row(int i) { return 4 * (lane_id() >> 4) + i; }
__device__ __forceinline__ int acc_col() { return lane_id() & 15; }

// Cross-lane moves within a row of 16 lanes by DPP (no LDS round trip): the value of
// the partner lane.  Quad permutations 0xB1 (lane ^ 1) and 0x4E (lane ^ 2), half-row
// mirror 0x141 (lane ^ 7 within 8), row mirror 0x140 (lane ^ 15 within 16) and row
// rotation by 8, 0x128 (lane ^ 8 within 16).  Every lane of the wave must be active.
template <int CTRL> __device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), CTRL, 0xF, 0xF, false));
}
// Sum over the 16 lanes sharing lane/16 (one tile row group); the same value in all of
// them (each step adds a partner's value, and a + b == b + a exactly).
__device__ __forceinline__ float sum16(float v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return v;
}
__device__ __forceinline__ float max16(float v) {
  v = fmaxf(v, dpp<0xB1>(v));
  v = fmaxf(v, dpp<0x4E>(v));
  v = fmaxf(v, dpp<0x141>(v));
  v = fmaxf(v, dpp<0x140>(v));
  return v;
}
// Sum over the 4 lanes l, l^16, l^32, l^48 (one tile column across row groups).
__device__ __forceinline__ float sum_cols4(float v) {
  v += __shfl_xor(v, 16);
  v += __shfl_xor(v, 32);
  return v;
}

// Load of a weight stored as T (float or bf16) as float.
__device__ __forceinline__ float ldw(const float *p, int i) { return p[i]; }
__device__ __forceinline__ float ldw(const bf16_t *p, int i) { return (float)p[i]; }

}  // namespace dp
