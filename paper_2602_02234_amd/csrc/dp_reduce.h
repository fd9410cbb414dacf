// Float64 sums with Neumaier compensation in a fixed order, by one workgroup.
#pragma once
#include "dp_internal.h"

namespace dp {
namespace {

struct Neu {
  double s, c;
};
__device__ __forceinline__ void neu_add(Neu &a, double x) {
  const double t = a.s + x;
  if (fabs(a.s) >= fabs(x)) a.c += (a.s - t) + x;
  else a.c += (x - t) + a.s;
  a.s = t;
}
__device__ __forceinline__ void neu_merge(Neu &a, const Neu &b) {
  neu_add(a, b.s);
  a.c += b.c;
}

// Sum of src[k * ncomp + comp] over k0 <= k < k1 by the whole workgroup (NT threads, a
// power of two): thread t takes k0 + t, k0 + t + NT, ..., then a fixed tree.  The result
// is returned to every thread.  ss/sc: NT doubles each of LDS.
template <int NT>
__device__ double block_neumaier(const double *__restrict__ src, int k0, int k1, int ncomp, int comp, double *ss,
                                 double *sc) {
  Neu a{0.0, 0.0};
  for (int k = k0 + (int)threadIdx.x; k < k1; k += NT) neu_add(a, src[(size_t)k * ncomp + comp]);
  __syncthreads();
  ss[threadIdx.x] = a.s;
  sc[threadIdx.x] = a.c;
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      Neu x{ss[threadIdx.x], sc[threadIdx.x]};
      neu_merge(x, Neu{ss[threadIdx.x + h], sc[threadIdx.x + h]});
      ss[threadIdx.x] = x.s;
      sc[threadIdx.x] = x.c;
    }
    __syncthreads();
  }
  const double r = ss[0] + sc[0];
  __syncthreads();
  return r;
}

}  // namespace
}  // namespace dp
