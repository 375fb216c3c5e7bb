// Device helpers shared by the sweep kernels and the small utility kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "kernels.hpp"

namespace lkp {
namespace dev {

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7u;
  const unsigned xcd = b & 7u, k = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// (x - d) mod n for |d| <= VM.  simple: n >= VM, one correction suffices.
__device__ __forceinline__ unsigned wrap_coord(unsigned x, int d, unsigned n, bool simple) {
  int t = (int)x - d;
  if (simple) {
    t += (t < 0) ? (int)n : 0;
    t -= (t >= (int)n) ? (int)n : 0;
    return (unsigned)t;
  }
  t %= (int)n;
  return (unsigned)(t < 0 ? t + (int)n : t);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// Reduce NUM_NORMS values over the 256-thread block in a fixed order;
// thread 0 writes them to dst.
__device__ __forceinline__ void block_norms(double (&v)[NUM_NORMS], double *dst) {
  __shared__ double red[4][NUM_NORMS];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NUM_NORMS; ++k) v[k] = (k == NORM_MAX_DPHI) ? wave_max(v[k]) : wave_sum(v[k]);
  if (lane == 0)
#pragma unroll
    for (int k = 0; k < NUM_NORMS; ++k) red[wave][k] = v[k];
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NUM_NORMS; ++k) {
      double a = red[0][k];
      for (int w = 1; w < 4; ++w) a = (k == NORM_MAX_DPHI) ? fmax(a, red[w][k]) : a + red[w][k];
      dst[k] = a;
    }
  }
}

}  // namespace dev
}  // namespace lkp
