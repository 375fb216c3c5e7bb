// Device helpers shared by the sweep kernels and the small utility kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>
#include <utility>

#include "kernels.hpp"

namespace lkp {
namespace dev {

// f(integral_constant<B>), ..., f(integral_constant<E - 1>) as one fold
// expression (no recursion: one instantiation per call site).
template <int B, class F, int... I>
__device__ __forceinline__ void static_for_seq(F &&f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, B + I>{}), ...);
}

template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) static_for_seq<B>(f, std::make_integer_sequence<int, E - B>{});
}

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7u;
  const unsigned xcd = b & 7u, k = b >> 3;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

// Runs of R consecutive blocks per XCD with the 8 XCDs on adjacent runs:
// block b = 8 k + xcd (dealt round-robin) becomes ((k / R) * 8 + xcd) * R +
// k % R.  The chip as a whole still walks one compact window of the grid,
// while neighbouring blocks inside a run share their XCD's L2.  Blocks past
// the last whole group of 8 R keep their number.
__device__ __forceinline__ unsigned xcd_runs(unsigned b, unsigned nb, unsigned R) {
  const unsigned full = nb / (8u * R) * (8u * R);
  if (b >= full) return b;
  const unsigned xcd = b & 7u, k = b >> 3;
  return ((k / R) * 8u + xcd) * R + k % R;
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
