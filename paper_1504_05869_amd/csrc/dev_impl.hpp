// Lattice-kinetic sweep with BF16 deviation storage, for gfx950.
//
// The scheme is the fused sweep of Sec. 4 and 5 (pull streaming, moment,
// relaxation toward phi_i Phi plus the source term); only the storage of the
// post-collision state differs.  Per cell x:
//   f_i(x)   = phi_i Phi(x - v_i) + n_i(x - v_i)        rebuild the streamed f
//   Phi'(x)  = sum_i f_i(x)                              FP64 sum, stored FP32
//   n'_i(x)  = (1 - omega) (f_i(x) - phi_i Phi'(x)) + s_i(x)
// which is f*'_i - phi_i Phi' for f*'_i = (1 - omega) f_i + omega phi_i Phi'
// + s_i, with s_i = chi_i S(x) (solve) or r_i(x) (correction solve of the
// iterative refinement).  n' is rounded to BF16 (nearest, ties to even).
//
// Layout and work split follow the population sweep: Q planes of n cells, x
// fastest; a wave owns 64 consecutive cells; P waves of a block share a
// column, each with Q/P velocities, and their partial moments meet in LDS.
// The upstream Phi values are read with the same shifted offsets as the
// deviation planes; neighbouring waves read the same Phi lines, which stay in
// L2, so HBM sees Phi about once per sweep.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "dev_kernels.hpp"
#include "device_common.hpp"
#include "kernels.hpp"
#include "lattices.hpp"

namespace lkp {
namespace dev_detail {

using namespace dev;

#pragma clang fp contract(off)

__device__ __forceinline__ float bf16_to_f32(uint16_t b) { return __uint_as_float((unsigned)b << 16); }

// FP32 -> BF16, round to nearest with ties to even (add 0x7fff plus the lowest
// kept bit, truncate); NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  const unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}

template <int LID, bool INNER, int P, int FLAGS>
__global__ void __launch_bounds__(256) k_sweep_dev(DevParams p) {
  using L = Lattice<LID>;
  constexpr int Q = L::Q;
  constexpr int QG = (Q + P - 1) / P;
  constexpr int CELLS = 256 / P;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;

  const unsigned blk = xcd_runs(blockIdx.x, p.nblocks, 16u);
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = wave % P;
  const int cw = wave / P;
  const unsigned ci = (unsigned)(cw * 64 + lane);
  const unsigned c = blk * CELLS + ci;
  const bool valid = c < p.ncells;
  const unsigned cc = valid ? c : p.ncells - 1;  // keep every lane's loads in bounds

  const unsigned x = cc % p.nx;
  const unsigned rr = cc / p.nx;
  const unsigned y = rr % p.ny;
  const unsigned z = rr / p.ny;
  const bool simple = p.simple_wrap != 0;
  unsigned xw[2 * VMX + 1], yw[2 * VMY + 1], zw[2 * VMZ + 1];
  static_for<0, 2 * VMX + 1>([&](auto J) { xw[J] = wrap_coord(x, (int)J - VMX, p.nx, simple); });
  static_for<0, 2 * VMY + 1>([&](auto J) { yw[J] = wrap_coord(y, (int)J - VMY, p.ny, simple); });
  static_for<0, 2 * VMZ + 1>([&](auto J) { zw[J] = wrap_coord(z, (int)J - VMZ, p.nz, simple); });
  const size_t plane = p.plane;

  float f[QG];
  // correction sweeps: the population source r_i, loaded with the pulled
  // values so that its loads overlap theirs instead of waiting one by one
  // after the moment (used unchanged in the store phase)
  float rs[INNER ? QG : 1];
  double part = 0.0;
  auto load_group = [&](auto Gc) {
    constexpr int G = decltype(Gc)::value;
    constexpr int lo = G * QG;
    constexpr int hi = (lo + QG < Q) ? lo + QG : Q;
    static_for<lo, hi>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int vx = L::table.v[i][0], vy = L::table.v[i][1], vz = L::table.v[i][2];
      const unsigned off = (zw[vz + VMZ] * p.ny + yw[vy + VMY]) * p.nx + xw[vx + VMX];
      const float nb = bf16_to_f32(p.nin[(size_t)i * plane + off]);
      f[i - lo] = p.phi[i] * p.phin[off] + nb;
      if constexpr (INNER) rs[i - lo] = p.src[(size_t)i * plane + cc];
    });
    static_for<lo, hi>([&](auto I) { part += (double)f[(int)I - lo]; });
  };
  if constexpr (P == 1) {
    load_group(std::integral_constant<int, 0>{});
  } else {
    static_for<0, P>([&](auto Gc) {
      if (g == (int)Gc) load_group(Gc);
    });
  }

  double Phi;
  if constexpr (P == 1) {
    Phi = part;
  } else {
    __shared__ double sh[P][CELLS];
    sh[g][ci] = part;
    __syncthreads();
    Phi = sh[0][ci];
#pragma unroll
    for (int k = 1; k < P; ++k) Phi += sh[k][ci];
  }
  const float Ph = (float)Phi;  // the stored moment; deviations are taken from it
  float S = 0.0f;
  if constexpr (!INNER) S = p.src[cc];

  auto store_group = [&](auto Gc) {
    constexpr int G = decltype(Gc)::value;
    constexpr int lo = G * QG;
    constexpr int hi = (lo + QG < Q) ? lo + QG : Q;
    static_for<lo, hi>([&](auto I) {
      constexpr int i = decltype(I)::value;
      float s;
      if constexpr (INNER) s = rs[i - lo];
      else s = p.chi[i] * S;
      const float nn = p.om1 * (f[i - lo] - p.phi[i] * Ph) + s;
      if (valid) p.nout[(size_t)i * plane + c] = f32_to_bf16(nn);
    });
  };
  if constexpr (P == 1) {
    store_group(std::integral_constant<int, 0>{});
  } else {
    static_for<0, P>([&](auto Gc) {
      if (g == (int)Gc) store_group(Gc);
    });
  }
  if (valid && g == 0) p.phout[c] = Ph;

  if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
    double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
    if (valid && g == 0) {
      const double o = (double)Ph;
      const double d = o - (double)p.phin[c];
      const bool ok = __builtin_isfinite(o) && __builtin_isfinite(d);
      v[NORM_MAX_DPHI] = ok ? fabs(d) : 0.0;
      v[NORM_SUM_DPHI2] = ok ? d * d : 0.0;
      v[NORM_SUM_PHI2] = ok ? o * o : 0.0;
      v[NORM_SUM_PHI] = ok ? o : 0.0;
      v[NORM_BAD] = ok ? 0.0 : 1.0;
    }
    block_norms(v, p.partials + (size_t)blk * NUM_NORMS);
  }
}

template <int LID, bool INNER>
hipError_t launch_inner(int flags, const DevParams &p, hipStream_t s) {
  constexpr int P = dev_split(LID);
  if (flags & FLAG_REDUCE)
    hipLaunchKernelGGL((k_sweep_dev<LID, INNER, P, FLAG_REDUCE>), dim3(p.nblocks), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_sweep_dev<LID, INNER, P, 0>), dim3(p.nblocks), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace dev_detail

template <int LID>
hipError_t launch_dev_tu(bool inner, int flags, DevParams p, hipStream_t s) {
  p.nblocks = dev_blocks(LID, p.ncells);
  return inner ? dev_detail::launch_inner<LID, true>(flags, p, s)
               : dev_detail::launch_inner<LID, false>(flags, p, s);
}

}  // namespace lkp
