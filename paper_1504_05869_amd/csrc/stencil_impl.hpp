// The sweep at omega = 1 (tau_lb = 1) as a scalar stencil, for gfx950.
//
// With omega = 1 the collision forgets f_i: after any sweep the post-collision
// state is f*_i = phi_i Phi + chi_i S (Sec. 3 separable equilibrium and
// source), so the next sweep's moment is
//     Phi'(x) = sum_i phi_i Phi(x - v_i) + G(x),   G(x) = sum_i chi_i S(x - v_i)
// exactly.  The state shrinks from Q populations to one field, and one sweep
// moves 3 values per cell (read Phi, read G, write Phi') instead of 2Q + 1.
//
// Tiling: a 256-thread block owns TX x TY x TZ output cells and stages the
// tile plus its halo (the largest velocity component on each side, periodic
// wrap) in LDS.  Each thread computes CY cells along y; for every (dx, dz)
// offset pair it walks the needed LDS rows once and adds each value to every
// one of its CY outputs that uses it, so a staged value is read from LDS once
// per thread instead of once per output.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "lattices.hpp"

namespace lkp {
namespace stencil_detail {

using namespace dev;

template <int DIM> struct Tile;
template <> struct Tile<1> { static constexpr int TX = 256, TY = 1, TZ = 1, CY = 1; };
template <> struct Tile<2> { static constexpr int TX = 64, TY = 16, TZ = 1, CY = 4; };
template <> struct Tile<3> { static constexpr int TX = 32, TY = 8, TZ = 4, CY = 4; };

// index of velocity (vx, vy, vz) in the table, -1 if absent
constexpr int vel_index(const VelTable &t, int vx, int vy, int vz) {
  for (int i = 0; i < t.q; ++i)
    if (t.v[i][0] == vx && t.v[i][1] == vy && t.v[i][2] == vz) return i;
  return -1;
}

template <int SM> struct SModeTraits;
template <> struct SModeTraits<SMODE_F64> {
  using TIN = double; using TOUT = double; using TSRC = double; using TC = double;
  static constexpr bool RESID = false;
};
template <> struct SModeTraits<SMODE_F32> {
  using TIN = float; using TOUT = float; using TSRC = float; using TC = float;
  static constexpr bool RESID = false;
};
template <> struct SModeTraits<SMODE_RESID> {
  using TIN = double; using TOUT = float; using TSRC = double; using TC = double;
  static constexpr bool RESID = true;
};

#pragma clang fp contract(off)

template <int LID, int SM, int FLAGS>
__global__ void __launch_bounds__(256) k_stencil(StencilParams p) {
  using L = Lattice<LID>;
  using MT = SModeTraits<SM>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  using T = Tile<L::DIM>;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;
  constexpr int LX = T::TX + 2 * VMX, LY = T::TY + 2 * VMY, LZ = T::TZ + 2 * VMZ;
  constexpr int NL = LX * LY * LZ;
  constexpr int RY = T::TY / T::CY;  // thread rows in y
  __shared__ TIN tile[NL];

  const unsigned nx = p.nx, ny = p.ny, nz = p.nz;
  const int x0 = (int)(blockIdx.x * T::TX), y0 = (int)(blockIdx.y * T::TY),
            z0 = (int)(blockIdx.z * T::TZ);
  const bool simple = p.simple_wrap != 0;
  const TIN *__restrict__ xin = reinterpret_cast<const TIN *>(p.xin);

  // stage the tile and its periodic halo
  for (int e = threadIdx.x; e < NL; e += 256) {
    const int lx = e % LX, ly = (e / LX) % LY, lz = e / (LX * LY);
    const unsigned gx = wrap_coord(0u, -(x0 + lx - VMX), nx, simple && nx > (unsigned)(T::TX + VMX));
    const unsigned gy = wrap_coord(0u, -(y0 + ly - VMY), ny, simple && ny > (unsigned)(T::TY + VMY));
    const unsigned gz = wrap_coord(0u, -(z0 + lz - VMZ), nz, simple && nz > (unsigned)(T::TZ + VMZ));
    tile[e] = xin[((size_t)gz * ny + gy) * nx + gx];
  }
  __syncthreads();

  const int tx = threadIdx.x % T::TX;
  const int ty = (threadIdx.x / T::TX) % RY;
  const int tz = threadIdx.x / (T::TX * RY);
  const int ly0 = ty * T::CY;  // first output row of this thread (tile coordinates)
  TC acc[T::CY];
#pragma unroll
  for (int k = 0; k < T::CY; ++k) acc[k] = (TC)0;

  // acc[k] += phi(v) * Phi(x_k - v): x_k - v sits at tile (tx + VMX - vx,
  // ly0 + k + VMY - vy, tz + VMZ - vz); walk row r = k + VMY - vy once.
  static_for<-VMX, VMX + 1>([&](auto DX) {
    static_for<-VMZ, VMZ + 1>([&](auto DZ) {
      constexpr int vx = (int)DX, vz = (int)DZ;
      static_for<0, T::CY + 2 * VMY>([&](auto R) {
        constexpr int r = (int)R;
        constexpr bool used = [] {
          for (int k = 0; k < T::CY; ++k) {
            const int vy = k + VMY - r;
            if (vy >= -VMY && vy <= VMY && vel_index(L::table, vx, vy, vz) >= 0) return true;
          }
          return false;
        }();
        if constexpr (used) {
          const TC v = (TC)tile[((tz + VMZ - vz) * LY + (ly0 + r)) * LX + (tx + VMX - vx)];
          static_for<0, T::CY>([&](auto K) {
            constexpr int k = (int)K;
            constexpr int vy = k + VMY - r;
            if constexpr (vy >= -VMY && vy <= VMY) {
              constexpr int i = vel_index(L::table, vx, vy, vz);
              if constexpr (i >= 0) {
                constexpr int o = orbit_index(L::table, i);
                TC c;
                if constexpr (sizeof(TC) == 8) c = (TC)p.coef.d[o];
                else c = (TC)p.coef.f[o];
                acc[k] = acc[k] + c * v;
              }
            }
          });
        }
      });
      // Compiler-only fence (emits nothing): the accumulators pass through it
      // and it clobbers memory, so this column's arithmetic cannot sink below
      // it and the next column's LDS reads cannot rise above it.  Without it
      // the scheduler issues every LDS read of the stencil first and spills
      // the staged values to scratch.
#pragma unroll
      for (int k = 0; k < T::CY; ++k) asm volatile("" : "+v"(acc[k]) : : "memory");
    });
  });

  double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
  const TSRC *__restrict__ src = reinterpret_cast<const TSRC *>(p.src);
  TOUT *__restrict__ xout = reinterpret_cast<TOUT *>(p.xout);
  const int gx = x0 + tx, gz = z0 + tz;
#pragma unroll
  for (int k = 0; k < T::CY; ++k) {
    const int gy = y0 + ly0 + k;
    if (gx < (int)nx && gy < (int)ny && gz < (int)nz) {
      const size_t c = ((size_t)gz * ny + gy) * nx + gx;
      TC out = acc[k];
      if (src) out = out + (TC)src[c];
      const double centre = (double)tile[((tz + VMZ) * LY + (ly0 + k + VMY)) * LX + (tx + VMX)];
      if constexpr (MT::RESID) {
        const double r = (double)out - centre;  // R = A X + G - X
        xout[c] = (TOUT)r;
        if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
          const bool ok = __builtin_isfinite(r) && __builtin_isfinite((double)out);
          v[NORM_SUM_R2] += ok ? r * r : 0.0;
          v[NORM_SUM_PHI2] += ok ? (double)out * (double)out : 0.0;
          v[NORM_SUM_PHI] += ok ? (double)out : 0.0;
          v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(r)) : v[NORM_MAX_DPHI];
          v[NORM_SUM_DPHI2] += ok ? r * r : 0.0;
          v[NORM_BAD] += ok ? 0.0 : 1.0;
        }
      } else {
        xout[c] = (TOUT)out;
        if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
          const double o = (double)(TOUT)out;
          const double d = o - centre;
          const bool ok = __builtin_isfinite(o) && __builtin_isfinite(d);
          v[NORM_MAX_DPHI] = ok ? fmax(v[NORM_MAX_DPHI], fabs(d)) : v[NORM_MAX_DPHI];
          v[NORM_SUM_DPHI2] += ok ? d * d : 0.0;
          v[NORM_SUM_PHI2] += ok ? o * o : 0.0;
          v[NORM_SUM_PHI] += ok ? o : 0.0;
          v[NORM_BAD] += ok ? 0.0 : 1.0;
        }
      }
    }
  }
  if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
    const unsigned blk = (blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
    block_norms(v, p.partials + (size_t)blk * NUM_NORMS);
  }
}

template <int LID, int SM>
hipError_t launch_smode(int flags, const StencilParams &p, hipStream_t s) {
  using T = Tile<Lattice<LID>::DIM>;
  dim3 grid((p.nx + T::TX - 1) / T::TX, (p.ny + T::TY - 1) / T::TY, (p.nz + T::TZ - 1) / T::TZ);
  if (flags & FLAG_REDUCE)
    hipLaunchKernelGGL((k_stencil<LID, SM, FLAG_REDUCE>), grid, dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_stencil<LID, SM, 0>), grid, dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace stencil_detail

template <int LID>
hipError_t launch_stencil_tu(int smode, int flags, const StencilParams &p, hipStream_t s) {
  switch (smode) {
    case SMODE_F64: return stencil_detail::launch_smode<LID, SMODE_F64>(flags, p, s);
    case SMODE_F32: return stencil_detail::launch_smode<LID, SMODE_F32>(flags, p, s);
    case SMODE_RESID: return stencil_detail::launch_smode<LID, SMODE_RESID>(flags, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace lkp
