// Fused lattice-kinetic Poisson sweep for gfx950 (MI355X).
//
// One sweep (Sec. 3 and 4 of the paper): for every cell x
//   f_i(x)    = f*_i(x - v_i)                                   pull streaming
//   Phi(x)    = sum_i f_i(x)                                    moment, FP64 sum
//   f*_i'(x)  = (1 - omega) f_i(x) + omega phi_i Phi(x) + chi_i S(x)
// in a single pass: every population is read once and written once.
//
// Layout: Q planes of n cells, x fastest.  A wavefront owns 64 consecutive
// cells, so each of its loads for velocity i is one contiguous 64-element run
// of plane i shifted by v_i (coalesced; only the periodic seam wraps), and
// each store is an aligned contiguous run.  Plane bases are wave-uniform
// 64-bit pointers; per-lane offsets are 32-bit.
//
// Velocity groups: with P > 1 the four waves of a block split the Q
// velocities into P groups for the same 64-cell column, so each lane keeps
// only ~Q/P populations in registers between the moment and the collision;
// the partial moments meet in LDS.  P is chosen per (lattice, precision) by
// the runtime's tuner.
//
// Blocks are renumbered so that consecutive cell ranges land on the same XCD
// (the hardware deals workgroups round-robin over the 8 XCDs), keeping the
// seam cache lines shared by neighbouring blocks in one L2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "device_common.hpp"
#include "kernels.hpp"
#include "lattices.hpp"

namespace lkp {
namespace sweep_detail {

using namespace dev;

template <int M> struct ModeTraits;
template <> struct ModeTraits<MODE_F64> {
  using TIN = double; using TOUT = double; using TSRC = double; using TC = double;
  static constexpr bool POPSRC = false, RESID = false;
};
template <> struct ModeTraits<MODE_F32> {
  using TIN = float; using TOUT = float; using TSRC = float; using TC = float;
  static constexpr bool POPSRC = false, RESID = false;
};
template <> struct ModeTraits<MODE_RESID> {
  using TIN = double; using TOUT = float; using TSRC = double; using TC = double;
  static constexpr bool POPSRC = false, RESID = true;
};
template <> struct ModeTraits<MODE_INNER> {
  using TIN = float; using TOUT = float; using TSRC = float; using TC = float;
  static constexpr bool POPSRC = true, RESID = false;
};

// Every product and sum of the collision rounds on its own (no fused
// multiply-add), as the scheme is written: the kernel is bound by memory
// traffic, so this costs nothing, and decisions taken on FP64 values (a stop
// rule on max |dPhi|) see the same rounding as a plain evaluation.
#pragma clang fp contract(off)

template <int LID, int MODE, int P, int FLAGS>
__global__ void __launch_bounds__(256) k_sweep(SweepParams p) {
  using L = Lattice<LID>;
  using MT = ModeTraits<MODE>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  constexpr int Q = L::Q;
  constexpr int QG = (Q + P - 1) / P;
  constexpr int CELLS = 256 / P;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;

  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int g = wave % P;
  const int cw = wave / P;
  const unsigned blk = xcd_remap(blockIdx.x, p.nblocks);
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

  const size_t plane = p.ncells;
  const TIN *__restrict__ fin = reinterpret_cast<const TIN *>(p.fin);
  TOUT *__restrict__ fout = reinterpret_cast<TOUT *>(p.fout);
  const TSRC *__restrict__ src = reinterpret_cast<const TSRC *>(p.src);
  const TC *__restrict__ coef = reinterpret_cast<const TC *>(p.coef);

  TIN vals[QG];
  double part = 0.0;

  auto load_group = [&](auto Gc) {
    constexpr int G = decltype(Gc)::value;
    constexpr int lo = G * QG;
    constexpr int hi = (lo + QG < Q) ? lo + QG : Q;
    static_for<lo, hi>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int vx = L::table.v[i][0], vy = L::table.v[i][1], vz = L::table.v[i][2];
      const unsigned off = (zw[vz + VMZ] * p.ny + yw[vy + VMY]) * p.nx + xw[vx + VMX];
      vals[i - lo] = fin[(size_t)i * plane + off];
    });
    // moment in velocity order, FP64
    static_for<lo, hi>([&](auto I) { part += (double)vals[(int)I - lo]; });
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

  const TC phic = (TC)Phi;
  const TC om1 = (TC)p.om1;
  TC sc = 0;
  if constexpr (!MT::POPSRC) sc = (TC)src[cc];
  double r2 = 0.0;

  auto store_group = [&](auto Gc) {
    constexpr int G = decltype(Gc)::value;
    constexpr int lo = G * QG;
    constexpr int hi = (lo + QG < Q) ? lo + QG : Q;
    static_for<lo, hi>([&](auto I) {
      constexpr int i = decltype(I)::value;
      TC val;
      if constexpr (MT::POPSRC) {
        val = om1 * (TC)vals[i - lo] + coef[i] * phic + (TC)src[(size_t)i * plane + cc];
      } else {
        val = om1 * (TC)vals[i - lo] + coef[i] * phic + coef[Q + i] * sc;
      }
      if constexpr (MT::RESID) {
        const double r = (double)val - (double)fin[(size_t)i * plane + cc];
        r2 += r * r;
        if (valid) fout[(size_t)i * plane + c] = (TOUT)r;
      } else {
        if (valid) fout[(size_t)i * plane + c] = (TOUT)val;
      }
    });
  };
  if constexpr (P == 1) {
    store_group(std::integral_constant<int, 0>{});
  } else {
    static_for<0, P>([&](auto Gc) {
      if (g == (int)Gc) store_group(Gc);
    });
  }

  if constexpr ((FLAGS & (FLAG_PHI | FLAG_REDUCE)) != 0) {
    if (valid && g == 0) p.phi_out[c] = Phi;
  }
  if constexpr ((FLAGS & FLAG_REDUCE) != 0) {
    double v[NUM_NORMS] = {0, 0, 0, 0, 0, 0};
    if (valid) {
      if (g == 0) {
        const double prev = p.phi_prev ? p.phi_prev[c] : 0.0;
        const double d = Phi - prev;
        const bool ok = __builtin_isfinite(Phi) && __builtin_isfinite(d);
        v[NORM_MAX_DPHI] = ok ? fabs(d) : 0.0;
        v[NORM_SUM_DPHI2] = ok ? d * d : 0.0;
        v[NORM_SUM_PHI2] = ok ? Phi * Phi : 0.0;
        v[NORM_SUM_PHI] = ok ? Phi : 0.0;
        v[NORM_BAD] = ok ? 0.0 : 1.0;
      }
      if constexpr (MT::RESID) {
        const bool okr = __builtin_isfinite(r2);
        v[NORM_SUM_R2] = okr ? r2 : 0.0;
        v[NORM_BAD] += okr ? 0.0 : 1.0;
      }
    }
    block_norms(v, p.partials + (size_t)blk * NUM_NORMS);
  }
}

template <int LID, int MODE, int P>
hipError_t launch_flags(int flags, SweepParams p, hipStream_t s) {
  dim3 grid(p.nblocks), block(256);
  if (flags & FLAG_REDUCE)
    hipLaunchKernelGGL((k_sweep<LID, MODE, P, FLAG_REDUCE | FLAG_PHI>), grid, block, 0, s, p);
  else if constexpr (MODE != MODE_RESID) {
    if (flags & FLAG_PHI)
      hipLaunchKernelGGL((k_sweep<LID, MODE, P, FLAG_PHI>), grid, block, 0, s, p);
    else
      hipLaunchKernelGGL((k_sweep<LID, MODE, P, 0>), grid, block, 0, s, p);
  } else {
    return hipErrorInvalidValue;  // the residual sweep always reduces
  }
  return hipGetLastError();
}

template <int LID, int MODE>
hipError_t launch_mode(int P, int flags, SweepParams p, hipStream_t s) {
  switch (P) {
    case 1:
      if constexpr (sweep_variant_built(LID, MODE, 1)) return launch_flags<LID, MODE, 1>(flags, p, s);
      break;
    case 2:
      if constexpr (sweep_variant_built(LID, MODE, 2)) return launch_flags<LID, MODE, 2>(flags, p, s);
      break;
    case 4:
      if constexpr (sweep_variant_built(LID, MODE, 4)) return launch_flags<LID, MODE, 4>(flags, p, s);
      break;
  }
  return hipErrorInvalidValue;
}

template <int LID>
hipError_t launch_lattice(int mode, int P, int flags, SweepParams p, hipStream_t s) {
  switch (mode) {
    case MODE_F64: return launch_mode<LID, MODE_F64>(P, flags, p, s);
    case MODE_F32: return launch_mode<LID, MODE_F32>(P, flags, p, s);
    case MODE_RESID: return launch_mode<LID, MODE_RESID>(P, flags, p, s);
    case MODE_INNER: return launch_mode<LID, MODE_INNER>(P, flags, p, s);
  }
  return hipErrorInvalidValue;
}

}  // namespace sweep_detail

template <int LID>
hipError_t launch_lattice_tu(int mode, int P, int flags, SweepParams p, hipStream_t s) {
  return sweep_detail::launch_lattice<LID>(mode, P, flags, p, s);
}

}  // namespace lkp
