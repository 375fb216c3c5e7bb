// Fused lattice-kinetic Poisson sweep for gfx950 (MI355X).
//
// One sweep (Sec. 4 and 5 of the paper): for every cell x
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
// the runtime's tuner.  The moment is always summed in the same order, so
// every P gives the same bits: four fixed runs of ceil(Q/4) consecutive
// velocities are summed in velocity order, then combined as
// (s0 + s1) + (s2 + s3); a group of P = 2 holds two runs, P = 4 one.  Sets of
// at most 25 velocities (built for P = 1 only) sum in plain velocity order.
//
// Blocks are renumbered so that runs of 16 consecutive blocks land on one XCD
// (the hardware deals workgroups round-robin over the 8 XCDs): neighbouring
// blocks of a run share their seam cache lines in one L2, while the chip as a
// whole still streams one compact window of every plane.  Measured against
// handing each XCD one contiguous eighth of the grid, this is 2-3 % faster.
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

// Cache policy of the streamed population planes: every value is read once
// and written once per sweep, so the stores may skip cache allocation.
#ifndef LKP_NT_STORE
#define LKP_NT_STORE 1
#endif
#ifndef LKP_NT_LOAD
#define LKP_NT_LOAD 0
#endif
// Block order: -1 = each XCD takes one contiguous eighth of the grid,
// 0 = hardware order, R > 0 = runs of R blocks per XCD (xcd_runs).
#ifndef LKP_XCD_REMAP
#define LKP_XCD_REMAP 16
#endif

template <typename T>
__device__ __forceinline__ T ld(const char *base, unsigned byte_off) {
  const T *p = reinterpret_cast<const T *>(base + byte_off);
#if LKP_NT_LOAD
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

template <typename T>
__device__ __forceinline__ void st(char *base, unsigned byte_off, T v) {
  T *p = reinterpret_cast<T *>(base + byte_off);
#if LKP_NT_STORE
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

// Every product and sum of the collision rounds on its own (no fused
// multiply-add), as the scheme is written: the kernel is bound by memory
// traffic, so this costs nothing, and decisions taken on FP64 values (a stop
// rule on max |dPhi|) see the same rounding as a plain evaluation.
#pragma clang fp contract(off)

// Coefficients of one problem: omega phi_i and chi_i in the compute precision.
template <typename TC>
struct CoefTable {  // precomputed on the host (single-problem launches)
  const TC *c;
  int q;
  __device__ __forceinline__ TC wphi(int i) const { return c[i]; }
  __device__ __forceinline__ TC chi(int i) const { return c[q + i]; }
};

template <typename TC>
struct CoefScaled {  // batched launches: omega phi_i formed in FP64 exactly as the host does
  double omega;
  const double *phi;
  const double *chi_;
  __device__ __forceinline__ TC wphi(int i) const { return (TC)(omega * phi[i]); }
  __device__ __forceinline__ TC chi(int i) const { return (TC)chi_[i]; }
};

// One block's share of a sweep: cells [blk * CELLS, blk * CELLS + CELLS) of
// the problem described by p (SweepParams or BatchMember).
//
// AA selects the storage of the input state (in-place single-buffer sweeps
// alternate between two layouts; the values computed are those of the pull
// sweep, in the same order):
//   AA = 0  pull layout, two buffers: f*_i(y) at plane i, cell y.
//   AA = 1  swapped layout: f*_i(y) at plane opp(i), cell y.  The sweep reads
//           f*_i(x - v_i) there and writes f*'_i(x) to plane i, cell x + v_i.
//   AA = 2  pushed layout: f*_i(y) at plane i, cell y + v_i.  The sweep reads
//           f*_i(x - v_i) at plane i, cell x, and writes f*'_i(x) to plane
//           opp(i), cell x: the swapped layout again.
// Every location an AA sweep writes is read by the same cell in the same
// sweep (and by nothing else), before the block's barrier, so the update is
// safe in place.
template <int LID, int MODE, int P, int FLAGS, int AA, class Params, class C>
__device__ __forceinline__ void sweep_block(const Params &p, unsigned blk, const C &coef) {
  using L = Lattice<LID>;
  using MT = ModeTraits<MODE>;
  using TIN = typename MT::TIN;
  using TOUT = typename MT::TOUT;
  using TSRC = typename MT::TSRC;
  using TC = typename MT::TC;
  constexpr int Q = L::Q;
  constexpr int NRUNS = Q <= 25 ? 1 : 4;  // summation runs (small sets: one, in velocity order)
  static_assert(NRUNS % P == 0, "a velocity group holds whole summation runs");
  constexpr int QS = (Q + NRUNS - 1) / NRUNS;  // velocities of one run
  constexpr int RUNS = NRUNS / P;      // runs per velocity group
  constexpr int QG = QS * RUNS;        // velocities of a group (the last may hold fewer)
  constexpr int CELLS = 256 / P;
  constexpr int VMX = L::VMX, VMY = L::VMY, VMZ = L::VMZ;

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

  // Plane i starts at a wave-uniform base; lanes add a 32-bit byte offset
  // (every plane is < 4 GiB), which maps to scalar-base + vector-offset
  // addressing.
  const size_t plane = p.plane;
  // in place (AA > 0) the two point to the same buffer: no restrict
  const char *fin = reinterpret_cast<const char *>(p.fin);
  char *fout = reinterpret_cast<char *>(p.fout);
  const char *__restrict__ src = reinterpret_cast<const char *>(p.src);
  const unsigned c_in = cc * (unsigned)sizeof(TIN);
  const unsigned c_out = c * (unsigned)sizeof(TOUT);

  TIN vals[QG];
  double part = 0.0;

  auto load_group = [&](auto Gc) {
    constexpr int G = decltype(Gc)::value;
    constexpr int lo = G * QG;
    constexpr int hi = (lo + QG < Q) ? lo + QG : Q;
    static_for<lo, hi>([&](auto I) {
      constexpr int i = decltype(I)::value;
      constexpr int vx = L::table.v[i][0], vy = L::table.v[i][1], vz = L::table.v[i][2];
      static_assert(L::vel(-vx, -vy, -vz) >= 0, "in-place layouts need a symmetric velocity set");
      constexpr int li = AA == 1 ? L::vel(-vx, -vy, -vz) : i;  // plane holding f*_i
      const unsigned off = AA == 2 ? cc : (zw[vz + VMZ] * p.ny + yw[vy + VMY]) * p.nx + xw[vx + VMX];
      vals[i - lo] = ld<TIN>(fin + (size_t)li * plane * sizeof(TIN), off * (unsigned)sizeof(TIN));
    });
    // moment, FP64: each run in velocity order, runs combined pairwise
    double run[RUNS];
    static_for<0, RUNS>([&](auto Rc) {
      constexpr int R = decltype(Rc)::value;
      constexpr int rlo = lo + R * QS < Q ? lo + R * QS : Q;
      constexpr int rhi = rlo + QS < Q ? rlo + QS : Q;
      run[R] = 0.0;
      static_for<rlo, rhi>([&](auto I) { run[R] += (double)vals[(int)I - lo]; });
    });
    if constexpr (RUNS == 4) part = (run[0] + run[1]) + (run[2] + run[3]);
    else if constexpr (RUNS == 2) part = run[0] + run[1];
    else part = run[0];
    if constexpr (MT::POPSRC) {
      // correction sweeps: fold the population source in now, (1 - omega) f_i
      // + r_i, so that the r_i loads overlap the pulled loads instead of
      // waiting one by one after the moment
      const TC om1 = (TC)p.om1;
      static_for<lo, hi>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const TSRC ri = ld<TSRC>(src + (size_t)i * plane * sizeof(TSRC), cc * (unsigned)sizeof(TSRC));
        vals[i - lo] = (TIN)(om1 * (TC)vals[i - lo] + (TC)ri);
      });
    }
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
    if constexpr (P == 4) Phi = (sh[0][ci] + sh[1][ci]) + (sh[2][ci] + sh[3][ci]);
    else Phi = sh[0][ci] + sh[1][ci];
  }

  const TC phic = (TC)Phi;
  const TC om1 = (TC)p.om1;
  TC sc = 0;
  if constexpr (!MT::POPSRC) sc = (TC)ld<TSRC>(src, cc * (unsigned)sizeof(TSRC));
  double r2 = 0.0;

  if constexpr (AA == 1 || (AA == 2 && MT::RESID)) {
    // In-place stores (and the pushed reads of the residual) reuse the pull
    // offsets of the opposite velocities; left alone the compiler keeps all Q
    // of them live from the loads, doubling the registers.  An empty asm
    // makes the wrapped coordinates opaque, so the offsets are recomputed.
#pragma unroll
    for (int j = 0; j < 2 * VMX + 1; ++j) asm volatile("" : "+v"(xw[j]));
#pragma unroll
    for (int j = 0; j < 2 * VMY + 1; ++j) asm volatile("" : "+v"(yw[j]));
#pragma unroll
    for (int j = 0; j < 2 * VMZ + 1; ++j) asm volatile("" : "+v"(zw[j]));
  }

  auto store_group = [&](auto Gc) {
    constexpr int G = decltype(Gc)::value;
    constexpr int lo = G * QG;
    constexpr int hi = (lo + QG < Q) ? lo + QG : Q;
    static_for<lo, hi>([&](auto I) {
      constexpr int i = decltype(I)::value;
      TC val;
      if constexpr (MT::POPSRC) {
        val = (TC)vals[i - lo] + coef.wphi(i) * phic;  // vals holds (1 - omega) f_i + r_i
      } else {
        val = om1 * (TC)vals[i - lo] + coef.wphi(i) * phic + coef.chi(i) * sc;
      }
      constexpr int vx = L::table.v[i][0], vy = L::table.v[i][1], vz = L::table.v[i][2];
      constexpr int oi = L::vel(-vx, -vy, -vz);
      if constexpr (MT::RESID) {
        // own f*_i(x) in the input layout; r is written in the pull layout
        double xi;
        if constexpr (AA == 2) {
          const unsigned pushed =
              (zw[VMZ - vz] * p.ny + yw[VMY - vy]) * p.nx + xw[VMX - vx];  // x + v_i
          xi = (double)ld<TIN>(fin + (size_t)i * plane * sizeof(TIN), pushed * (unsigned)sizeof(TIN));
        } else {
          xi = (double)ld<TIN>(fin + (size_t)(AA == 1 ? oi : i) * plane * sizeof(TIN), c_in);
        }
        const double r = (double)val - xi;
        r2 += r * r;
        if (valid && fout) st<TOUT>(fout + (size_t)i * plane * sizeof(TOUT), c_out, (TOUT)r);
      } else if constexpr (AA == 1) {
        const unsigned pushed = (zw[VMZ - vz] * p.ny + yw[VMY - vy]) * p.nx + xw[VMX - vx];
        if (valid && fout)
          st<TOUT>(fout + (size_t)i * plane * sizeof(TOUT), pushed * (unsigned)sizeof(TOUT), (TOUT)val);
      } else {
        char *obase = fout + (size_t)(AA == 2 ? oi : i) * plane * sizeof(TOUT);
        if (valid && fout) st<TOUT>(obase, c_out, (TOUT)val);  // no fout: norms only
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

__device__ __forceinline__ unsigned block_order(unsigned b, unsigned nb) {
#if LKP_XCD_REMAP < 0
  return xcd_remap(b, nb);
#elif LKP_XCD_REMAP == 0
  (void)nb;
  return b;
#else
  return xcd_runs(b, nb, LKP_XCD_REMAP);
#endif
}

template <int LID, int MODE, int P, int FLAGS, int AA>
__global__ void __launch_bounds__(256) k_sweep(SweepParams p) {
  using TC = typename ModeTraits<MODE>::TC;
  const unsigned blk = block_order(blockIdx.x, p.nblocks);
  CoefTable<TC> coef;
  if constexpr (sizeof(TC) == 8) coef.c = p.coef.d;
  else coef.c = p.coef.f;
  coef.q = Lattice<LID>::Q;
  sweep_block<LID, MODE, P, FLAGS, AA>(p, blk, coef);
}

// Many problems of one lattice class in one launch: blocks are numbered
// member after member; each block finds its member in the (wave-uniform)
// table and sweeps its cells exactly as a single-problem launch would.
template <int LID, int MODE, int P, int FLAGS>
__global__ void __launch_bounds__(256) k_sweep_batch(BatchParams<Lattice<LID>::Q> bp) {
  using TC = typename ModeTraits<MODE>::TC;
  const unsigned gb = block_order(blockIdx.x, bp.nblocks);
  unsigned j = 0;
  for (unsigned k = 1; k < bp.nmembers; ++k)
    if (bp.m[k].block_begin <= gb) j = k;
  const BatchMember &m = bp.m[j];
  CoefScaled<TC> coef{m.omega, bp.phi, bp.chi};
  sweep_block<LID, MODE, P, FLAGS, 0>(m, gb - m.block_begin, coef);
}



template <int LID, int MODE, int P, int AA>
hipError_t launch_flags(int flags, SweepParams p, hipStream_t s) {
  dim3 grid(p.nblocks), block(256);
  if (flags & FLAG_REDUCE)
    hipLaunchKernelGGL((k_sweep<LID, MODE, P, FLAG_REDUCE | FLAG_PHI, AA>), grid, block, 0, s, p);
  else if constexpr (MODE != MODE_RESID) {
    if (flags & FLAG_PHI)
      hipLaunchKernelGGL((k_sweep<LID, MODE, P, FLAG_PHI, AA>), grid, block, 0, s, p);
    else
      hipLaunchKernelGGL((k_sweep<LID, MODE, P, 0, AA>), grid, block, 0, s, p);
  } else {
    return hipErrorInvalidValue;  // the residual sweep always reduces
  }
  return hipGetLastError();
}

template <int LID, int MODE, int P>
hipError_t launch_aa(int aa, int flags, SweepParams p, hipStream_t s) {
  switch (aa) {
    case 0: return launch_flags<LID, MODE, P, 0>(flags, p, s);
    case 1: return launch_flags<LID, MODE, P, 1>(flags, p, s);
    case 2: return launch_flags<LID, MODE, P, 2>(flags, p, s);
  }
  return hipErrorInvalidValue;
}

template <int LID, int MODE, int P>
hipError_t launch_batch_flags(int flags, const BatchParams<Lattice<LID>::Q> &bp, hipStream_t s) {
  dim3 grid(bp.nblocks), block(256);
  if constexpr (MODE == MODE_RESID) {
    return hipErrorInvalidValue;  // residual sweeps are launched one problem at a time
  } else {
    if (flags & FLAG_REDUCE)
      hipLaunchKernelGGL((k_sweep_batch<LID, MODE, P, FLAG_REDUCE | FLAG_PHI>), grid, block, 0, s, bp);
    else if (flags & FLAG_PHI)
      hipLaunchKernelGGL((k_sweep_batch<LID, MODE, P, FLAG_PHI>), grid, block, 0, s, bp);
    else
      hipLaunchKernelGGL((k_sweep_batch<LID, MODE, P, 0>), grid, block, 0, s, bp);
  }
  return hipGetLastError();
}

template <int LID, int MODE>
hipError_t launch_batch_mode(int P, int flags, const void *bp, hipStream_t s) {
  const auto &b = *reinterpret_cast<const BatchParams<Lattice<LID>::Q> *>(bp);
  switch (P) {
    case 1:
      if constexpr (sweep_variant_built(LID, MODE, 1)) return launch_batch_flags<LID, MODE, 1>(flags, b, s);
      break;
    case 2:
      if constexpr (sweep_variant_built(LID, MODE, 2)) return launch_batch_flags<LID, MODE, 2>(flags, b, s);
      break;
    case 4:
      if constexpr (sweep_variant_built(LID, MODE, 4)) return launch_batch_flags<LID, MODE, 4>(flags, b, s);
      break;
  }
  return hipErrorInvalidValue;
}

template <int LID, int MODE>
hipError_t launch_mode(int P, int aa, int flags, SweepParams p, hipStream_t s) {
  switch (P) {
    case 1:
      if constexpr (sweep_variant_built(LID, MODE, 1)) return launch_aa<LID, MODE, 1>(aa, flags, p, s);
      break;
    case 2:
      if constexpr (sweep_variant_built(LID, MODE, 2)) return launch_aa<LID, MODE, 2>(aa, flags, p, s);
      break;
    case 4:
      if constexpr (sweep_variant_built(LID, MODE, 4)) return launch_aa<LID, MODE, 4>(aa, flags, p, s);
      break;
  }
  return hipErrorInvalidValue;
}

}  // namespace sweep_detail

// Entry points of one (lattice, mode): each is compiled in a translation unit
// of its own, so the large sets build in parallel.
template <int LID, int MODE>
hipError_t launch_mode_tu(int P, int aa, int flags, SweepParams p, hipStream_t s) {
  return sweep_detail::launch_mode<LID, MODE>(P, aa, flags, p, s);
}

template <int LID, int MODE>
hipError_t launch_batch_mode_tu(int P, int flags, const void *bp, hipStream_t s) {
  return sweep_detail::launch_batch_mode<LID, MODE>(P, flags, bp, s);
}

template <int LID>
hipError_t launch_lattice_tu(int mode, int P, int aa, int flags, SweepParams p, hipStream_t s) {
  switch (mode) {
    case MODE_F64: return launch_mode_tu<LID, MODE_F64>(P, aa, flags, p, s);
    case MODE_F32: return launch_mode_tu<LID, MODE_F32>(P, aa, flags, p, s);
    case MODE_RESID: return launch_mode_tu<LID, MODE_RESID>(P, aa, flags, p, s);
    case MODE_INNER: return launch_mode_tu<LID, MODE_INNER>(P, aa, flags, p, s);
  }
  return hipErrorInvalidValue;
}

template <int LID>
hipError_t launch_batch_tu(int mode, int P, int flags, const void *bp, hipStream_t s) {
  switch (mode) {
    case MODE_F64: return launch_batch_mode_tu<LID, MODE_F64>(P, flags, bp, s);
    case MODE_F32: return launch_batch_mode_tu<LID, MODE_F32>(P, flags, bp, s);
    case MODE_INNER: return launch_batch_mode_tu<LID, MODE_INNER>(P, flags, bp, s);
  }
  return hipErrorInvalidValue;  // residual sweeps are launched one problem at a time
}

}  // namespace lkp
